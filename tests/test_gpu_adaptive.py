"""Per-Jacobian perturbation size: the power-iteration estimate of rho(A^{-1} D) against
LAPACK's eigenvalues and the oracle's iteration, and psp_solve_adaptive (the error test
from the perturbed solutions and the rescaled second solve) bitwise equal to the oracle's
adaptive_batch in every output, on the benchmark scenarios (whose rho spans four decades),
small batches, both tolerance extremes, a Gaussian D, and a captured HIP graph."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HARD = [236, 450, 312, 507, 467, 223, 0, 1]   # largest rho(A^-1) among the 512 benchmark scenarios, and two typical


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch(W):
    ip, ix, vals, bs = W.scenario_batch(300, 512)
    return ip, ix, vals[HARD].copy(), bs[HARD].copy()


def test_rho_estimate_matches_eigenvalues(dev, W, batch):
    from paper_2311_11833_amd import psp
    from paper_2311_11833_amd.adaptive import estimate_rho
    ip, ix, vals, bs = batch
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    print("[gpu adaptive] rho estimate", flush=True)
    rho = estimate_rho(plan, torch.from_numpy(vals).to(dev))
    for s in range(len(HARD)):
        ref = 1.0 / np.abs(np.linalg.eigvals(W.to_dense(n, ip, ix, vals[s]))).min()
        assert 0.5 < rho[s] / ref < 2.0, (HARD[s], rho[s], ref)


@pytest.mark.parametrize("gaussian_d", [False, True])
def test_rho_iteration_matches_oracle(dev, O, W, batch, gaussian_d):
    """psp_estimate_rho runs the oracle's pivot-free power iteration: the same start
    vectors, the same perturbed solves (bitwise), the same ascending fma norms and IEEE
    divisions, so every iterate is identical and only log/exp may differ in the last bits."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = batch
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    d = None
    if gaussian_d:
        d = np.random.default_rng(1311).standard_normal(n)
        d /= np.abs(d).max()
    v0 = np.random.default_rng(9).standard_normal((len(HARD), n))
    sym = O.symbolic(n, ip, ix)
    print(f"[gpu adaptive] rho iteration vs oracle, gaussian d {gaussian_d}", flush=True)
    for probe, iters in ((1e-8, 24), (1e-6, 7)):
        rho = psp.estimate_rho(plan, torch.from_numpy(vals).to(dev), torch.from_numpy(v0).to(dev),
                               d=None if d is None else torch.from_numpy(d).to(dev), probe=probe,
                               iters=iters).cpu().numpy()
        for s in range(len(HARD)):
            ref = O.power_rho_pivot_free(n, ip, ix, vals[s], sym, d, probe, v0[s], iters)
            assert abs(rho[s] - ref) <= 1e-13 * ref, (HARD[s], probe, rho[s], ref)
    one = psp.estimate_rho(plan, torch.from_numpy(vals[:1]).to(dev), torch.from_numpy(v0[:1]).to(dev), iters=1)
    ref = O.power_rho_pivot_free(n, ip, ix, vals[0], sym, None, 1e-8, v0[0], 1)
    assert abs(float(one[0]) - ref) <= 1e-13 * ref
    with pytest.raises(psp.PSPError):
        psp.estimate_rho(plan, torch.from_numpy(vals).to(dev), torch.from_numpy(v0).to(dev), probe=0.0)
    with pytest.raises(psp.PSPError):
        psp.estimate_rho(plan, torch.from_numpy(vals).to(dev), torch.from_numpy(v0).to(dev), iters=0)


def _check_adaptive(O, ip, ix, vals, bs, eps, tol, out, d=None):
    n = len(ip) - 1
    sym = O.symbolic(n, ip, ix)
    xo, io, eo, so = O.adaptive_batch(n, ip, ix, vals, sym, eps, bs, tol, d=d)
    x, info, est, scale = (t.cpu().numpy() for t in out)
    assert np.array_equal(scale, so)
    assert np.array_equal(info, io)
    assert np.array_equal(est, eo, equal_nan=True)
    assert np.array_equal(x, xo, equal_nan=True)
    return so


def test_error_test_rescale_full_batch_matches_oracle(dev, O, W):
    """512 Jacobians of the 300-bus network: the first solve runs one workgroup per Jacobian
    (perturbed solutions kept for the error test), the rescaled ones run per system."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(300, 512)
    plan = psp.Plan(ip, ix)
    eps = W.config_eps("n601")
    print("[gpu adaptive] error test + rescale, 512 x K=5", flush=True)
    out = psp.solve_adaptive(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), tol=1e-10)
    torch.cuda.synchronize()
    so = _check_adaptive(O, ip, ix, vals, bs, eps, 1e-10, out)
    assert 50 <= int((so != 1.0).sum()) <= 150


def test_error_test_rescale_small_batch_matches_oracle(dev, O, W, batch):
    """The hard scenarios alone: the first solve runs one workgroup per perturbed system."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = batch
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    eps = W.config_eps("n601")
    print("[gpu adaptive] error test + rescale, hard scenarios", flush=True)
    out = psp.solve_adaptive(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), tol=1e-10)
    torch.cuda.synchronize()
    so = _check_adaptive(O, ip, ix, vals, bs, eps, 1e-10, out)
    assert int((so != 1.0).sum()) >= 6
    x = out[0].cpu().numpy()
    for s in range(len(HARD)):
        xs = np.linalg.solve(W.to_dense(n, ip, ix, vals[s]), bs[s])
        assert np.abs(x[s] - xs).max() / np.abs(xs).max() < 1e-9, HARD[s]


@pytest.mark.parametrize("tol", [0.0, 1e300])
def test_error_test_tolerance_extremes(dev, O, W, tol):
    """tol = 0 sends every Jacobian to the second solve, a huge tol none (the first solve is kept)."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(300, 40)
    plan = psp.Plan(ip, ix)
    eps = W.config_eps("n601")
    print(f"[gpu adaptive] tol {tol}", flush=True)
    out = psp.solve_adaptive(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), tol=tol)
    torch.cuda.synchronize()
    so = _check_adaptive(O, ip, ix, vals, bs, eps, tol, out)
    assert np.all(so != 1.0) if tol == 0.0 else np.all(so == 1.0)
    if tol > 1.0:
        x1, _ = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                  path="sparse_steps")
        assert torch.equal(out[0], x1)


def test_error_test_gaussian_d_and_other_nodes(dev, O, W):
    """A Gaussian diagonal D and K = 4 nodes at another ratio, on the 118-bus network."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(118, 24)
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    d = np.random.default_rng(1311).standard_normal(n)
    d /= np.abs(d).max()
    eps = W.geometric_eps(4e-3, 4, ratio=0.6)
    print("[gpu adaptive] gaussian D, K=4", flush=True)
    out = psp.solve_adaptive(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), tol=1e-11,
                             d=torch.from_numpy(d).to(dev))
    torch.cuda.synchronize()
    _check_adaptive(O, ip, ix, vals, bs, eps, 1e-11, out, d=d)


def test_error_test_graph_replays_bitwise(dev, W):
    """No host synchronisation inside the call: it captures into a HIP graph, whose replays (with
    eager work between them) reproduce the eager results."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(300, 96)
    plan = psp.Plan(ip, ix)
    eps = W.config_eps("n601")
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    ref = psp.solve_adaptive(plan, v, eps, b)
    torch.cuda.synchronize()
    print("[gpu adaptive] graph capture", flush=True)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        psp.solve_adaptive(plan, v, eps, b)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        outg = psp.solve_adaptive(plan, v, eps, b)
    for _ in range(3):
        for t in outg:
            t.fill_(-3)
        psp.solve_adaptive(plan, v, eps, b * 2.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a_, r_ in zip(outg, ref):
            assert torch.equal(a_.nan_to_num(7.0), r_.nan_to_num(7.0))


def test_error_test_argument_errors(dev, W):
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(300, 2)
    plan = psp.Plan(ip, ix)
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    with pytest.raises(psp.PSPError):
        psp.solve_adaptive(plan, v, [1e-3, 5e-4], b)          # K < 3: no estimate
    with pytest.raises(psp.PSPError):
        psp.solve_adaptive(plan, v, W.config_eps("n601"), b, tol=-1.0)
    with pytest.raises(psp.PSPError):
        psp.solve_adaptive(plan, v, [1e-3, 1e-3, 5e-4], b)    # nodes not distinct


def test_rho_iteration_kept_factors_branch(dev, O, W):
    """A pattern too large for the step schedule (1354 buses, n = 2709) keeps one factorisation
    and solves with it each step; the iteration still equals the oracle's."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, _ = W.scenario_batch(1354, 2)
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    sym = O.symbolic(n, ip, ix)
    v0 = np.random.default_rng(10).standard_normal((2, n))
    print("[gpu adaptive] rho iteration, n = 2709", flush=True)
    rho = psp.estimate_rho(plan, torch.from_numpy(vals).to(dev), torch.from_numpy(v0).to(dev), iters=12).cpu().numpy()
    for s in range(2):
        ref = O.power_rho_pivot_free(n, ip, ix, vals[s], sym, None, 1e-8, v0[s], 12)
        assert abs(rho[s] - ref) <= 1e-13 * ref, (s, rho[s], ref)


@pytest.mark.parametrize("count", [14, 110])
def test_error_test_on_dense_block_path_matches_oracle(dev, O, W, count):
    """n = 2,709 (no step schedule: the dense-trailing-block path, factors below the block
    interleaved): the first solve keeps the perturbed solutions, the error test picks the node
    scales, every Jacobian is solved again at its scale (1 for those that passed: the same bits);
    x, info, est and scale equal the oracle's, and the recovered x meet 1e-9 against a pivoted
    solve on all but a few (the 110-Jacobian item of the uneven batch: most need a smaller scale)."""
    from paper_2311_11833_amd import psp
    import scipy.sparse as sps
    import scipy.sparse.linalg as spla
    ip, ix, vals, bs = W.scenario_batch(1354, count)
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    assert plan.info().steps == 0 and plan.info().tail_n > 0
    eps = W.config_eps("n601")
    print(f"[gpu adaptive] error test + rescale, dense-block path, {count} x K=5", flush=True)
    out = psp.solve_adaptive(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), tol=1e-10)
    torch.cuda.synchronize()
    so = _check_adaptive(O, ip, ix, vals, bs, eps, 1e-10, out)
    assert int((so != 1.0).sum()) >= count // 4
    x = out[0].cpu().numpy()
    err = np.array([np.abs(x[s] - (xs := spla.splu(sps.csr_matrix((vals[s], ix, ip), shape=(n, n)).tocsc())
                                   .solve(bs[s]))).max() / np.abs(xs).max() for s in range(count)])
    assert int((err > 1e-9).sum()) <= max(1, count // 50)
