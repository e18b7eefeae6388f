"""GPU parity of the sparse (fill-pattern) path against the oracle, through the C ABI.

The level-scheduled kernels evaluate every factor entry and every substitution
row with the oracle's operations in the oracle's order, so factors, perturbed
solutions and combined solutions are compared bit for bit (the 1e-12 relative
bound is asserted first so a failure names which bar broke)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def psp():
    from paper_2311_11833_amd import psp as m
    m.lib()
    return m


def _cmp(xg, xo):
    rel = np.abs(xg - xo).max() / np.abs(xo).max()
    assert rel <= 1e-12, rel
    assert np.array_equal(xg, xo)


@pytest.mark.parametrize("N,count,nrhs", [(14, 3, 1), (30, 4, 1), (30, 2, 7), (118, 2, 1), (300, 3, 1),
                                          (500, 1, 2), (1354, 2, 1)])
def test_fused_sparse_matches_oracle(psp, O, W, dev, N, count, nrhs):
    ip, ix, vals, bs = W.scenario_batch(N, count)
    n = len(ip) - 1
    if nrhs > 1:
        bs = np.random.default_rng(N).standard_normal((count, n, nrhs))
    eps = W.config_eps("small" if N == 14 else "n601")
    print(f"[gpu sparse] N={N} n={n} count={count} nrhs={nrhs}", flush=True)
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), path="sparse")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    assert np.array_equal(info.cpu().numpy(), io)
    _cmp(x.cpu().numpy(), xo)


@pytest.mark.parametrize("N", [30, 1354])
def test_split_sparse_solve_trans_grad(psp, O, W, dev, N):
    ip, ix, vals, _ = W.scenario_batch(N, 2)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    rng = np.random.default_rng(3)
    B = rng.standard_normal((2, n, 4))
    Wt = rng.standard_normal((2, n, 4))
    plan = psp.Plan(ip, ix)
    F = psp.Factors(plan, torch.from_numpy(vals).to(dev), eps, path="sparse", nrhs_cap=4)
    Xk = F.solve(torch.from_numpy(B).to(dev))
    Lk = F.solve(torch.from_numpy(Wt).to(dev), transpose=True)
    X = F.combine(Xk)
    gA = F.grad_values(Lk, Xk)
    torch.cuda.synchronize()
    assert np.all(F.info.cpu().numpy() == 0)
    sym = O.symbolic(n, ip, ix)
    c = O.weights(eps)
    for s in range(2):
        xk = np.stack([O.sparse_system(n, ip, ix, vals[s], sym, e, B[s])[0] for e in eps])
        lk = np.stack([O.sparse_system(n, ip, ix, vals[s], sym, e, Wt[s], trans=True)[0] for e in eps])
        _cmp(Xk[s].cpu().numpy(), xk)
        _cmp(Lk[s].cpu().numpy(), lk)
        _cmp(X[s].cpu().numpy(), O.combine(c, xk))
        _cmp(gA[s].cpu().numpy(), O.grad_values(n, ip, ix, c, xk, lk))


@pytest.mark.parametrize("N", [14, 1354])
def test_sparse_breakdown_info(psp, O, W, dev, N):
    ip, ix, vals, bs = W.scenario_batch(N, 2)
    vals = vals.copy()
    vals[1, 3] = np.inf
    n = len(ip) - 1
    eps = W.config_eps("small")
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), path="sparse")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    ig = info.cpu().numpy()
    assert np.array_equal(ig, io) and np.all(ig[1] > 0) and np.all(ig[0] == 0)
    xg = x.cpu().numpy()
    assert np.all(np.isnan(xg[1]))
    _cmp(xg[0], xo[0])


def test_large_sparse_sampled(psp, O, W, dev):
    """20,001 unknowns (10,000-bus network), K = 4, 32 right-hand sides, forward and
    transposed solves in the launch configuration of the benchmark (the dense trailing
    block of 1,521 columns on the MFMA unit); one perturbed system and four RHS columns
    recomputed by the oracle, and the gradient on the whole pattern equal to the oracle's
    on the same perturbed solutions and adjoints."""
    from paper_2311_11833_amd.workloads import make_network, make_state, jacobian, seed_state
    net = make_network(10000)
    vm, va, p = make_state(10000, seed_state(10000, 0))
    J = jacobian(net, vm, va, p)
    n = J.n
    eps = W.large_eps()
    rng = np.random.default_rng(10)
    B = rng.standard_normal((1, n, 32))
    plan = psp.Plan(J.indptr, J.indices)
    F = psp.Factors(plan, torch.from_numpy(J.data[None]).to(dev), eps, path="sparse", nrhs_cap=32)
    Xk = F.solve(torch.from_numpy(B).to(dev))
    Lk = F.solve(torch.from_numpy(B).to(dev), transpose=True)
    torch.cuda.synchronize()
    assert np.all(F.info.cpu().numpy() == 0)
    sym = O.symbolic(n, J.indptr, J.indices)
    xo, info = O.sparse_system(n, J.indptr, J.indices, J.data, sym, eps[0], B[0][:, :4].copy())
    lo, _ = O.sparse_system(n, J.indptr, J.indices, J.data, sym, eps[0], B[0][:, :4].copy(), trans=True)
    assert info == 0
    _cmp(Xk[0, 0, :, :4].cpu().numpy(), xo)
    _cmp(Lk[0, 0, :, :4].cpu().numpy(), lo)
    assert np.all(np.isfinite(Xk.cpu().numpy()))
    # the gradient on A's pattern from these K perturbed solutions and adjoints, all 154,001 entries
    gA = F.grad_values(Lk, Xk)
    torch.cuda.synchronize()
    go = O.grad_values(n, J.indptr, J.indices, O.weights(eps), Xk[0].cpu().numpy(), Lk[0].cpu().numpy())
    _cmp(gA[0].cpu().numpy(), go)


@pytest.mark.parametrize("variant", ["sparse_batched", "sparse_grouped", "sparse_lds", "sparse_levels", "sparse_steps"])
def test_sparse_variants_match_oracle(psp, O, W, dev, variant):
    """The executions of the sparse path (systems interleaved across lanes per level or
    per group, one workgroup per system in LDS by levels or by dataflow steps, per-level
    kernels over task-major factors) on the same 64-Jacobian batch: each equal to the
    oracle bitwise."""
    ip, ix, vals, bs = W.scenario_batch(118, 64)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), path=variant)
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    assert np.array_equal(info.cpu().numpy(), io)
    _cmp(x.cpu().numpy(), xo)


def test_tuner_picks_a_path_and_auto_uses_it(psp, O, W, dev):
    ip, ix, vals, bs = W.scenario_batch(118, 64)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    chosen, times = psp.tune(plan, v, eps, b)
    assert chosen in times and times[chosen] == min(times.values())
    assert set(times) >= {"dense", "sparse_batched", "sparse_grouped", "sparse_lds", "sparse_levels", "sparse_steps"}
    x, info = psp.solve_batched(plan, v, eps, b, path="auto")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    _cmp(x.cpu().numpy(), xo)


@pytest.mark.parametrize("path", ["sparse", "sparse_steps"])
def test_sparse_full_size_batched_sampled(psp, O, W, dev, path):
    """n=601, 512 Jacobians x K=5 in the benchmark's launch configurations: every
    system info == 0, all finite, sampled Jacobians equal to the oracle bitwise,
    and a broken-down Jacobian among them reported alone."""
    ip, ix, vals, bs = W.scenario_batch(300, 512)
    vals = vals.copy()
    vals[300, 10] = np.nan
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    print(f"[gpu sparse] full size path={path}", flush=True)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), path=path)
    torch.cuda.synchronize()
    xg, ig = x.cpu().numpy(), info.cpu().numpy()
    bad = np.zeros(512, bool)
    bad[300] = True
    assert np.all(ig[~bad] == 0) and np.all(ig[300] > 0)
    assert np.all(np.isfinite(xg[~bad])) and np.all(np.isnan(xg[300]))
    sym = O.symbolic(n, ip, ix)
    for s in (0, 255, 300, 511):
        xo, io, _, _ = O.sparse_batch(n, ip, ix, vals[s:s + 1], sym, eps, bs[s:s + 1])
        assert np.array_equal(ig[s:s + 1], io)
        if s != 300:
            _cmp(xg[s:s + 1], xo)


@pytest.mark.parametrize("N,count", [(14, 3), (30, 300), (118, 260), (30, 520), (118, 600)])
def test_steps_path_modes_and_breakdown(psp, O, W, dev, N, count):
    """Dataflow-step execution in both launch modes (one workgroup per perturbed system
    plus a combine launch when the batch is smaller than the resident workgroup slots,
    two per CU here; one workgroup per Jacobian with the combine fused otherwise), with
    one Jacobian broken by an infinite entry: info and solutions equal to the oracle, the
    broken Jacobian NaN."""
    ip, ix, vals, bs = W.scenario_batch(N, count)
    vals = vals.copy()
    vals[1, 2] = np.inf
    n = len(ip) - 1
    eps = W.config_eps("small" if N == 14 else "n601")
    print(f"[gpu sparse] steps N={N} count={count}", flush=True)
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                path="sparse_steps")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    ig, xg = info.cpu().numpy(), x.cpu().numpy()
    assert np.array_equal(ig, io) and np.all(ig[1] > 0)
    assert np.all(np.isnan(xg[1]))
    keep = np.ones(count, bool)
    keep[1] = False
    _cmp(xg[keep], xo[keep])


@pytest.mark.parametrize("count", [3, 260])
def test_steps_path_packed_slots(psp, O, W, dev, count):
    """The 500-bus pattern (n = 1,001) fits in LDS only with its L and U values packed into
    shared slots by live interval; in both launch modes the results equal the oracle bit for
    bit (every Jacobian for 3, sampled ones for 260)."""
    ip, ix, vals, bs = W.scenario_batch(500, count)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    print(f"[gpu sparse] packed steps n={n} count={count}", flush=True)
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                path="sparse_steps")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    pick = list(range(count)) if count <= 3 else [0, 1, 129, 255, 259]
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals[pick], sym, eps, bs[pick])
    assert np.array_equal(info.cpu().numpy()[pick], io)
    _cmp(x.cpu().numpy()[pick], xo)


def test_steps_path_rejects_what_it_cannot_run(psp, W, dev):
    """nrhs > 1, and a fill too large for LDS even packed, are refused with PSP_E_UNSUPPORTED."""
    ip, ix, vals, bs = W.scenario_batch(30, 2)
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    b2 = torch.zeros((2, n, 2), dtype=torch.float64, device=dev)
    with pytest.raises(psp.PSPError, match="UNSUPPORTED|cannot run"):
        psp.solve_batched(plan, torch.from_numpy(vals).to(dev), W.config_eps("n601"), b2, path="sparse_steps")
    ip, ix, vals, bs = W.scenario_batch(1354, 1)
    plan = psp.Plan(ip, ix)
    with pytest.raises(psp.PSPError, match="UNSUPPORTED|cannot run"):
        psp.solve_batched(plan, torch.from_numpy(vals).to(dev), W.config_eps("n601"),
                          torch.from_numpy(bs).to(dev), path="sparse_steps")


@pytest.mark.parametrize("variant", ["sparse_batched", "sparse_grouped", "sparse_lds", "sparse_levels", "sparse_steps"])
def test_gaussian_diagonal_and_symmetric_nodes(psp, O, W, dev, variant):
    """The paper's own scheme (nodes +-alpha eps, alpha = 1, 2, eps = 2e-3) with a diagonal
    D of normally distributed entries scaled to max |d_i| = 1, on every sparse execution:
    bitwise equal to the oracle with the same D."""
    ip, ix, vals, bs = W.scenario_batch(118, 12)
    n = len(ip) - 1
    eps = np.array([2e-3, -2e-3, 4e-3, -4e-3])
    d = np.random.default_rng(41).standard_normal(n)
    d /= np.abs(d).max()
    plan = psp.Plan(ip, ix)
    print(f"[gpu sparse] gaussian D, symmetric nodes, {variant}", flush=True)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                path=variant, d=torch.from_numpy(d).to(dev))
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs, d=d)
    assert np.array_equal(info.cpu().numpy(), io)
    _cmp(x.cpu().numpy(), xo)


def test_gaussian_diagonal_split_steps_and_adjoint(psp, O, W, dev):
    """Split calls (kept factors, forward and transposed solves, gradient) with the same
    Gaussian D: equal to the oracle bitwise."""
    ip, ix, vals, _ = W.scenario_batch(30, 3)
    n = len(ip) - 1
    eps = np.array([2e-3, -2e-3, 4e-3, -4e-3])
    rng = np.random.default_rng(42)
    d = rng.standard_normal(n)
    d /= np.abs(d).max()
    B = rng.standard_normal((3, n, 2))
    Wt = rng.standard_normal((3, n, 2))
    plan = psp.Plan(ip, ix)
    F = psp.Factors(plan, torch.from_numpy(vals).to(dev), eps, path="sparse", d=torch.from_numpy(d).to(dev), nrhs_cap=2)
    Xk = F.solve(torch.from_numpy(B).to(dev))
    Lk = F.solve(torch.from_numpy(Wt).to(dev), transpose=True)
    X = F.combine(Xk)
    gA = F.grad_values(Lk, Xk)
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    c = O.weights(eps)
    for s in range(3):
        xo, _, xko, _ = O.sparse_batch(n, ip, ix, vals[s:s + 1], sym, eps, B[s:s + 1], d=d, keep_xk=True)
        lo, _, lko, _ = O.sparse_batch(n, ip, ix, vals[s:s + 1], sym, eps, Wt[s:s + 1], d=d, trans=True, keep_xk=True)
        _cmp(Xk[s].cpu().numpy(), xko[0])
        _cmp(Lk[s].cpu().numpy(), lko[0])
        _cmp(X[s].cpu().numpy(), xo[0])
        _cmp(gA[s].cpu().numpy(), O.grad_values(n, ip, ix, c, xko[0], lko[0]))


@pytest.mark.parametrize("N,count,nrhs", [(500, 3, 1), (1354, 4, 3), (3000, 2, 1)])
def test_dense_tail_path_matches_oracle(psp, O, W, dev, N, count, nrhs):
    """The dense trailing block (top separator and slack column, 87 / 231 / 547 columns at
    n = 1001 / 2709 / 6001): sparse levels below it, the block's external updates, its
    panel factorisation on the MFMA unit and its dense solves, bitwise equal to the oracle."""
    ip, ix, vals, bs = W.scenario_batch(N, count)
    n = len(ip) - 1
    if nrhs > 1:
        bs = np.random.default_rng(N).standard_normal((count, n, nrhs))
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    print(f"[gpu sparse] dense tail N={N} n={n} count={count} nrhs={nrhs}", flush=True)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                path="sparse_tail")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    assert np.array_equal(info.cpu().numpy(), io)
    _cmp(x.cpu().numpy(), xo)


@pytest.mark.parametrize("count,nrhs", [(14, 1), (13, 2), (14, 7)])
def test_dense_tail_interleaved_matches_oracle(psp, O, W, dev, count, nrhs):
    """From 64 systems on, the fused call keeps the factors below the block interleaved across
    systems (one wave serves an item of 64 systems) and each block in a region of its own: one
    Jacobian broken below the block, one inside it; info equal to the oracle's, the broken ones
    NaN, every other solution bitwise equal."""
    ip, ix, vals, bs = W.scenario_batch(1354, count)
    n = len(ip) - 1
    vals = vals.copy()
    vals[2, 0] = np.nan
    lam_entries = np.nonzero(ix == n - 1)[0]
    vals[5, lam_entries[len(lam_entries) // 3]] = np.inf
    if nrhs > 1:
        bs = np.random.default_rng(count).standard_normal((count, n, nrhs))
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    print(f"[gpu sparse] dense tail interleaved count={count} nrhs={nrhs}", flush=True)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                path="sparse_tail")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    ig, xg = info.cpu().numpy(), x.cpu().numpy()
    assert np.array_equal(ig, io) and np.all(ig[2] > 0) and np.all(ig[5] > 0)
    assert np.all(np.isnan(xg[2])) and np.all(np.isnan(xg[5]))
    keep = np.ones(count, bool)
    keep[[2, 5]] = False
    _cmp(xg[keep], xo[keep])


def test_dense_tail_breakdown_inside_block(psp, O, W, dev):
    """A NaN entry in the slack column (inside the dense block) breaks that Jacobian's K systems at
    the same pivot as the oracle's; the other Jacobian is untouched."""
    ip, ix, vals, bs = W.scenario_batch(1354, 2)
    n = len(ip) - 1
    vals = vals.copy()
    lam_entries = np.nonzero(ix == n - 1)[0]          # column of lambda, the last unknown
    vals[0, lam_entries[len(lam_entries) // 2]] = np.nan
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    print("[gpu sparse] dense tail breakdown", flush=True)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev),
                                path="sparse_tail")
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    ig = info.cpu().numpy()
    assert np.array_equal(ig, io) and np.all(ig[0] > 0) and np.all(ig[1] == 0)
    assert np.all(np.isnan(x.cpu().numpy()[0]))
    _cmp(x.cpu().numpy()[1], xo[1])


@pytest.mark.parametrize("N,count", [(1354, 13), (3000, 13)])
def test_dense_tail_launch_choices_match_oracle(psp, O, W, dev, N, count):
    """65 perturbed systems (one past the 64 of a wave of the interleaved layout) at n = 2,709 and
    6,001: every combination of the layout below the block (interleaved or one system after
    another) and of the block's LU and solves (per-panel launches across the device, split into a
    GETRF and a many-workgroup TRSM below 256 systems, or one workgroup per system) returns the
    oracle's bits."""
    ip, ix, vals, bs = W.scenario_batch(N, count)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    for il, lu in ((1, 0), (1, 1), (0, 1), (0, 0)):
        print(f"[gpu sparse] dense tail N={N} count={count} interleaved={il} lu={lu}", flush=True)
        psp.set_tune_choice(plan, count, len(eps), 1, "sparse_tail", tail_il=il, tail_lu=lu)
        x, info = psp.solve_batched(plan, v, eps, b, path="auto")
        torch.cuda.synchronize()
        assert np.array_equal(info.cpu().numpy(), io)
        _cmp(x.cpu().numpy(), xo)
