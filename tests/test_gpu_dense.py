"""GPU parity of the dense path against the oracle (through the C ABI).

The dense kernels apply the oracle's operation sequence (ascending-pivot fma
updates, IEEE division, column-oriented substitutions, ascending-k combine),
so results are compared bit for bit; the 1e-12 relative bound of the
perturbed solves is asserted as well, so a failure says which one broke.
"""
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


def _run_fused(psp, dev, ip, ix, vals, bs, eps, order="md", path="dense"):
    plan = psp.Plan(ip, ix, order=order)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), path=path)
    torch.cuda.synchronize()
    return plan, x.cpu().numpy(), info.cpu().numpy()


def _check(xg, xo, info_g, info_o):
    assert np.array_equal(info_g, info_o)
    ok = info_o.max(axis=1) == 0
    rel = np.abs(xg[ok] - xo[ok]).max() / np.abs(xo[ok]).max()
    assert rel <= 1e-12, rel
    assert np.array_equal(xg[ok], xo[ok])


@pytest.mark.parametrize("N,count,order", [(14, 3, "md"), (14, 2, "natural"), (30, 4, "md"), (118, 2, "md"),
                                           (300, 2, "md"), (300, 1, "natural"), (500, 1, "md")])
def test_fused_matches_oracle_bitwise(psp, O, W, dev, N, count, order):
    ip, ix, vals, bs = W.scenario_batch(N, count)
    n = len(ip) - 1
    eps = W.config_eps("small" if N == 14 else "n601")
    print(f"[gpu dense] N={N} n={n} count={count} order={order}", flush=True)
    plan, xg, ig = _run_fused(psp, dev, ip, ix, vals, bs, eps, order)
    sym = O.symbolic(n, ip, ix, natural=(order == "natural"))
    xo, io, _, _ = O.dense_batch(n, ip, ix, vals, eps, bs, perm=sym.perm)
    _check(xg, xo, ig, io)


def test_fused_multi_rhs_and_d(psp, O, W, dev):
    ip, ix, vals, _ = W.scenario_batch(30, 2)
    n = len(ip) - 1
    rng = np.random.default_rng(2)
    B = rng.standard_normal((2, n, 5))
    d = rng.standard_normal(n)
    d /= np.abs(d).max()
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(B).to(dev), path="dense",
                                d=torch.from_numpy(d).to(dev))
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.dense_batch(n, ip, ix, vals, eps, B, perm=sym.perm, d=d)
    _check(x.cpu().numpy(), xo, info.cpu().numpy(), io)


def test_breakdown_reported_in_info(psp, O, W, dev):
    ip, ix, vals, bs = W.scenario_batch(14, 2)
    vals = vals.copy()
    vals[1, 5] = np.nan
    n = len(ip) - 1
    eps = W.config_eps("small")
    plan, xg, ig = _run_fused(psp, dev, ip, ix, vals, bs, eps)
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.dense_batch(n, ip, ix, vals, eps, bs, perm=sym.perm)
    assert np.array_equal(ig, io) and np.all(ig[1] > 0) and np.all(ig[0] == 0)
    assert np.all(np.isnan(xg[1]))
    assert np.array_equal(xg[0], xo[0])


def test_split_factor_solve_combine_grad(psp, O, W, dev):
    ip, ix, vals, _ = W.scenario_batch(30, 2)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    rng = np.random.default_rng(6)
    B = rng.standard_normal((2, n, 3))
    Wt = rng.standard_normal((2, n, 3))
    plan = psp.Plan(ip, ix)
    F = psp.Factors(plan, torch.from_numpy(vals).to(dev), eps, path="dense", nrhs_cap=3)
    Xk = F.solve(torch.from_numpy(B).to(dev))
    Lk = F.solve(torch.from_numpy(Wt).to(dev), transpose=True)
    X = F.combine(Xk)
    gb = F.combine(Lk)
    gA = F.grad_values(Lk, Xk)
    torch.cuda.synchronize()
    sym = O.symbolic(n, ip, ix)
    for s in range(2):
        for k, e in enumerate(eps):
            xo, info = O.dense_system(n, ip, ix, vals[s], e, B[s], perm=sym.perm)
            assert info == 0
            assert np.array_equal(Xk[s, k].cpu().numpy(), xo)
        # transposed: oracle sparse_system(trans) equals the dense transposed sequence bitwise
        lk = np.stack([O.sparse_system(n, ip, ix, vals[s], sym, e, Wt[s], trans=True)[0] for e in eps])
        xk = np.stack([O.sparse_system(n, ip, ix, vals[s], sym, e, B[s])[0] for e in eps])
        assert np.array_equal(Lk[s].cpu().numpy(), lk)
        c = O.weights(eps)
        assert np.array_equal(X[s].cpu().numpy(), O.combine(c, xk))
        assert np.array_equal(gb[s].cpu().numpy(), O.combine(c, lk))
        assert np.array_equal(gA[s].cpu().numpy(), O.grad_values(n, ip, ix, c, xk, lk))


def test_full_size_batched_sampled(psp, O, W, dev):
    """The n=601 batched workload at full size (512 scenarios x K=5) in the
    benchmark's launch configuration; a sample of Jacobians checked against
    the oracle bitwise, the rest checked for finiteness and info == 0."""
    ip, ix, vals, bs = W.scenario_batch(300, 512)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan, xg, ig = _run_fused(psp, dev, ip, ix, vals, bs, eps)
    assert np.all(ig == 0) and np.all(np.isfinite(xg))
    sym = O.symbolic(n, ip, ix)
    for s in (0, 77, 511):
        xo, io, _, _ = O.dense_batch(n, ip, ix, vals[s:s + 1], eps, bs[s:s + 1], perm=sym.perm)
        _check(xg[s:s + 1], xo, ig[s:s + 1], io)
