"""Newton-Raphson power flow on the GPU (psp_pf_eval / psp_pf_newton) against the oracle.

The kernels apply the oracle's operations in its order (no contraction), so the only
difference is cos/sin: the device's and the host's may differ in the last bit.  Each
P_i, Q_i and Jacobian entry is a short sum of products of those values, so the tolerance
is 64 units of rounding times the row's magnitude sum_j |V_i V_j| (|G_ij| + |B_ij|) plus the
entry's own size.  Newton iterates then agree to the conditioning of the converged
system times that (1e-11 absolute here), and every status and iteration count is equal."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U = np.finfo(np.float64).eps / 2
EPS = np.array([1e-3 * 0.5 ** k for k in range(5)])


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2311_11833_amd import psp, workloads as W
    from oracle import powerflow as PF
    return torch, psp, W, PF


def _case(mods, N, batch, seed=3110):
    torch, psp, W, PF = mods
    c = W.pf_case(N)
    sc = W.pf_scenarios(c, batch, seed=seed)
    plan = psp.Plan(c.indptr, c.indices)
    pf = psp.PowerFlow(plan, c.y_indptr, c.y_indices, c.g, c.b, c.pv)
    return c, sc, plan, pf


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _row_scale(c, x):
    N = c.N
    i = np.repeat(np.arange(N), np.diff(c.y_indptr))
    j = c.y_indices
    w = np.abs(x[N + i] * x[N + j]) * (np.abs(c.g) + np.abs(c.b))
    s = np.zeros(N)
    np.add.at(s, i, w)
    return s


def _random_states(c, batch, seed):
    rng = np.random.default_rng(seed)
    N = c.N
    return np.concatenate([rng.uniform(-0.3, 0.3, (batch, N)), rng.uniform(0.9, 1.1, (batch, N)),
                           rng.uniform(-1, 1, (batch, 1))], axis=1)


@pytest.mark.parametrize("N,batch", [(14, 8), (300, 8), (1354, 3)])
def test_eval_matches_oracle(mods, N, batch):
    torch, psp, W, PF = mods
    c, sc, plan, pf = _case(mods, N, batch)
    x = _random_states(c, batch, 5 + N)
    x[0] = sc.x_target[0]                      # one state at a root
    F, J, fn = pf.eval(_dev(torch, x), _dev(torch, sc.spec), _dev(torch, sc.part))
    torch.cuda.synchronize()
    F, J, fn = F.cpu().numpy(), J.cpu().numpy(), fn.cpu().numpy()
    rows = np.repeat(np.arange(c.n), np.diff(c.indptr))
    bus = np.where(rows < 2 * N, rows % N, 0)
    nbit = 0
    for s in range(batch):
        Fo = PF.mismatch(c.y_indptr, c.y_indices, c.g, c.b, c.pv, x[s], sc.spec[s], sc.part[s])
        Jo = PF.jacobian_values(c.y_indptr, c.y_indices, c.g, c.b, c.pv, x[s], sc.part[s], c.indptr, c.indices)
        rs = _row_scale(c, x[s])
        fscale = np.concatenate([rs + np.abs(sc.spec[s, :N]) + np.abs(sc.part[s] * x[s, -1]),
                                 rs + np.abs(sc.spec[s, N:2 * N]) + 1.0, [1.0]])
        assert np.all(np.abs(F[s] - Fo) <= 64 * U * fscale), s
        jscale = rs[bus] / np.minimum(x[s, N + bus], 1.0) + np.abs(Jo) + 1.0
        assert np.all(np.abs(J[s] - Jo) <= 64 * U * jscale), s
        assert fn[s] == np.abs(F[s]).max()
        nbit += int(np.sum(J[s] == Jo))
    assert np.abs(F[0]).max() <= 1e-12 * max(1.0, np.abs(sc.spec[0]).max())
    print(f"N={N}: {nbit} of {J.size} Jacobian entries bit-identical to the oracle")


@pytest.mark.parametrize("N,batch", [(14, 6), (300, 12), (1354, 3)])
def test_newton_matches_oracle(mods, N, batch):
    """(1354 buses, n = 2709: too large for the step schedule, so the per-level path solves.)"""
    torch, psp, W, PF = mods
    c, sc, plan, pf = _case(mods, N, batch)
    x, iters, status, fn = pf.newton(_dev(torch, sc.x0), _dev(torch, sc.spec), _dev(torch, sc.part), EPS,
                                     tol=1e-9, max_iter=10)
    torch.cuda.synchronize()
    xo, io, so, fo, _ = PF.newton(c.y_indptr, c.y_indices, c.g, c.b, c.pv, c.indptr, c.indices, sc.x0, sc.spec,
                                  sc.part, EPS, tol=1e-9, max_iter=10)
    x, iters, status, fn = x.cpu().numpy(), iters.cpu().numpy(), status.cpu().numpy(), fn.cpu().numpy()
    assert np.array_equal(status, so) and np.all(status == 0)
    assert np.array_equal(iters, io)
    assert np.abs(x - xo).max() <= 1e-11
    assert np.all(fn <= 1e-9)
    # stopping at max|F| <= 1e-9 leaves x - x* ~ J^-1 F, of order ||J^-1|| 1e-9
    assert np.abs(x - sc.x_target).max() <= 1e-8


def test_newton_paths_and_gaussian_d_agree(mods):
    """The solve is bitwise identical on every sparse path, so the Newton loop is too."""
    torch, psp, W, PF = mods
    c, sc, plan, pf = _case(mods, 300, 16)
    args = (_dev(torch, sc.x0), _dev(torch, sc.spec), _dev(torch, sc.part))
    ref = pf.newton(*args, EPS, path="sparse_batched")
    for path in ("auto", "sparse_steps", "sparse_levels", "sparse_lds"):
        out = pf.newton(*args, EPS, path=path)
        for a, b in zip(ref, out):
            assert torch.equal(a, b), path
    d = np.random.default_rng(1311).standard_normal(c.n)
    d /= np.abs(d).max()
    xg, ig, sg, fg = pf.newton(*args, EPS, d=_dev(torch, d))
    xo, io, so, fo, _ = PF.newton(c.y_indptr, c.y_indices, c.g, c.b, c.pv, c.indptr, c.indices, sc.x0[:4],
                                  sc.spec[:4], sc.part[:4], EPS, d=d)
    assert np.array_equal(sg.cpu().numpy()[:4], so) and np.array_equal(ig.cpu().numpy()[:4], io)
    assert np.abs(xg.cpu().numpy()[:4] - xo).max() <= 1e-11


def test_newton_status_codes(mods):
    torch, psp, W, PF = mods
    c, sc, plan, pf = _case(mods, 14, 4)
    x0 = sc.x0.copy()
    x0[1] = sc.x_target[1]            # already a root
    x0[2, c.N + 3] = np.nan           # not finite
    args = (_dev(torch, x0), _dev(torch, sc.spec), _dev(torch, sc.part))
    x, it, st, fn = [t.cpu().numpy() for t in pf.newton(*args, EPS, max_iter=10)]
    assert list(st) == [0, 0, 3, 0] and it[1] == 0 and it[2] == 0 and np.isnan(fn[2])
    assert np.array_equal(x[2], x0[2], equal_nan=True)
    x, it, st, fn = [t.cpu().numpy() for t in pf.newton(*args, EPS, max_iter=1)]
    assert list(st) == [1, 0, 3, 1] and list(it) == [1, 0, 0, 1]
    x, it, st, fn = [t.cpu().numpy() for t in pf.newton(*args, EPS, max_iter=0)]
    assert list(st) == [1, 0, 3, 1] and np.all(it == 0)
    assert np.array_equal(x, x0, equal_nan=True)
    with pytest.raises(psp.PSPError):
        pf.newton(*args, EPS, tol=-1.0)
    with pytest.raises(psp.PSPError):
        pf.newton(*args, np.array([1e-3, 1e-3]))


def test_newton_full_batch_sampled(mods):
    """The benchmark's configuration (300 buses, 512 scenarios, flat start, at most 20
    iterations): every scenario converges (max|F| <= 1e-9).  A few pass near a fold of the
    power-flow equations, converge only linearly and may reach another root than the one
    their specification was drawn from (the same happens with LAPACK's pivoted solve);
    every such scenario, and five random others, must equal the oracle's loop."""
    torch, psp, W, PF = mods
    c, sc, plan, pf = _case(mods, 300, 512)
    x, it, st, fn = [t.cpu().numpy() for t in pf.newton(_dev(torch, sc.x0), _dev(torch, sc.spec),
                                                        _dev(torch, sc.part), EPS, max_iter=20)]
    assert np.all(st == 0) and np.all(fn <= 1e-9)
    far = np.nonzero(np.abs(x - sc.x_target).max(axis=1) > 1e-8)[0]
    assert len(far) <= 8
    print(f"{512 - len(far)} of 512 at their target; others {far.tolist()}, iterations {it[far].tolist()}")
    pick = np.concatenate([far, np.random.default_rng(7).choice(512, 5, replace=False)])
    xo, io, so, _, _ = PF.newton(c.y_indptr, c.y_indices, c.g, c.b, c.pv, c.indptr, c.indices, sc.x0[pick],
                                 sc.spec[pick], sc.part[pick], EPS, max_iter=20)
    assert np.array_equal(it[pick], io) and np.array_equal(st[pick], so)
    assert np.abs(x[pick] - xo).max() <= 1e-11
