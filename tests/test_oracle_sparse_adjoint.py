"""Oracle pins for the sparse pivot-free LU / substitutions (equal to the dense ones
bitwise, since they apply the same operations in the same order and skip only exact
zeros) and for the adjoint gradient (central finite differences, dense-inverse
gradient, dot-product test)."""
import numpy as np
import pytest


def _sys(W, N, count=1, first=0):
    ip, ix, vals, bs = W.scenario_batch(N, count, first=first)
    return len(ip) - 1, ip, ix, vals, bs


def _dense_from_sparse_factors(n, s, ud, lv, uv):
    L = np.eye(n)
    U = np.diag(ud)
    for j in range(n):
        rows = s.li[s.lp[j]:s.lp[j + 1]]
        L[rows, j] = lv[s.lp[j]:s.lp[j + 1]]
        U[j, rows] = uv[s.lp[j]:s.lp[j + 1]]
    return L, U


@pytest.mark.parametrize("N,natural", [(14, False), (14, True), (118, False), (300, False)])
def test_sparse_lu_equals_dense_lu_bitwise(O, W, N, natural):
    n, ip, ix, vals, bs = _sys(W, N)
    s = O.symbolic(n, ip, ix, natural=natural)
    for eps in (1e-3, 2.5e-3):
        ud, lv, uv, info = O.sparse_lu(n, ip, ix, vals[0], s, eps)
        assert info == 0
        L, U = _dense_from_sparse_factors(n, s, ud, lv, uv)
        A = W.to_dense(n, ip, ix, vals[0])[np.ix_(s.perm, s.perm)] + eps * np.eye(n)
        LU, info_d = O.lu_nopiv(A)
        assert info_d == 0
        # every dense entry outside the fill is exactly zero, every entry inside equal
        assert np.array_equal(np.tril(LU, -1) + np.eye(n), L)
        assert np.array_equal(np.triu(LU), U)
        for trans in (False, True):
            xs, _ = O.sparse_system(n, ip, ix, vals[0], s, eps, bs[0], trans=trans)
            xd_perm = O.solve_lu(LU, bs[0][s.perm], trans=trans)
            xd = np.empty(n)
            xd[s.perm] = xd_perm
            assert np.array_equal(xs, xd)


def test_sparse_multi_rhs_and_trans_vs_library(O, W):
    n, ip, ix, vals, _ = _sys(W, 300)
    s = O.symbolic(n, ip, ix)
    B = np.random.default_rng(1).standard_normal((n, 8))
    A = W.to_dense(n, ip, ix, vals[0]) + 1e-3 * np.eye(n)
    for trans in (False, True):
        x, info = O.sparse_system(n, ip, ix, vals[0], s, 1e-3, B, trans=trans)
        ref = np.linalg.solve(A.T if trans else A, B)
        assert np.abs(x - ref).max() / np.abs(ref).max() < 1e-10


def test_sparse_breakdown_info(O, W):
    n, ip, ix, vals, bs = _sys(W, 14)
    s = O.symbolic(n, ip, ix, natural=True)
    v = vals[0].copy()
    v[0] = np.nan          # entry (0, *) of row 0: first row's first stored value
    ud, lv, uv, info = O.sparse_lu(n, ip, ix, v, s, 0.0)
    assert info >= 1
    x, info2 = O.sparse_system(n, ip, ix, v, s, 0.0, bs[0])
    assert info2 == info and np.all(np.isnan(x))


def _method(O, n, ip, ix, v, b, s, eps):
    x, info, _, _ = O.sparse_batch(n, ip, ix, v[None], s, eps, b[None])
    assert np.all(info == 0)
    return x[0]


def _adjoint(O, n, ip, ix, v, Wt, X, s, eps):
    c = O.weights(eps)
    xk = np.stack([O.sparse_system(n, ip, ix, v, s, e, X)[0] for e in eps])
    lk = np.stack([O.sparse_system(n, ip, ix, v, s, e, Wt, trans=True)[0] for e in eps])
    gb = O.combine(c, lk)
    gA = O.grad_values(n, ip, ix, c, xk, lk)
    return gA, gb


def test_adjoint_vs_central_fd_small(O, W):
    """L = sum w . x_hat; every pattern entry of A and every entry of b, h = 1e-6 absolute."""
    n, ip, ix, vals, bs = _sys(W, 14)
    s = O.symbolic(n, ip, ix)
    eps = W.config_eps("small")
    rng = np.random.default_rng(4)
    nrhs = 2
    B = np.stack([bs[0], rng.standard_normal(n)], axis=1)
    Wt = rng.standard_normal((n, nrhs))
    gA, gb = _adjoint(O, n, ip, ix, vals[0], Wt, B, s, eps)

    def loss(v, Bm):
        x, info, _, _ = O.sparse_batch(n, ip, ix, v[None], s, eps, Bm[None])
        return float(np.sum(Wt * x[0]))

    h = 1e-6
    fd = np.empty_like(gA)
    for e in range(len(gA)):
        vp, vm = vals[0].copy(), vals[0].copy()
        vp[e] += h
        vm[e] -= h
        fd[e] = (loss(vp, B) - loss(vm, B)) / (2 * h)
    assert np.abs(fd - gA).max() <= 1e-6 * np.abs(gA).max()
    fdb = np.empty_like(gb)
    for i in range(n):
        for r in range(nrhs):
            Bp, Bm = B.copy(), B.copy()
            Bp[i, r] += h
            Bm[i, r] -= h
            fdb[i, r] = (loss(vals[0], Bp) - loss(vals[0], Bm)) / (2 * h)
    assert np.abs(fdb - gb).max() <= 1e-6 * np.abs(gb).max()


def test_adjoint_vs_dense_inverse_and_dot_product(O, W):
    """601 unknowns, 8 RHS: gradient of x_hat agrees with the exact-solution gradient
    -A^{-T} W X*^T on pat(A) up to the truncation level; directional FD matches."""
    n, ip, ix, vals, bs = _sys(W, 300, first=1)      # scenario with rho(A^{-1}) ~ 20
    s = O.symbolic(n, ip, ix)
    eps = W.config_eps("adjoint")
    rng = np.random.default_rng(8)
    nrhs = 8
    B = rng.standard_normal((n, nrhs))
    Wt = rng.standard_normal((n, nrhs))
    gA, gb = _adjoint(O, n, ip, ix, vals[0], Wt, B, s, eps)
    A = W.to_dense(n, ip, ix, vals[0])
    Xs = np.linalg.solve(A, B)
    Lam = np.linalg.solve(A.T, Wt)
    rows = np.repeat(np.arange(n), np.diff(ip))
    gA_ref = -np.einsum("er,er->e", Lam[rows], Xs[ix])
    assert np.abs(gA - gA_ref).max() <= 1e-9 * np.abs(gA_ref).max()
    assert np.abs(gb - Lam).max() <= 1e-9 * np.abs(Lam).max()
    # dot-product test against a directional central difference
    dA = rng.standard_normal(len(gA))
    dB = rng.standard_normal(B.shape)
    h = 1e-6

    def loss(t):
        x = np.stack([_method(O, n, ip, ix, vals[0] + t * dA, B[:, r] + t * dB[:, r], s, eps)
                      for r in range(nrhs)], axis=1)
        return float(np.sum(Wt * x))

    fd = (loss(h) - loss(-h)) / (2 * h)
    an = float(np.dot(gA, dA) + np.sum(gb * dB))
    assert fd == pytest.approx(an, rel=1e-6)
