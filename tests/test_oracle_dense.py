"""Oracle pins for dense pivot-free LU, substitutions, the pivoted ground truth and
the expansion error of the combined solution (Sec. II-B, III-A, IV).

Pins: exact integer factorisations, exact rational arithmetic on tiny systems,
LAPACK special cases (scipy.linalg.lu without row exchanges, numpy.linalg.solve),
the Neumann-series closed form of the truncation error, the Theorem 1
coefficient, and the zero-pivot breakdown that the paper reports.
"""
from fractions import Fraction as F

import numpy as np
import pytest
import scipy.linalg as sla


def _exact_lu(A):
    """Doolittle LU in exact rationals (unique when it exists)."""
    n = len(A)
    a = [[F(v) for v in row] for row in A]
    for k in range(n):
        assert a[k][k] != 0
        for i in range(k + 1, n):
            a[i][k] = a[i][k] / a[k][k]
            for j in range(k + 1, n):
                a[i][j] -= a[i][k] * a[k][j]
    return a


def test_lu_exact_integer_factors(O):
    """A = L0 U0 with small integers and power-of-two pivots: every step is exact."""
    rng = np.random.default_rng(3)
    for n in (1, 2, 5, 17, 40):
        L0 = np.tril(rng.integers(-3, 4, (n, n)), -1).astype(float) + np.eye(n)
        U0 = np.triu(rng.integers(-3, 4, (n, n)), 1).astype(float) + np.diag(2.0 ** rng.integers(-2, 3, n))
        A = L0 @ U0
        assert np.abs(A).max() < 2 ** 40
        LU, info = O.lu_nopiv(A)
        assert info == 0
        assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
        assert np.array_equal(np.triu(LU), U0)


def test_lu_and_solves_vs_exact_rationals(O):
    rng = np.random.default_rng(5)
    for n in (2, 3, 4, 6):
        A = rng.integers(-9, 10, (n, n)).astype(float) + np.diag(np.full(n, 25.0))
        b = rng.integers(-9, 10, n).astype(float)
        ex = _exact_lu(A)
        LU, info = O.lu_nopiv(A)
        assert info == 0
        for i in range(n):
            for j in range(n):
                assert abs(LU[i, j] - float(ex[i][j])) <= 4e-16 * max(1.0, abs(float(ex[i][j]))) * n
        xs = [F(v) for v in b]
        # exact solve x = A^{-1} b by Cramer-free rational Gauss-Jordan
        M = [[F(v) for v in row] + [xs[i]] for i, row in enumerate(A)]
        for k in range(n):
            for i in range(n):
                if i != k:
                    f = M[i][k] / M[k][k]
                    M[i] = [M[i][t] - f * M[k][t] for t in range(n + 1)]
        x_exact = np.array([float(M[i][n] / M[i][i]) for i in range(n)])
        x = O.solve_lu(LU, b)
        assert np.allclose(x, x_exact, rtol=1e-13, atol=1e-14)
        # transposed solve: A^T y = b
        M = [[F(A[j][i]) for j in range(n)] + [xs[i]] for i in range(n)]
        for k in range(n):
            for i in range(n):
                if i != k:
                    f = M[i][k] / M[k][k]
                    M[i] = [M[i][t] - f * M[k][t] for t in range(n + 1)]
        yt_exact = np.array([float(M[i][n] / M[i][i]) for i in range(n)])
        assert np.allclose(O.solve_lu(LU, b, trans=True), yt_exact, rtol=1e-13, atol=1e-14)


def test_lu_matches_lapack_without_row_exchange(O):
    """Column diagonal dominance makes partial pivoting choose no exchanges, so
    LAPACK's getrf (via scipy) computes the same unique L and U."""
    rng = np.random.default_rng(11)
    for n in (8, 33, 100):
        A = rng.standard_normal((n, n))
        A += np.diag(np.abs(A).sum(axis=0) + 1.0)
        P, L, U = sla.lu(A)
        assert np.array_equal(P, np.eye(n))
        LU, info = O.lu_nopiv(A)
        assert info == 0
        assert np.allclose(np.tril(LU, -1), np.tril(L, -1), rtol=0, atol=1e-14)
        assert np.allclose(np.triu(LU), U, rtol=1e-13, atol=1e-13)


def test_lu_backward_error_bound(O):
    rng = np.random.default_rng(13)
    n = 120
    A = rng.standard_normal((n, n)) + n ** 0.5 * np.eye(n)
    LU, info = O.lu_nopiv(A)
    assert info == 0
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    u = 2.0 ** -53
    gamma = n * u / (1 - n * u)
    assert np.abs(A - L @ U).max() <= gamma * np.abs(np.abs(L) @ np.abs(U)).max()


def test_info_on_breakdown(O):
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    assert O.lu_nopiv(A)[1] == 1
    B = np.array([[1.0, 2.0, 0.0], [2.0, 4.0, 1.0], [0.0, 1.0, 1.0]])   # leading 2x2 singular
    assert O.lu_nopiv(B)[1] == 2
    C = np.eye(3)
    C[1, 1] = np.nan
    assert O.lu_nopiv(C)[1] == 2
    # the pivoted ground truth solves what the pivot-free LU cannot
    x = O.pivoted_solve(B, np.array([1.0, 2.0, 3.0]))
    assert np.allclose(B @ x, [1.0, 2.0, 3.0], rtol=0, atol=1e-14)


def test_pivoted_matches_lapack(O, W):
    rng = np.random.default_rng(17)
    for n in (5, 64, 200):
        A = rng.standard_normal((n, n))
        b = rng.standard_normal((n, 3))
        x = O.pivoted_solve(A, b)
        xr = np.linalg.solve(A, b)
        k = np.linalg.cond(A)
        assert np.abs(x - xr).max() / np.abs(xr).max() <= 10 * 2.0 ** -53 * k * n
    ip, ix, vals, bs = W.scenario_batch(300, 1)
    n = len(ip) - 1
    A = W.to_dense(n, ip, ix, vals[0])
    x = O.pivoted_solve(A, bs[0])
    xr = np.linalg.solve(A, bs[0])
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-11


def test_partial_pivot_tie_rule(O):
    """Equal magnitudes: the row with the smaller index is the pivot."""
    A = np.array([[1.0, 2.0], [-1.0, 3.0]])
    b = np.array([3.0, 2.0])
    assert np.allclose(O.pivoted_solve(A, b), np.linalg.solve(A, b), atol=1e-15)


def _jac(W, N, scen=0):
    ip, ix, vals, bs = W.scenario_batch(N, 1, first=scen)
    n = len(ip) - 1
    return n, ip, ix, vals[0], bs[0]


@pytest.mark.parametrize("N", [14, 30, 300])
def test_unperturbed_pivot_free_breaks_down(O, W, N):
    """Sec. IV: the distributed-slack Jacobian meets a (numerically) zero leading pivot.
    P depends on angles only through differences, so every row of the leading N x N block
    (P rows, angle columns) sums to zero: that block is singular and the natural-order pivot
    at 0-based index N-1 vanishes in exact arithmetic."""
    n, ip, ix, v, b = _jac(W, N)
    A = W.to_dense(n, ip, ix, v)
    LU, info = O.lu_nopiv(A)
    u = 2.0 ** -53
    piv = np.abs(np.diag(LU))
    assert info != 0 or (int(np.argmin(piv)) == N - 1 and piv[N - 1] <= 1e3 * n * u * np.abs(A).max())
    # the leading block really is singular: the angle columns of every P and Q row sum to zero
    assert np.abs(A[:2 * N, :N].sum(axis=1)).max() <= 1e-12 * np.abs(A).max()
    x_star = O.pivoted_solve(A, b)
    x0, info0 = O.dense_system(n, ip, ix, v, 0.0, b)
    bad = info0 != 0 or not np.all(np.isfinite(x0)) or np.abs(x0 - x_star).max() / np.abs(x_star).max() > 1e-2
    assert bad
    # A + eps D is factorable: no breakdown, pivots well away from rounding level, tiny backward error
    for eps in (1e-2, 1e-3):
        Ae = A + eps * np.eye(n)
        LUe, infoe = O.lu_nopiv(Ae)
        assert infoe == 0
        assert np.abs(np.diag(LUe)).min() > n * u * np.abs(Ae).max()
        L = np.tril(LUe, -1) + np.eye(n)
        Ue = np.triu(LUe)
        assert np.abs(Ae - L @ Ue).max() / np.abs(Ae).max() <= 1e-12


def test_truncation_error_closed_form_small(O, W):
    """x_hat - x* = sum_{j>=K} mu_j (-1)^j (A^{-1} D)^j x*, mu_j = sum_k c_k eps_k^j (Neumann series,
    eq. neumann_2, with Remark 2's moment conditions mu_0 = 1, mu_1..mu_{K-1} = 0).  The leading
    term is -(prod eps_k) (A^{-1} D)^K x*; the first three terms must match within 1%."""
    n, ip, ix, v, b = _jac(W, 14)
    A = W.to_dense(n, ip, ix, v)
    eps = W.config_eps("small")
    K = len(eps)
    x, info, _, _ = O.dense_batch(n, ip, ix, v[None], eps, b[None])
    assert np.all(info == 0)
    xs = O.pivoted_solve(A, b)
    M = np.linalg.solve(A, np.eye(n))
    V = np.vander(eps, K, increasing=True)                   # V[k, j] = eps_k^j
    c_lib = np.linalg.solve(V.T, np.eye(K)[0])                # library solve of the moment system
    pred = sum(np.dot(c_lib, (-eps) ** j) * np.linalg.matrix_power(M, j) @ xs for j in range(K, K + 3))
    lead = -np.prod(eps) * np.linalg.matrix_power(M, K) @ xs
    err = x[0] - xs
    assert np.linalg.norm(err - pred) <= 0.01 * np.linalg.norm(pred)
    assert np.linalg.norm(err - lead) <= 0.10 * np.linalg.norm(lead)


def test_error_order_in_eps_and_K(O, W):
    """Scaling every node by s scales the error by s^K (Theorem 1's order, geometric nodes)."""
    n, ip, ix, v, b = _jac(W, 14)
    A = W.to_dense(n, ip, ix, v)
    xs = O.pivoted_solve(A, b)
    for K in (1, 2, 3):
        base = W.geometric_eps(8e-3, K)
        errs = []
        for s in (1.0, 0.5):
            x, info, _, _ = O.dense_batch(n, ip, ix, v[None], base * s, b[None])
            errs.append(np.linalg.norm(x[0] - xs) / np.linalg.norm(xs))
        ratio = errs[1] / errs[0]
        assert ratio == pytest.approx(0.5 ** K, rel=0.15), (K, errs)
    # more solves, smaller error, at fixed largest node
    e = [np.linalg.norm(O.dense_batch(n, ip, ix, v[None], W.geometric_eps(4e-3, K), b[None])[0][0] - xs)
         for K in (1, 2, 3, 4)]
    assert all(e[i + 1] < 0.2 * e[i] for i in range(3)), e


@pytest.mark.parametrize("m", [1, 2, 3])
def test_theorem1_symmetric_scheme(O, W, m):
    """Nodes +-alpha eps (eqs. xap/xam): x_hat - x* = sum_{j>=m} g_j eps^{2j} (A^{-1}D)^{2j} x* with
    g_j = sum_alpha beta_alpha alpha^{2j}; the first, g_m = (-1)^{m+1} (m!)^2, is Theorem 1's
    O(eps^{2m}) term.  beta comes from a library solve of Gamma_m^T beta = e1."""
    from math import factorial
    n, ip, ix, v, b = _jac(W, 14)
    A = W.to_dense(n, ip, ix, v)
    xs = O.pivoted_solve(A, b)
    M = np.linalg.solve(A, np.eye(n))
    rho = np.abs(np.linalg.eigvals(M)).max()
    eps = 0.05 / (m * rho)
    nodes = np.array([s * a * eps for a in range(1, m + 1) for s in (1, -1)])
    x, info, _, _ = O.dense_batch(n, ip, ix, v[None], nodes, b[None])
    G = np.array([[a ** (2 * j) for j in range(m)] for a in range(1, m + 1)], float)
    beta = np.linalg.solve(G.T, np.eye(m)[0])
    g = [float(np.dot(beta, np.arange(1, m + 1, dtype=float) ** (2 * j))) for j in (m, m + 1)]
    assert g[0] == pytest.approx((-1) ** (m + 1) * factorial(m) ** 2, rel=1e-10)
    pred = sum(gj * eps ** (2 * j) * np.linalg.matrix_power(M, 2 * j) @ xs for gj, j in zip(g, (m, m + 1)))
    assert np.linalg.norm(x[0] - xs - pred) <= 0.02 * np.linalg.norm(pred)


@pytest.mark.parametrize("scen", [0, 1, 2])
def test_n601_recovers_pivoted_solution(O, W, scen):
    """601 unknowns, 5 geometric nodes from 1e-3.  Where the predicted truncation
    (the Neumann series of the combination, leading terms) is below 1e-10, x_hat must match
    the pivoted x* within 1e-9; where it is larger (rho(A^{-1}) > ~80), the observed error
    must equal the prediction."""
    n, ip, ix, v, b = _jac(W, 300, scen)
    A = W.to_dense(n, ip, ix, v)
    xs = O.pivoted_solve(A, b)
    sym = O.symbolic(n, ip, ix)
    eps = W.config_eps("n601")
    K = len(eps)
    x, info, _, _ = O.sparse_batch(n, ip, ix, v[None], sym, eps, b[None])
    assert np.all(info == 0)
    M = np.linalg.solve(A, np.eye(n))
    c_lib = np.linalg.solve(np.vander(eps, K, increasing=True).T, np.eye(K)[0])
    pred = np.zeros(n)
    t = np.linalg.matrix_power(M, K) @ xs
    for j in range(K, K + 8):
        pred += np.dot(c_lib, (-eps) ** j) * t
        t = M @ t
    err = x[0] - xs
    scale = np.abs(xs).max()
    if np.abs(pred).max() / scale < 1e-10:
        assert np.abs(err).max() / scale < 1e-9
    else:
        assert np.abs(err - pred).max() <= 0.03 * np.abs(pred).max()
    r = A @ x[0] - b
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-6


def test_batch_equals_single_systems(O, W):
    ip, ix, vals, bs = W.scenario_batch(30, 3)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    x, info, xk, _ = O.dense_batch(n, ip, ix, vals, eps, bs, keep_xk=True)
    c = O.weights(eps)
    for s in range(3):
        parts = []
        for k, e in enumerate(eps):
            xs_k, inf = O.dense_system(n, ip, ix, vals[s], e, bs[s])
            assert inf == info[s, k] == 0
            assert np.array_equal(xs_k, xk[s, k])
            parts.append(xs_k)
        assert np.array_equal(O.combine(c, np.stack(parts)), x[s])


def test_spectral_radius_helper_vs_lapack(O, W):
    """rho(A^{-1} D) by power iteration against LAPACK eigenvalues (diagnostics helper)."""
    for N, scen in ((14, 0), (30, 1)):
        n, ip, ix, v, b = _jac(W, N, scen)
        A = W.to_dense(n, ip, ix, v)
        d = np.linspace(0.5, 1.0, n)
        rho = O.spectral_radius_AinvD(A, d, iters=600)
        ref = np.abs(np.linalg.eigvals(np.linalg.solve(A, np.diag(d)))).max()
        assert rho == pytest.approx(ref, rel=2e-2)
