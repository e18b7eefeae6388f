"""Pins for the oracle's end-to-end dense assembly: the permuted, perturbed system
P (A + eps D) P^T of Sec. III-A (the perturbed systems behind eqs. xap / xam) as
oracle_dense_system / oracle_dense_batch build it from CSR, with a symmetric
permutation and a non-identity diagonal D.

Each system is formed here a second way, by plain numpy indexing of the dense
matrix: A[perm][:, perm], then the diagonal plus fl(eps * d[perm]).  The oracle's
pivot-free LU and substitutions (pinned on their own in test_oracle_dense.py) then
have to reproduce the same bits, and so does the sparse oracle on the fill pattern
(pinned against the dense one on an explicitly permuted matrix).  A slip in the
permutation (inverted, or applied to one side only) or in the indexing of d (by
position instead of by original index) changes the system and fails here.
"""
import numpy as np
import pytest


def _explicit_system(n, ip, ix, vals, perm, eps, d):
    A = np.zeros((n, n))
    for i in range(n):
        for e in range(ip[i], ip[i + 1]):
            A[i, ix[e]] = vals[e]
    P = A[np.asarray(perm)][:, np.asarray(perm)]
    dd = np.ones(n) if d is None else np.asarray(d)[np.asarray(perm)]
    P[np.arange(n), np.arange(n)] = P[np.arange(n), np.arange(n)] + eps * dd   # fl(a + fl(eps d))
    return P


def _explicit_solve(O, P, perm, b):
    LU, info = O.lu_nopiv(P)
    if info != 0:
        return None, info, LU
    z = O.solve_lu(LU, b[np.asarray(perm)])
    x = np.empty_like(z)
    x[np.asarray(perm)] = z          # x = P^T z
    return x, info, LU


def _case(W, N, seed_d):
    ip, ix, vals, bs = W.scenario_batch(N, 3)
    n = len(ip) - 1
    d = np.random.default_rng(seed_d).standard_normal(n)
    d = d / np.abs(d).max()
    return n, ip, ix, vals, bs, d


@pytest.mark.parametrize("N", [14, 300])
@pytest.mark.parametrize("gauss_d", [False, True])
def test_dense_system_matches_explicit_permuted_system(O, W, N, gauss_d):
    n, ip, ix, vals, bs, dg = _case(W, N, 1311)
    d = dg if gauss_d else None
    sym = O.symbolic(n, ip, ix)
    assert not np.array_equal(sym.perm, np.arange(n)), "the ordering must permute for this pin to bite"
    eps_set = W.config_eps("small") if N == 14 else W.geometric_eps(1e-3, 5)
    for s in range(2):
        for eps in eps_set[:2]:
            P = _explicit_system(n, ip, ix, vals[s], sym.perm, eps, d)
            xe, info_e, LUe = _explicit_solve(O, P, sym.perm, bs[s])
            x, info, lu = O.dense_system(n, ip, ix, vals[s], eps, bs[s], perm=sym.perm, d=d, return_lu=True)
            assert info == info_e == 0
            assert np.array_equal(lu, LUe), "factors differ from those of the explicitly permuted system"
            assert np.array_equal(x, xe), "solution differs from that of the explicitly permuted system"
            # and the sparse oracle on the fill pattern reproduces the same bits
            xs, info_s = O.sparse_system(n, ip, ix, vals[s], sym, eps, bs[s], d=d)
            assert info_s == 0
            assert np.array_equal(xs, x)


@pytest.mark.parametrize("N", [14, 300])
@pytest.mark.parametrize("gauss_d", [False, True])
def test_dense_batch_matches_explicit_systems(O, W, N, gauss_d):
    n, ip, ix, vals, bs, dg = _case(W, N, 2718)
    d = dg if gauss_d else None
    sym = O.symbolic(n, ip, ix)
    eps = W.config_eps("small") if N == 14 else W.geometric_eps(1e-3, 5)
    x, info, xk, _ = O.dense_batch(n, ip, ix, vals, eps, bs, perm=sym.perm, d=d, keep_xk=True)
    assert not info.any()
    c = O.weights(eps)
    for s in range(vals.shape[0]):
        per = []
        for k, e in enumerate(eps):
            xe, info_e, _ = _explicit_solve(O, _explicit_system(n, ip, ix, vals[s], sym.perm, e, d), sym.perm, bs[s])
            assert info_e == 0
            assert np.array_equal(xk[s, k], xe), f"system ({s}, {k}) differs from the explicit one"
            per.append(xe)
        assert np.array_equal(x[s], O.combine(c, np.stack(per)))
    xsb, info_sb, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs, d=d)
    assert np.array_equal(info_sb, info) and np.array_equal(xsb, x)


def test_planted_assembly_slips_fail(O, W):
    """The explicit construction distinguishes the two plausible slips."""
    n, ip, ix, vals, bs, dg = _case(W, 14, 99)
    sym = O.symbolic(n, ip, ix)
    perm = np.asarray(sym.perm)
    eps = 1e-2
    good = _explicit_system(n, ip, ix, vals[0], perm, eps, dg)
    x, _ = O.dense_system(n, ip, ix, vals[0], eps, bs[0], perm=perm, d=dg)
    # permutation applied the other way round
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n)
    xw, _, _ = _explicit_solve(O, _explicit_system(n, ip, ix, vals[0], inv, eps, dg), inv, bs[0])
    assert not np.array_equal(xw, x)
    # d indexed by position instead of by original index
    bad = good.copy()
    bad[np.arange(n), np.arange(n)] -= eps * dg[perm]
    bad[np.arange(n), np.arange(n)] += eps * dg
    xb, _, _ = _explicit_solve(O, bad, perm, bs[0])
    assert not np.array_equal(xb, x)
