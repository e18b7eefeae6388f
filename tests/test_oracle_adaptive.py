"""Pins of the oracle's a-posteriori error estimate and node-scale rule.

The estimate rests on the expansion of Sec. II-B, x(eps) = sum_j (-eps)^j M^j x*
with M = A^{-1} D: divided differences of the perturbed solutions over the
nodes recover the series' coefficients, and the combination's leading error
is -(prod eps_k) M^K x* (Theorem 1, general nodes).  None of the checks below
re-evaluates the oracle's own formula:

* divided differences against their closed form for a diagonal system
  (1/(a + eps) has f[eps_0..eps_j] = (-1)^j / prod_l (a + eps_l));
* the estimate against the exact error of a diagonal system (the error of the
  combination has a closed form there), and against LAPACK's pivoted solve on
  power-flow Jacobians whose error is dominated by truncation;
* the node scale against a numerical minimiser of the stated error model;
* the whole rule on the 512 seeded scenarios of the 300-bus network against
  LAPACK (the target of 1e-9 relative is met on at least 505 of them).
"""
import math

import numpy as np
import pytest


def _diag_xk(a, b, eps):
    return np.stack([b / (a + e) for e in eps])


def test_divided_differences_closed_form(O):
    rng = np.random.default_rng(5)
    a = rng.uniform(1.0, 3.0, 40)
    b = rng.standard_normal(40)
    eps = np.array([0.4, -0.3, 0.2, 0.1, -0.05])
    xk = _diag_xk(a, b, eps)
    for j in range(len(eps)):
        f = O.divided_difference(j, eps, xk)
        ref = (-1) ** j * b / np.prod([a + eps[l] for l in range(j + 1)], axis=0)
        assert np.abs(f - ref).max() <= 1e-12 * np.abs(ref).max(), j


def test_estimate_matches_exact_error_of_diagonal_system(O):
    # one small diagonal entry dominates M = A^{-1}: the leading error term is
    # -(prod eps) b_0 / a_0^{K+1}, and est sees it through m_{K-1}^2 / m_{K-2}
    rng = np.random.default_rng(6)
    a = rng.uniform(1.0, 2.0, 30)
    a[7] = 0.02
    b = rng.standard_normal(30)
    b[7] = 0.5
    for K in (3, 4, 5):
        eps = 5e-4 * 0.5 ** np.arange(K)      # eps / a_0 <= 0.025: truncation far above rounding
        xk = _diag_xk(a, b, eps)
        c = O.weights(eps)
        x = O.combine(c, xk)
        # exact error of the combination: sum_k c_k b/(a+eps_k) - b/a written as a single fraction
        # per entry, evaluated in exact rationals
        from fractions import Fraction as Fr
        err = max(abs(sum(Fr(c[k]) * Fr(b[i]) / (Fr(a[i]) + Fr(eps[k])) for k in range(K)) - Fr(b[i]) / Fr(a[i]))
                  for i in range(30))
        true_rel = float(err) / np.abs(b / a).max()
        est, rho = O.error_estimate(eps, xk, x)
        assert abs(rho - 1 / 0.02) <= 0.05 / 0.02, (K, rho)
        assert 0.85 <= est / true_rel <= 1.15, (K, est, true_rel)


def test_estimate_tracks_pivoted_error_on_power_flow_jacobians(O, W):
    ip, ix, vals, bs = W.scenario_batch(300, 64)
    n = len(ip) - 1
    sym = O.symbolic(n, ip, ix)
    eps = W.config_eps("n601")
    x, info, xk, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs, keep_xk=True)
    checked = 0
    for s in range(64):
        xs = np.linalg.solve(W.to_dense(n, ip, ix, vals[s]), bs[s])
        true = np.abs(x[s] - xs).max() / np.abs(xs).max()
        est, _ = O.error_estimate(eps, xk[s], x[s])
        if 1e-9 <= true <= 1e-3:          # truncation dominates, inside the convergence radius
            assert 0.7 <= est / true <= 1.4, (s, est, true)
            checked += 1
        elif true < 1e-11:
            assert est < 1e-9, (s, est, true)
    assert checked >= 3


def test_scale_minimises_the_error_model(O):
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(8)
    u = 2.0 ** -53
    cases = 0
    for _ in range(300):
        K = int(rng.integers(3, 9))
        eps = 10.0 ** rng.uniform(-5, -2) * 0.5 ** np.arange(K)
        est = 10.0 ** rng.uniform(-9, 1)
        rho = 10.0 ** rng.uniform(0, 5)
        j = O.scale_exponent(eps, est, rho)
        a = est if est < 1e-2 else np.prod(np.abs(eps)) * rho ** K
        bcoef = 50 * u / np.abs(eps).max()
        model = lambda ls: a * math.exp(K * ls) + bcoef * math.exp(-ls)   # noqa: E731
        opt = minimize_scalar(model, bounds=(-200.0, 5.0), method="bounded", options={"xatol": 1e-12})
        s_star = math.exp(opt.x)
        s = 2.0 ** -j
        if 1 <= j < 60 and s_star < 0.5:
            assert s <= s_star * (1 + 1e-6) and s_star < 2 * s * (1 + 1e-6), (K, est, rho, j, s_star)
            cases += 1
        elif s_star >= 0.5:
            assert j == 1
    assert cases > 200
    assert O.scale_exponent(np.array([1e-3, 5e-4, 2.5e-4]), float("nan"), 1.0) == 10


def test_rule_meets_the_target_on_the_300_bus_scenarios(O, W):
    ip, ix, vals, bs = W.scenario_batch(300, 512)
    n = len(ip) - 1
    sym = O.symbolic(n, ip, ix)
    eps = W.config_eps("n601")
    x, info, est, scale = O.adaptive_batch(n, ip, ix, vals, sym, eps, bs, 1e-10)
    xs = np.stack([np.linalg.solve(W.to_dense(n, ip, ix, vals[s]), bs[s]) for s in range(512)])
    err = np.abs(x - xs).max(axis=1) / np.abs(xs).max(axis=1)
    x0, _, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    err0 = np.abs(x0 - xs).max(axis=1) / np.abs(xs).max(axis=1)
    assert int((err0 > 1e-9).sum()) > 50          # the fixed nodes miss on the tail
    assert int((err > 1e-9).sum()) <= 7
    assert err.max() < 1e-8
    assert np.all(info == 0)
    # kept Jacobians are exactly the first solve; rescaled ones used powers of two below 1
    kept = scale == 1.0
    assert np.array_equal(x[kept], x0[kept])
    assert np.all(np.log2(scale[~kept]) == np.round(np.log2(scale[~kept])))
    assert np.all(est[kept] <= 1e-10)


def test_large_case_nodes_meet_the_target(O, W):
    """The 10,000-bus Jacobian (n = 20,001) with its node set +-1e-5, +-2e-5: the recovered
    solutions of 32 right-hand sides are within 1e-9 of SuperLU's partially pivoted solve
    (itself within 1e-12 of the solution refined with residuals in extended precision); the
    geometric nodes 1e-5 * 2^-k, whose combination amplifies the rounding of the pivot-free
    solves 24 times more, miss it."""
    sps = pytest.importorskip("scipy.sparse")
    spla = pytest.importorskip("scipy.sparse.linalg")
    from paper_2311_11833_amd.workloads import make_network, make_state, jacobian, seed_state
    net = make_network(10000)
    vm, va, p = make_state(10000, seed_state(10000, 0))
    J = jacobian(net, vm, va, p)
    n = J.n
    A = sps.csr_matrix((J.data, J.indices, J.indptr), shape=(n, n))
    B = np.random.default_rng(7).standard_normal((n, 32))
    lu = spla.splu(A.tocsc(), permc_spec="COLAMD")
    xs = lu.solve(B)
    xr = xs.copy()
    for _ in range(2):
        r = B.astype(np.longdouble) - A.astype(np.longdouble) @ xr.astype(np.longdouble)
        xr = xr + lu.solve(np.asarray(r, dtype=np.float64))
    assert (np.abs(xs - xr).max(axis=0) / np.abs(xr).max(axis=0)).max() < 1e-12
    sym = O.symbolic(n, J.indptr, J.indices)
    errs = {}
    for name, eps in (("symmetric", W.large_eps()), ("geometric", W.geometric_eps(1e-5, 4))):
        x, info, _, _ = O.sparse_batch(n, J.indptr, J.indices, J.data[None], sym, eps, B[None])
        assert np.all(info == 0)
        errs[name] = np.abs(x[0] - xs).max(axis=0) / np.abs(xs).max(axis=0)
    assert errs["symmetric"].max() < 1e-9
    assert (errs["geometric"] > 1e-9).sum() > 5
