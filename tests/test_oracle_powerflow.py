"""Pins of the power-flow oracle (Newton loop of Sec. IV) against facts fixed
independently of its own formulas: branch currents, conservation of power,
finite differences, a known root, and LAPACK in place of the perturbed solve."""
import numpy as np
import pytest

from oracle import powerflow as PF
from paper_2311_11833_amd import workloads as W

EPS = W.geometric_eps(1e-3, 5)


def _args(c):
    return (c.y_indptr, c.y_indices, c.g, c.b, c.pv)


def _random_state(c, seed):
    rng = np.random.default_rng(seed)
    N = c.N
    return np.concatenate([rng.uniform(-0.3, 0.3, N), rng.uniform(0.9, 1.1, N), [rng.uniform(-1, 1)]])


def _branch_injections(net, x):
    """S_i = V_i conj(I_i) with I_i the sum of the series currents leaving bus i, from the branch list."""
    N = net.N
    V = x[N:2 * N] * np.exp(1j * x[:N])
    I_l = (V[net.fbus] - V[net.tbus]) / (net.r + 1j * net.x)
    I = np.zeros(N, complex)
    np.add.at(I, net.fbus, I_l)
    np.add.at(I, net.tbus, -I_l)
    return V * np.conj(I), I_l


@pytest.mark.parametrize("N", [14, 300])
def test_injections_equal_branch_current_form(N):
    c = W.pf_case(N)
    for seed in range(3):
        x = _random_state(c, seed)
        P, Q = PF.injections(c.y_indptr, c.y_indices, c.g, c.b, x)
        S, _ = _branch_injections(c.net, x)
        scale = np.abs(S).max()
        assert np.abs(P - S.real).max() <= 1e-12 * scale
        assert np.abs(Q - S.imag).max() <= 1e-12 * scale


def test_injections_conserve_power():
    """With series branches only, sum P = sum r|I|^2 and sum Q = sum x|I|^2 (losses)."""
    c = W.pf_case(300)
    x = _random_state(c, 7)
    P, Q = PF.injections(c.y_indptr, c.y_indices, c.g, c.b, x)
    _, I_l = _branch_injections(c.net, x)
    i2 = np.abs(I_l) ** 2
    assert abs(P.sum() - np.sum(c.net.r * i2)) <= 1e-10 * np.sum(c.net.r * i2)
    assert abs(Q.sum() - np.sum(c.net.x * i2)) <= 1e-10 * np.sum(c.net.x * i2)


def test_jacobian_equals_finite_differences():
    c = W.pf_case(14)
    sc = W.pf_scenarios(c, 2)
    n = c.n
    for s in range(2):
        x = _random_state(c, 11 + s)
        J = PF.jacobian_values(*_args(c), x, sc.part[s], c.indptr, c.indices)
        Jd = W.to_dense(n, c.indptr, c.indices, J)
        h = 1e-6
        Jfd = np.zeros((n, n))
        for k in range(n):
            e = np.zeros(n)
            e[k] = h
            Jfd[:, k] = (PF.mismatch(*_args(c), x + e, sc.spec[s], sc.part[s])
                         - PF.mismatch(*_args(c), x - e, sc.spec[s], sc.part[s])) / (2 * h)
        assert np.abs(Jd - Jfd).max() <= 1e-7 * np.abs(Jd).max()
        # entries outside the pattern have zero derivative
        mask = W.to_dense(n, c.indptr, c.indices, np.ones(len(c.indices))) == 0
        assert np.abs(Jfd[mask]).max() <= 1e-8


def test_jacobian_pq_rows_match_the_workload_jacobian():
    """On PQ rows the Newton Jacobian is the workload's distributed-slack Jacobian."""
    c = W.pf_case(30)
    sc = W.pf_scenarios(c, 1)
    x = _random_state(c, 3)
    N = c.N
    J = PF.jacobian_values(*_args(c), x, sc.part[0], c.indptr, c.indices)
    ref = W.jacobian(c.net, x[N:2 * N], x[:N], sc.part[0])
    assert np.array_equal(ref.indptr, c.indptr) and np.array_equal(ref.indices, c.indices)
    rows = np.repeat(np.arange(c.n), np.diff(c.indptr))
    keep = ~((rows >= N) & (rows < 2 * N) & (c.pv[np.clip(rows - N, 0, N - 1)] != 0))
    assert np.abs(J[keep] - ref.data[keep]).max() <= 1e-12 * np.abs(ref.data).max()


@pytest.mark.parametrize("N", [14, 300])
def test_target_is_a_root(N):
    c = W.pf_case(N)
    sc = W.pf_scenarios(c, 4)
    for s in range(4):
        F = PF.mismatch(*_args(c), sc.x_target[s], sc.spec[s], sc.part[s])
        assert np.abs(F).max() <= 1e-12 * max(1.0, np.abs(sc.spec[s]).max())


def test_newton_converges_quadratically_to_the_target():
    c = W.pf_case(300)
    sc = W.pf_scenarios(c, 4)
    x, iters, status, fnorm, hist = PF.newton(*_args(c), c.indptr, c.indices, sc.x0, sc.spec, sc.part, EPS,
                                              tol=1e-9, max_iter=10)
    assert np.all(status == PF.CONVERGED)
    assert np.all(iters <= 8) and np.all(fnorm <= 1e-9)
    # the loop stops at max|F| <= 1e-9, so x - x* ~ J^-1 F is of order ||J^-1|| 1e-9
    assert np.abs(x - sc.x_target).max() <= 1e-8
    for h in hist:
        # once close, each step squares the mismatch (up to a modest constant)
        tail = [v for v in h if v < 1e-2]
        for a, b in zip(tail, tail[1:]):
            assert b <= max(100 * a * a, 1e-12)


def test_newton_matches_a_pivoted_newton_loop():
    """The same loop with LAPACK's pivoted solve reaches the same state."""
    c = W.pf_case(118)
    sc = W.pf_scenarios(c, 2)
    x, iters, status, _, _ = PF.newton(*_args(c), c.indptr, c.indices, sc.x0, sc.spec, sc.part, EPS)
    for s in range(2):
        xs = sc.x0[s].copy()
        for _ in range(10):
            F = PF.mismatch(*_args(c), xs, sc.spec[s], sc.part[s])
            if np.abs(F).max() <= 1e-9:
                break
            J = W.to_dense(c.n, c.indptr, c.indices,
                           PF.jacobian_values(*_args(c), xs, sc.part[s], c.indptr, c.indices))
            xs = xs - np.linalg.solve(J, F)
        assert np.abs(x[s] - xs).max() <= 1e-10


def test_newton_status_codes():
    c = W.pf_case(14)
    sc = W.pf_scenarios(c, 2)
    _, iters, status, _, hist = PF.newton(*_args(c), c.indptr, c.indices, sc.x0, sc.spec, sc.part, EPS,
                                          max_iter=1)
    assert np.all(status == PF.MAXITER) and np.all(iters == 1) and all(len(h) == 2 for h in hist)
    x0 = sc.x0.copy()
    x0[0, c.N + 3] = np.nan
    _, iters, status, fnorm, _ = PF.newton(*_args(c), c.indptr, c.indices, x0, sc.spec, sc.part, EPS)
    assert status[0] == PF.DIVERGED and iters[0] == 0 and np.isnan(fnorm[0])
    assert status[1] == PF.CONVERGED
    # already at the root: no update
    _, iters, status, _, _ = PF.newton(*_args(c), c.indptr, c.indices, sc.x_target, sc.spec, sc.part, EPS)
    assert np.all(status == PF.CONVERGED) and np.all(iters == 0)
