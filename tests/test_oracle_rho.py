"""Pins of the oracle's power iteration for rho(A^{-1} D) (the radius of Sec. II-B that the
perturbation size is chosen from): closed-form spectra, a complex dominant pair, a
non-identity D, and LAPACK's eigenvalues on a power-flow Jacobian."""
import numpy as np

from oracle import oracle as O
from paper_2311_11833_amd import workloads as W


def _orth(n, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return q


def test_symmetric_spectrum():
    n = 12
    a = np.array([0.1, 0.5] + list(np.linspace(1.0, 3.0, n - 2)))
    Q = _orth(n, 1)
    A = Q @ np.diag(a) @ Q.T
    p = 1e-8
    rho = O.power_rho(A, None, p, np.random.default_rng(2).standard_normal(n), 40)
    assert abs(rho - 1 / (0.1 + p)) <= 1e-6 * 10


def test_complex_dominant_pair():
    """A^{-1} acts on a plane as r times a rotation: every step grows that component by r."""
    n, r, th = 8, 7.0, 0.9
    Minv = np.zeros((n, n))
    Minv[:2, :2] = r * np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    Minv[2:, 2:] = np.diag(np.linspace(0.5, 2.0, n - 2))
    T = _orth(n, 3)          # orthogonal, so the plane's growth is exactly r in the 2-norm
    A = np.linalg.inv(T @ Minv @ T.T)
    rho = O.power_rho(A, None, 1e-12, np.random.default_rng(4).standard_normal(n), 60)
    assert abs(rho - r) <= 1e-6 * r


def test_diagonal_d():
    d = np.array([0.3, -2.0, 1.5, 0.7])
    p = 1e-3
    rho = O.power_rho(np.eye(4), d, p, np.ones(4), 60)
    want = np.max(np.abs(d / (1 + p * d)))
    assert abs(rho - want) <= 1e-9 * want


def test_power_flow_jacobian_against_eigenvalues():
    ip, ix, vals, _ = W.scenario_batch(30, 2)
    n = len(ip) - 1
    for s in range(2):
        A = W.to_dense(n, ip, ix, vals[s])
        ev = np.abs(np.linalg.eigvals(np.linalg.inv(A))).max()
        rho = O.power_rho(A, None, 1e-10, np.random.default_rng(s).standard_normal(n), 400)
        assert abs(rho - ev) <= 0.05 * ev


def test_norm2():
    assert O.norm2(np.array([3.0, 4.0])) == 5.0
    x = np.random.default_rng(5).standard_normal(1000)
    assert abs(O.norm2(x) - np.linalg.norm(x)) <= 1e-14 * np.linalg.norm(x)


def test_pivot_free_iteration_tracks_the_pivoted_one():
    """The library's sequence (pivot-free perturbed solves) stays within the pivot-free
    solve's accuracy of the pivoted iteration, with D = I and with a Gaussian D."""
    for N, S in ((14, 3), (300, 2)):
        ip, ix, vals, _ = W.scenario_batch(N, S)
        n = len(ip) - 1
        sym = O.symbolic(n, ip, ix)
        dg = np.random.default_rng(1311).standard_normal(n)
        dg /= np.abs(dg).max()
        for s in range(S):
            A = W.to_dense(n, ip, ix, vals[s])
            v0 = np.random.default_rng(s).standard_normal(n)
            for d in (None, dg):
                a = O.power_rho(A, d, 1e-8, v0, 24)
                b = O.power_rho_pivot_free(n, ip, ix, vals[s], sym, d, 1e-8, v0, 24)
                assert abs(a - b) <= 1e-6 * a, (N, s, d is None)
