"""Pins of the oracle's error test (Alg. 1 step 5): r = b - A x and the 2-norms.

The residual has a plain definition, so the pins are values worked by hand, an
independent dense evaluation of b - A x, norms with exact Pythagorean values,
and the residual of the pivoted (ground-truth) solution, which must be at the
rounding level."""
import numpy as np


def test_hand_example(O):
    # A = [[2, 1], [0, 3]] in CSR, x = (1, 1), b = (4, 3): r = (1, 0)
    ip = np.array([0, 2, 3], np.int32)
    ix = np.array([0, 1, 1], np.int32)
    va = np.array([2.0, 1.0, 3.0])
    r, rn, bn = O.residual(2, ip, ix, va, np.array([4.0, 3.0]), np.array([1.0, 1.0]))
    assert np.array_equal(r, [1.0, 0.0])
    assert rn[0] == 1.0 and bn[0] == 5.0


def test_pythagorean_norms(O):
    # A = 0 (no entries): r = b; b = (3, 4, 12) has norm 13 exactly, per column
    ip = np.zeros(4, np.int32)
    ix = np.zeros(0, np.int32)
    b = np.array([[3.0, 0.0], [4.0, 5.0], [12.0, 12.0]])
    r, rn, bn = O.residual(3, ip, ix, np.zeros(0), b, np.ones((3, 2)))
    assert np.array_equal(r, b)
    assert np.array_equal(rn, [13.0, 13.0]) and np.array_equal(bn, [13.0, 13.0])


def test_matches_dense_product(O, W):
    ip, ix, vals, bs = W.scenario_batch(30, 1)
    n = len(ip) - 1
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, 3))
    b = rng.standard_normal((n, 3))
    A = W.to_dense(n, ip, ix, vals[0])
    r, rn, bn = O.residual(n, ip, ix, vals[0], b, x)
    ref = b - A @ x
    scale = np.abs(A) @ np.abs(x) + np.abs(b)
    assert np.all(np.abs(r - ref) <= 4 * n * 2.0 ** -53 * scale)
    assert np.allclose(rn, np.linalg.norm(ref, axis=0), rtol=1e-13, atol=0)
    assert np.allclose(bn, np.linalg.norm(b, axis=0), rtol=1e-14, atol=0)


def test_residual_of_pivoted_solution_is_tiny(O, W):
    ip, ix, vals, bs = W.scenario_batch(300, 1)
    n = len(ip) - 1
    A = W.to_dense(n, ip, ix, vals[0])
    x = O.pivoted_solve(A, bs[0])
    _, rn, bn = O.residual(n, ip, ix, vals[0], bs[0], x)
    assert rn[0] / bn[0] < 1e-12
    # and a perturbed right-hand side is detected: r = -delta exactly for x = A^-1 b, b' = b + delta
    d = np.zeros(n)
    d[7] = 1e-3
    _, rn2, _ = O.residual(n, ip, ix, vals[0], bs[0] + d, x)
    assert abs(rn2[0] - 1e-3) < 1e-9
