"""Oracle pins for the combination weights (Sec. III-A, Theorem 1, Remark 2, Examples 1-3).

The weights are pinned to the paper's printed examples, to the moment
conditions that define them (Gamma^T beta = e1), and to a library solve of
the Vandermonde system; none of these re-evaluates the oracle's product
formula.
"""
import os
from fractions import Fraction as F
from math import factorial

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    rows = {}
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split(None, 1)
            rows.setdefault(key, []).append(rest[0] if rest else "")
    return rows


def _fracs(s):
    return [F(t) for t in s.split()]


def _symmetric_nodes(m, eps):
    """Nodes +alpha*eps, -alpha*eps for alpha = 1..m (eqs. xap, xam)."""
    nodes = []
    for a in range(1, m + 1):
        nodes += [a * eps, -a * eps]
    return np.array(nodes)


def _beta_from_c(c, m):
    """Fold symmetric weights back onto the averaged solutions x_hat_alpha."""
    beta = []
    for a in range(m):
        cp, cm = c[2 * a], c[2 * a + 1]
        assert cp == pytest.approx(cm, rel=1e-12)  # Remark 1: + and - enter equally
        beta.append(cp + cm)
    return np.array(beta)


def test_example3_beta_m2(O):
    g = _gold("ex3_vandermonde_m2.txt")
    want = _fracs(g["beta"][0])
    beta = _beta_from_c(O.weights(_symmetric_nodes(2, 1e-3)), 2)
    assert np.allclose(beta, [float(w) for w in want], rtol=1e-13, atol=0)


def test_example1_moments_m2(O):
    g = _gold("ex1_m2_combination.txt")
    beta = [float(w) for w in _fracs(g["beta"][0])]
    moments = [float(w) for w in _fracs(g["moments"][0])]
    got = _beta_from_c(O.weights(_symmetric_nodes(2, 2e-3)), 2)
    assert np.allclose(got, beta, rtol=1e-13)
    # coefficient of T_{2j}: sum_alpha beta_alpha alpha^{2j} (eq. avg_hats)
    for j, mj in enumerate(moments):
        s = sum(F(got[a]).limit_denominator(10**6) * (a + 1) ** (2 * j) for a in range(2))
        assert float(s) == pytest.approx(mj, abs=1e-9)


def test_example2_corrected_m3(O):
    g = _gold("ex2_m3_combination.txt")
    x21 = _fracs(g["x21"][0])
    x31 = _fracs(g["x31"][0])
    printed = [x31[a] - F(9, 4) * x21[a] for a in range(3)]
    scale = sum(printed)                    # coefficient of A^{-1} as printed: -5/4
    assert scale == F(-5, 4)
    normalised = [p / scale for p in printed]
    want = _fracs(g["beta"][0])
    assert normalised == want
    got = _beta_from_c(O.weights(_symmetric_nodes(3, 1e-3)), 3)
    assert np.allclose(got, [float(w) for w in want], rtol=1e-12)
    moments = [float(w) for w in _fracs(g["moments"][0])]
    for j, mj in enumerate(moments):
        assert sum(float(want[a]) * (a + 1) ** (2 * j) for a in range(3)) == pytest.approx(mj, abs=1e-12)


def test_gamma3_table_and_library_solve(O):
    g = _gold("gamma3_and_avg_hats.txt")
    G3 = np.array([[float(v) for v in r.split()] for r in g["gamma3"][0].split(";")])
    assert np.array_equal(G3, np.array([[a ** (2 * j) for j in range(3)] for a in (1, 2, 3)], float))
    for line in g["avg"]:
        a, coeffs = line.split(":")
        a = int(a)
        assert [int(v) for v in coeffs.split()] == [a ** (2 * j) for j in range(4)]
    for m in range(1, 6):
        Gm = np.array([[a ** (2 * j) for j in range(m)] for a in range(1, m + 1)], float)
        beta_lib = np.linalg.solve(Gm.T, np.eye(m)[0])       # Remark 2 via LAPACK
        got = _beta_from_c(O.weights(_symmetric_nodes(m, 1e-3)), m)
        assert np.allclose(got, beta_lib, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_closed_form_symmetric_beta(O, m):
    """beta_alpha = 2 (-1)^{alpha+1} (m!)^2 / ((m-alpha)! (m+alpha)!) solves Gamma_m^T beta = e1."""
    want = [2 * (-1) ** (a + 1) * F(factorial(m) ** 2, factorial(m - a) * factorial(m + a)) for a in range(1, m + 1)]
    for j in range(m):
        assert sum(want[a - 1] * a ** (2 * j) for a in range(1, m + 1)) == (1 if j == 0 else 0)
    # leading surviving moment (Theorem 1's O(eps^{2m}) term) = (-1)^{m+1} (m!)^2
    lead = sum(want[a - 1] * a ** (2 * m) for a in range(1, m + 1))
    assert lead == (-1) ** (m + 1) * factorial(m) ** 2
    got = _beta_from_c(O.weights(_symmetric_nodes(m, 1e-3)), m)
    assert np.allclose(got, [float(w) for w in want], rtol=1e-11)


@pytest.mark.parametrize("eps", [
    [1e-2, 5e-3, 2.5e-3],
    [1e-3 * 0.5 ** k for k in range(5)],
    [1e-6 * 0.5 ** k for k in range(4)],
    [3e-3, -1e-3, 7e-4, -2.2e-3, 1.5e-3, 9e-4],
])
def test_moment_conditions_exact(O, eps):
    """sum_k c_k eps_k^j = delta_{j0} (j < K) and sum_k c_k eps_k^K = (-1)^{K+1} prod eps_k."""
    c = O.weights(eps)
    K = len(eps)
    Fe = [F(e) for e in eps]
    Fc = [F(v) for v in c]
    scale = max(abs(v) for v in Fc)
    for j in range(K):
        s = sum(Fc[k] * Fe[k] ** j for k in range(K))
        ref = max(abs(Fc[k] * Fe[k] ** j) for k in range(K))
        assert abs(s - (1 if j == 0 else 0)) <= 64 * F(2) ** -52 * max(ref, scale if j == 0 else ref)
    prod = F(1)
    for e in Fe:
        prod *= e
    sK = sum(Fc[k] * Fe[k] ** K for k in range(K))
    assert abs(sK - (-1) ** (K + 1) * prod) <= 1e-12 * abs(prod)


@pytest.mark.parametrize("bad", [[1e-3, 1e-3], [0.0, 1e-3], [float("nan"), 1e-3], [float("inf")], []])
def test_invalid_nodes_rejected(O, bad):
    with pytest.raises(ValueError):
        O.weights(bad)
