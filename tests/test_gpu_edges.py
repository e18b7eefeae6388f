"""Degenerate and maximum cases of the method on every path, bitwise against the oracle:
one node (K = 1: no combination, x_hat = x_1), the maximum K = 16, the smallest systems
(n = 1 and n = 2, including a structurally zero diagonal that only the perturbation fills),
and a batch of one Jacobian; K outside 1..16 is refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PATHS = ["dense", "sparse_batched", "sparse_grouped", "sparse_lds", "sparse_levels", "sparse_steps"]


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


def _oracle(O, n, ip, ix, vals, eps, bs, path):
    sym = O.symbolic(n, ip, ix)
    if path == "dense":
        return O.dense_batch(n, ip, ix, vals, eps, bs, perm=sym.perm)[:2]
    return O.sparse_batch(n, ip, ix, vals, sym, eps, bs)[:2]


def _run(psp, dev, ip, ix, vals, eps, bs, path):
    plan = psp.Plan(ip, ix)
    x, info = psp.solve_batched(plan, torch.from_numpy(vals).to(dev), eps, torch.from_numpy(bs).to(dev), path=path)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("K", [1, 16])
def test_node_count_extremes(psp, O, W, dev, path, K):
    ip, ix, vals, bs = W.scenario_batch(30, 3)
    n = len(ip) - 1
    eps = 1e-3 * 0.5 ** np.arange(K)
    print(f"[gpu edges] K={K} {path}", flush=True)
    xg, ig = _run(psp, dev, ip, ix, vals, eps, bs, path)
    xo, io = _oracle(O, n, ip, ix, vals, eps, bs, path)
    assert np.array_equal(ig, io)
    assert np.array_equal(xg, xo)


@pytest.mark.parametrize("path", PATHS)
def test_smallest_systems_and_single_jacobian(psp, O, dev, path):
    # n = 1: a single unknown; n = 2 with a zero (2,2) entry absent from the pattern
    cases = [
        (np.array([0, 1], np.int32), np.array([0], np.int32), np.array([[4.0]]), np.array([[2.0]])),
        (np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32), np.array([[2.0, 1.0, 3.0]]),
         np.array([[1.0, -1.0]])),
    ]
    eps = np.array([1e-2, 5e-3, 2.5e-3])
    for ip, ix, vals, bs in cases:
        n = len(ip) - 1
        xg, ig = _run(psp, dev, ip, ix, vals, eps, bs, path)
        xo, io = _oracle(O, n, ip, ix, vals, eps, bs, path)
        assert np.array_equal(ig, io), (n, ig, io)
        assert np.array_equal(xg, xo), (n, xg, xo)
    # n = 2 case: A = [[2, 1], [3, 0]], exact solution of A x = (1, -1) is (-1/3, 5/3); the
    # combination of three nodes recovers it to O(prod eps) ~ 1e-7
    assert np.allclose(xg[0], [-1.0 / 3.0, 5.0 / 3.0], rtol=1e-5)


def test_node_count_outside_range_is_refused(psp, dev):
    ip = np.array([0, 1], np.int32)
    ix = np.array([0], np.int32)
    plan = psp.Plan(ip, ix)
    v = torch.ones((1, 1), dtype=torch.float64, device=dev)
    b = torch.ones((1, 1), dtype=torch.float64, device=dev)
    for eps in (np.zeros(0), 1e-3 * 0.5 ** np.arange(17)):
        with pytest.raises(psp.PSPError) as e:
            psp.solve_batched(plan, v, eps, b)
        assert e.value.status == psp.PSP_E_INVALID
