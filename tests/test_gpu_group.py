"""Uneven batches through the group calls (psp_group_*): Jacobians of five networks (61 ..
2709 unknowns), ordered longest first over the group's stream lanes, each item equal to
the oracle bit for bit, with the path chosen per pattern (the autotuner's choice after
psp_tune, else the heuristic); the same work captured into one HIP graph replays to the
same bits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _items(psp, W, dev, counts):
    items, ref = [], []
    for N, c in counts.items():
        ip, ix, vals, bs = W.scenario_batch(N, c)
        plan = psp.Plan(ip, ix)
        items.append((plan, torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)))
        ref.append((len(ip) - 1, ip, ix, vals, bs))
    return items, ref


def _check(O, outs, ref, eps):
    for (x, info), (n, ip, ix, vals, bs) in zip(outs, ref):
        sym = O.symbolic(n, ip, ix)
        xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
        assert np.array_equal(info.cpu().numpy(), io), n
        assert np.array_equal(x.cpu().numpy(), xo), n


def test_uneven_group_matches_oracle(psp, O, W, dev):
    eps = W.config_eps("n601")
    items, ref = _items(psp, W, dev, {30: 3, 118: 2, 300: 4, 500: 1, 1354: 2})
    print("[gpu group] uneven 5 networks", flush=True)
    # tune the n = 601 item first: its path then comes from the tuner, the others from the heuristic
    psp.tune(items[2][0], items[2][1], eps, items[2][2])
    outs = psp.solve_group(items, eps)
    torch.cuda.synchronize()
    _check(O, outs, ref, eps)


def test_group_capture_replays_match_oracle(psp, O, W, dev):
    """Fresh plans (uploaded, never run): the group's first execution is the capture itself."""
    eps = W.config_eps("n601")
    items, ref = _items(psp, W, dev, {30: 5, 118: 3, 300: 6, 500: 2, 1354: 1})
    print("[gpu group] capture of 5 networks", flush=True)
    g = psp.Group([(p, v.shape[0]) for p, v, _ in items], eps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph, outs = g.capture([(v, b) for _, v, b in items], stream=s)
    for rep in range(3):
        for x, info in outs:
            x.fill_(float("nan"))
            info.fill_(-7)
        # eager work in between: the same group run on other outputs
        g.run([(v, b * 2.0) for _, v, b in items])
        torch.cuda.synchronize()
        g.replay(graph, stream=s)
        s.synchronize()
        _check(O, outs, ref, eps)


def test_group_workspace_too_small_is_reported(psp, W, dev):
    import ctypes as C
    eps = W.config_eps("n601")
    ip, ix, vals, bs = W.scenario_batch(30, 2)
    plan = psp.Plan(ip, ix)
    g = psp.Group([(plan, 2)], eps)
    tasks, _, _ = g.outputs([(torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev))])
    tiny = torch.empty(256, dtype=torch.uint8, device=dev)
    st = psp.lib().psp_group_run(g._h, C.byref(tasks), psp._dptr(tiny), 256, psp._stream(None))
    assert st == psp.PSP_E_NOMEM


def test_group_error_test_matches_oracle_and_replays(psp, O, W, dev):
    """The uneven group with the error test on every item (psp_group_run_adaptive: the step
    schedule for n <= 1,001, the dense-trailing-block path for 2,709): x, info, est and scale
    equal the oracle's adaptive solve; the captured graph replays to the same bits."""
    eps = W.config_eps("n601")
    items, ref = _items(psp, W, dev, {30: 4, 118: 3, 300: 20, 500: 9, 1354: 14})
    g = psp.Group([(p, v.shape[0]) for p, v, _ in items], eps)
    gin = [(v, b) for _, v, b in items]
    print("[gpu group] error test, eager", flush=True)
    outs = g.run_adaptive(gin, tol=1e-10)
    torch.cuda.synchronize()
    for (x, info, est, scale), (n, ip, ix, vals, bs) in zip(outs, ref):
        sym = O.symbolic(n, ip, ix)
        xo, io, eo, so = O.adaptive_batch(n, ip, ix, vals, sym, eps, bs, 1e-10)
        assert np.array_equal(scale.cpu().numpy(), so), n
        assert np.array_equal(info.cpu().numpy(), io), n
        assert np.array_equal(est.cpu().numpy(), eo, equal_nan=True), n
        assert np.array_equal(x.cpu().numpy(), xo, equal_nan=True), n
    print("[gpu group] error test, graph", flush=True)
    graph, gouts = g.capture_adaptive(gin, tol=1e-10)
    for _ in range(3):
        g.replay(graph)
        torch.cuda.synchronize()
        for a, b in zip(outs, gouts):
            for u, v in zip(a, b):
                assert torch.equal(u.nan_to_num(), v.nan_to_num())
