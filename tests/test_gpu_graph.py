"""The fused batched call captured in a HIP graph (torch.cuda.graph over the library's
stream): every replay, with eager work and synchronisations between replays, must
equal the eager result bit for bit, on both numeric paths."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("path,N,count", [("dense", 30, 8), ("sparse", 300, 64), ("sparse", 30, 4), ("sparse_steps", 300, 300)])
def test_graph_replays_match_eager(dev, W, path, N, count):
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(N, count)
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    v = torch.from_numpy(vals).to(dev)
    b = torch.from_numpy(bs).to(dev)
    x_eager, info_eager = psp.solve_batched(plan, v, eps, b, path=path)     # also uploads the plan
    torch.cuda.synchronize()
    ref = x_eager.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        psp.solve_batched(plan, v, eps, b, path=path)                       # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        x_g, info_g = psp.solve_batched(plan, v, eps, b, path=path)
    for rep in range(3):
        x_g.zero_()
        psp.solve_batched(plan, v, eps, b * 2.0, path=path)                   # eager work in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x_g.cpu().numpy(), ref), rep
        assert np.array_equal(info_g.cpu().numpy(), info_eager.cpu().numpy())


@pytest.mark.parametrize("path,N,count", [("sparse", 300, 64), ("sparse_steps", 300, 512), ("dense", 30, 8)])
def test_fresh_plan_first_call_captured(dev, W, O, path, N, count):
    """Only psp_plan_upload precedes the capture: the plan's first numeric call runs inside the
    graph (no allocation, copy or synchronisation in it) and every replay equals the oracle."""
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(N, count)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    plan.upload(dev)
    v = torch.from_numpy(vals).to(dev)
    b = torch.from_numpy(bs).to(dev)
    ws = torch.empty(plan.workspace_bytes(path, count, len(eps), 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        x_g, info_g = psp.solve_batched(plan, v, eps, b, path=path, workspace=ws)
    sym = O.symbolic(n, ip, ix)
    if path == "dense":
        xo, io, _, _ = O.dense_batch(n, ip, ix, vals, eps, bs, perm=sym.perm)
    else:
        xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    for rep in range(3):
        x_g.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(info_g.cpu().numpy(), io), rep
        assert np.array_equal(x_g.cpu().numpy(), xo), rep
