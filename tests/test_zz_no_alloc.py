"""psp_solve_batched_noalloc (the entry point for callers that cannot allocate):
through the C ABI, on the step-schedule path with a batch small enough that the
per-system solutions go to the library's static scratch, two calls in a row (the
second with a smaller batch, reusing what the first left in the scratch), each
bitwise equal to psp_solve_batched on the same inputs; a batch that needs more
than the scratch holds is refused before any launch."""
import ctypes as C

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


def _noalloc(psp, plan, vals, eps, b):
    batch = vals.shape[0]
    e = np.ascontiguousarray(eps, dtype=np.float64)
    x = torch.full_like(b, float("nan"))
    info = torch.full((batch, len(e)), -7, dtype=torch.int32, device=vals.device)
    st = psp.lib().psp_solve_batched_noalloc(plan.handle, batch, psp._dptr(vals), len(e), psp._np_ptr(e), None,
                                             psp._dptr(b), psp._dptr(x), psp._dptr(info), psp._stream(None))
    return st, x, info


def test_noalloc_matches_solve_batched_twice(psp, W, dev):
    eps = W.config_eps("n601")
    ip, ix, vals, bs = W.scenario_batch(300, 200)
    plan = psp.Plan(ip, ix)
    plan.ensure(dev)
    assert plan.info().steps > 0
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    for batch in (200, 37):
        print(f"[gpu noalloc] n=601 batch={batch} K=5", flush=True)
        vv, bb = v[:batch].contiguous(), b[:batch].contiguous()
        st, x, info = _noalloc(psp, plan, vv, eps, bb)
        assert st == psp.PSP_OK, psp.lib().psp_last_error().decode()
        xr, ir = psp.solve_batched(plan, vv, eps, bb, path="sparse_steps")
        torch.cuda.synchronize()
        assert torch.equal(info, ir)
        err = ((x - xr).abs().max() / xr.abs().max()).item()
        assert err <= 1e-12, err
        assert torch.equal(x, xr)


def test_noalloc_refuses_batch_beyond_scratch(psp, W, dev):
    # 300 Jacobians of n = 601 with K = 16 need 300*16*601*8 = 23 MB of per-system solutions
    eps = W.geometric_eps(1e-3, 16)
    ip, ix, vals, bs = W.scenario_batch(300, 1)
    plan = psp.Plan(ip, ix)
    plan.ensure(dev)
    v = torch.from_numpy(np.repeat(vals, 300, axis=0)).to(dev)
    b = torch.from_numpy(np.repeat(bs, 300, axis=0)).to(dev)
    st, _, _ = _noalloc(psp, plan, v, eps, b)
    assert st == psp.PSP_E_UNSUPPORTED
    assert "scratch" in psp.lib().psp_last_error().decode()
