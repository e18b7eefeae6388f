"""Uneven batches through psp_solve_group: Jacobians of five networks (61 .. 2709
unknowns) in one call on one stream, each equal to the oracle bit for bit, with the
path chosen per pattern (the autotuner's choice after psp_tune, else the heuristic)."""
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


def test_uneven_group_matches_oracle(psp, O, W, dev):
    eps = W.config_eps("n601")
    counts = {30: 3, 118: 2, 300: 4, 500: 1, 1354: 2}
    items, ref = [], []
    for N, c in counts.items():
        ip, ix, vals, bs = W.scenario_batch(N, c)
        plan = psp.Plan(ip, ix)
        items.append((plan, torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)))
        ref.append((len(ip) - 1, ip, ix, vals, bs))
    print("[gpu group] uneven 5 networks", flush=True)
    # tune the n = 601 item first: its path then comes from the tuner, the others from the heuristic
    psp.tune(items[2][0], items[2][1], eps, items[2][2])
    outs = psp.solve_group(items, eps)
    torch.cuda.synchronize()
    for (x, info), (n, ip, ix, vals, bs) in zip(outs, ref):
        sym = O.symbolic(n, ip, ix)
        xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
        assert np.array_equal(info.cpu().numpy(), io)
        assert np.array_equal(x.cpu().numpy(), xo), n


def test_group_workspace_too_small_is_reported(psp, W, dev):
    eps = W.config_eps("n601")
    ip, ix, vals, bs = W.scenario_batch(30, 2)
    plan = psp.Plan(ip, ix)
    tiny = torch.empty(256, dtype=torch.uint8, device=dev)
    with pytest.raises(psp.PSPError) as e:
        psp.solve_group([(plan, torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev))], eps, workspace=tiny)
    assert e.value.status == psp.PSP_E_NOMEM
