"""The autotuner (psp_tune): every launch choice it searches returns the oracle's bits, its
choice is recorded in the tuning cache file, and a fresh process finds the choice there and
uses it for PSP_PATH_AUTO without tuning again."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("N,count", [(118, 40), (300, 64)])
def test_every_step_launch_choice_matches_oracle(dev, O, W, N, count):
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(N, count)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    two = plan.info().steps_per_cu == 2
    for mode in (0, 1):
        for wgcu in ((0, 1) if two else (0,)):
            for ring in (7, 4):
                print(f"[gpu tune] N={N} mode={mode} wgcu={wgcu} ring={ring}", flush=True)
                psp.set_tune_choice(plan, count, len(eps), 1, "sparse_steps", mode, wgcu, ring, 16)
                x, info = psp.solve_batched(plan, v, eps, b, path="auto")
                torch.cuda.synchronize()
                assert np.array_equal(info.cpu().numpy(), io)
                assert np.array_equal(x.cpu().numpy(), xo)


def test_tail_assembly_choices_match_oracle(dev, O, W):
    from paper_2311_11833_amd import psp
    ip, ix, vals, bs = W.scenario_batch(1354, 3)
    n = len(ip) - 1
    eps = W.config_eps("n601")
    plan = psp.Plan(ip, ix)
    sym = O.symbolic(n, ip, ix)
    xo, io, _, _ = O.sparse_batch(n, ip, ix, vals, sym, eps, bs)
    v, b = torch.from_numpy(vals).to(dev), torch.from_numpy(bs).to(dev)
    for cols, il, lu in ((16, 1, 1), (16, 1, 0), (16, 0, 1), (16, 0, 0), (4, 0, 1), (1, 0, 0)):
        print(f"[gpu tune] tail cols={cols} interleaved={il} lu={lu}", flush=True)
        psp.set_tune_choice(plan, 3, len(eps), 1, "sparse_tail", tail_cols=cols, tail_il=il, tail_lu=lu)
        x, info = psp.solve_batched(plan, v, eps, b, path="auto")
        torch.cuda.synchronize()
        assert np.array_equal(info.cpu().numpy(), io)
        assert np.array_equal(x.cpu().numpy(), xo)
    with pytest.raises(psp.PSPError):
        psp.set_tune_choice(plan, 3, len(eps), 1, "sparse_tail", tail_cols=3)
    with pytest.raises(psp.PSPError):
        psp.set_tune_choice(plan, 3, len(eps), 1, "sparse_tail", tail_il=2)


_CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import torch
from paper_2311_11833_amd import psp, workloads as W
ip, ix, vals, bs = W.scenario_batch(118, 48)
eps = W.config_eps("n601")
plan = psp.Plan(ip, ix)
v, b = torch.from_numpy(vals).cuda(), torch.from_numpy(bs).cuda()
before = psp.tune_choice(plan, 48, len(eps), 1)
if {tune}:
    psp.tune(plan, v, eps, b)
x, info = psp.solve_batched(plan, v, eps, b, path="auto")
torch.cuda.synchronize()
print(json.dumps({{"before": before, "after": psp.tune_choice(plan, 48, len(eps), 1),
                   "x0": float(x[0, 0].item())}}))
"""


def _child(tune: bool, cache: str) -> dict:
    env = dict(os.environ, PSP_TUNE_CACHE=cache)
    out = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT, tune=tune)], env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_tuning_cache_is_reused_by_a_fresh_process(dev, tmp_path):
    cache = str(tmp_path / "tune.txt")
    print("[gpu tune] tuning in a child process", flush=True)
    first = _child(True, cache)
    assert first["before"]["source"] == "heuristic"
    assert first["after"]["source"] == "tuned"
    assert os.path.exists(cache)
    print("[gpu tune] reading the cache in a second child process", flush=True)
    second = _child(False, cache)
    assert second["before"]["source"] == "cache file"
    for key in ("path", "steps_mode", "steps_wgcu", "ring", "tail_cols", "tail_il", "tail_lu"):
        assert second["before"][key] == first["after"][key]
    assert second["x0"] == first["x0"]
