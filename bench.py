#!/usr/bin/env python3
"""Benchmark: batched pivot-free FP64 solves/s at n = 601 (300-bus synthetic network).

One step = Alg. 1 steps 1-4 over the whole batch: 512 Jacobians (seeded load
scenarios of one network) x K = 5 perturbations = 2560 perturbed systems of
601 unknowns, each factored without pivoting, solved, and combined into 512
recovered solutions, in one fused launch of the library.  Inputs are resident
in device memory before the timed region starts.

Also reported on the same GPU:
  * the plain path: one system per launch (K launches per Jacobian + combine);
  * the other numeric path (dense vs sparse) for the same workload;
  * the oracle (plain CPU FP64 code) on a bounded sample, for context;
  * relative error of the recovered solutions against the pivoted oracle on a
    sample of Jacobians.

Prints ONE JSON line.  Only one GPU is supported.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pivot-free FP64 solves/s at n≈600, batched vs plain; rel err vs pivoted oracle"
PEAK_FP64 = 78.6e12          # MI355X FP64 (vector and matrix), FLOP/s
PEAK_HBM = 8.0e12            # MI355X HBM3E, B/s


def dense_flops(n, nrhs=1):
    f = n * (n - 1) / 2 + (n - 1) * n * (2 * n - 1) / 3
    return f + nrhs * (2 * n * n - n)


def sparse_flops(info, n, nrhs=1):
    return info.flops_sparse_factor + nrhs * (4 * info.nnz_l + n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", choices=["best", "dense", "sparse"], default="best")
    ap.add_argument("--jacobians", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-system-per-launch timing")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (this build has no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_11833_amd import psp, workloads as W

    dev = torch.device("cuda:0")
    N, S = 300, args.jacobians
    eps = W.config_eps("n601")
    K = len(eps)
    t0 = time.time()
    ip, ix, vals, bs = W.scenario_batch(N, S)
    n = len(ip) - 1
    plan = psp.Plan(ip, ix)
    pinfo = plan.info()
    vals_d = torch.from_numpy(vals).to(dev)
    b_d = torch.from_numpy(bs).to(dev)
    print(f"[bench] inputs ready n={n} jacobians={S} K={K} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)

    def run(path, steps, warmup):
        for _ in range(warmup):
            x, info = psp.solve_batched(plan, vals_d, eps, b_d, path=path)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(st)
        for _ in range(steps):
            x, info = psp.solve_batched(plan, vals_d, eps, b_d, path=path)
        e1.record(st)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1e3 / steps
        return e0.elapsed_time(e1) / steps, wall, x, info

    results = {}
    paths = ["dense", "sparse"] if args.path == "best" else [args.path]
    for p in paths:
        ms, wall, x, info = run(p, args.steps, args.warmup)
        results[p] = dict(ms=ms, wall_ms=wall, x=x, info=info)
        print(f"[bench] {p}: {ms:.3f} ms/step (event), {wall:.3f} ms wall", file=sys.stderr, flush=True)
    best = min(results, key=lambda p: results[p]["ms"])
    r = results[best]
    ms = r["ms"]
    systems = S * K
    value = systems / (ms / 1e3)

    per_sys = dense_flops(n) if best == "dense" else sparse_flops(pinfo, n)
    achieved = per_sys * systems / (ms / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": None,
                "kernel": "dense_factor_solve_kernel" if best == "dense" else "sparse_lds_kernel",
                "flops_per_system": per_sys}

    others = {}
    for p, rr in results.items():
        f = dense_flops(n) if p == "dense" else sparse_flops(pinfo, n)
        others[p] = {"ms_per_step": rr["ms"], "solves_per_s": systems / (rr["ms"] / 1e3),
                     "tflops": f * systems / (rr["ms"] / 1e3) / 1e12}
    if len(results) == 2:
        xa, xb = results["dense"]["x"].cpu().numpy(), results["sparse"]["x"].cpu().numpy()
        others["dense_vs_sparse_bitwise_equal"] = bool(np.array_equal(xa, xb))

    info_np = r["info"].cpu().numpy()
    x_np = r["x"].cpu().numpy()
    from oracle import oracle as O
    # error of the recovered solution against the pivoted oracle on a sample
    errs, resid = [], []
    for s in (0, 1, 2, 3):
        A = W.to_dense(n, ip, ix, vals[s])
        xs = O.pivoted_solve(A, bs[s])
        errs.append(float(np.abs(x_np[s] - xs).max() / np.abs(xs).max()))
        resid.append(float(np.linalg.norm(A @ x_np[s] - bs[s]) / np.linalg.norm(bs[s])))

    plain = None
    if not args.no_plain:
        # one system per launch: each (s, k) alone (batch=1, K=1), then the combine
        J = min(S, 8)
        c = psp.weights(eps)
        for _ in range(2):
            for s in range(J):
                for k in range(K):
                    psp.solve_batched(plan, vals_d[s:s + 1], eps[k:k + 1], b_d[s:s + 1], path=best)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for s in range(J):
            xk = []
            for k in range(K):
                xk.append(psp.solve_batched(plan, vals_d[s:s + 1], eps[k:k + 1], b_d[s:s + 1], path=best)[0])
        torch.cuda.synchronize()
        pms = (time.perf_counter() - w0) * 1e3
        plain = {"solves_per_s": J * K / (pms / 1e3), "systems": J * K, "ms": pms,
                 "batched_speedup": value / (J * K / (pms / 1e3))}

    cpu = None
    if not args.no_cpu:
        sym = O.symbolic(n, ip, ix)
        cnt = 8 if best == "dense" else 256
        t = time.perf_counter()
        if best == "dense":
            xo, io, _, thr = O.dense_batch(n, ip, ix, vals[:cnt], eps, bs[:cnt], perm=sym.perm)
        else:
            xo, io, _, thr = O.sparse_batch(n, ip, ix, vals[:cnt], sym, eps, bs[:cnt])
        dt = time.perf_counter() - t
        cpu = {"value": cnt * K / dt, "unit": "solves/s", "cores": int(thr), "kind": "oracle",
               "sample": f"{cnt} Jacobians x K={K} = {cnt * K} systems of n={n}, {best} oracle, {dt:.1f} s",
               "bitwise_equal_to_gpu": bool(np.array_equal(xo, x_np[:cnt]))}

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n601_batched", "network_buses": N, "n": n, "nnz": int(pinfo.nnz),
                   "jacobians": S, "K": K, "systems_per_step": systems, "nrhs": 1, "path": best,
                   "eps": [float(e) for e in eps], "ordering": "minimum degree",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain": plain,
        "paths": others,
        "recovered_solutions_per_s": S / (ms / 1e3),
        "rel_err_vs_pivoted": {"max": max(errs), "median": float(np.median(errs)), "sample": 4,
                               "residual_max": max(resid)},
        "info_nonzero": int(np.count_nonzero(info_np)),
        "wall_ms_per_step": r["wall_ms"],
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
