#!/usr/bin/env python3
"""Benchmark: batched pivot-free FP64 solves/s at n = 601 (300-bus synthetic network).

One step = Alg. 1 over the whole batch, error test included: 512 Jacobians
(seeded load scenarios of one network) x K = 5 perturbations = 2560 perturbed
systems of 601 unknowns, each factored without pivoting, solved and combined
into 512 recovered solutions; the error of each combination is estimated from
its perturbed solutions and the Jacobians above the tolerance are solved again
at smaller nodes -- one call of the library (psp_solve_adaptive), timed as
eager calls and as a replayed HIP graph (the better is reported).  `value`
counts the 2560 systems of the batch per step (not the second solves).  Inputs
are resident in device memory before the timed region starts.

Also on the same GPU: the fixed nodes on every numeric path (the autotuner's
candidates; the step kernel's launch gives the roofline), the plain path (one
system per launch), the error of every recovered solution against a partially
pivoted LAPACK solve, the oracle (plain CPU code) on the host cores, and the
secondary configurations.

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

KERNELS = {"dense": "dense_factor_solve_kernel (one launch per step)",
           "sparse_batched": "all launches of one step: il_gather, il_diag + il_offdiag per factor level, "
                             "il_solve_level per solve level, il_combine",
           "sparse_lds": "sparse_lds_kernel (one launch per step)",
           "sparse_grouped": "il_group_kernel + il_combine (two launches per step)",
           "sparse_steps": "steps_kernel (one launch per step, combine fused)",
           "sparse_levels": "all launches of one step (per-level kernels)"}


def dense_flops(n, nrhs=1):
    return n * (n - 1) / 2 + (n - 1) * n * (2 * n - 1) / 3 + nrhs * (2 * n * n - n)


def sparse_flops(info, n, nrhs=1):
    return info.flops_sparse_factor + nrhs * (4 * info.nnz_l + n)


# counter summaries (FETCH_SIZE + WRITE_SIZE per launch) and the sources of the kernel they cover
TRAFFIC_PROFILES = {
    "sparse_steps": ("steps_kernel_n601_hbm_traffic.md", ["steps.hip"]),
    "dense": ("dense_kernel_n601_hbm_traffic.md", ["dense.hip", "dense_ops.h"]),
}


def measured_traffic(path):
    """HBM bytes per launch of a path's kernel from the committed counter summary,
    or None when the summary is missing or the kernel source changed since."""
    import hashlib
    if path not in TRAFFIC_PROFILES:
        return None
    name, sources = TRAFFIC_PROFILES[path]
    prof = os.path.join(ROOT, "profiles", name)
    try:
        text = open(prof).read()
        h = hashlib.sha256()
        for f in sources:
            h.update(open(os.path.join(ROOT, "paper_2311_11833_amd", "csrc", f), "rb").read())
        digest = h.hexdigest()[:16]
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes", "kernel_source")))
    if vals.get("kernel_source_sha256_16", "").strip() != digest:
        return None
    return float(vals["traffic_bytes_per_launch"])


def _events(torch, fn, reps):
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        out = fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def extra_configs(psp, W, torch, dev, only=None, tol=1e-10):
    """Secondary configurations, timed with HIP events: the adjoint with 64 right-hand
    sides at n=601, the paper's symmetric node scheme, an uneven batch, the Newton
    power-flow loop and the 20,001-unknown system.  `only`: names to run (all if None)."""
    out = {}
    eps = W.config_eps("n601")
    rng = np.random.default_rng(4)

    def want(name):
        return only is None or name in only

    if want("n601_adjoint_64rhs"):
        from paper_2311_11833_amd.autograd import perturbed_solve
        # 64 Jacobians of the 300-bus network, K=5, 64 RHS: forward and backward of the autograd op
        J, R = 64, 64
        ip, ix, vals, _ = W.scenario_batch(300, J)
        n = len(ip) - 1
        plan = psp.Plan(ip, ix)
        v = torch.from_numpy(vals).to(dev).requires_grad_(True)
        B = torch.from_numpy(rng.standard_normal((J, n, R))).to(dev).requires_grad_(True)
        G = torch.from_numpy(rng.standard_normal((J, n, R))).to(dev)

        def fwd():
            return perturbed_solve(v, B, plan, eps, path="sparse")

        def fwd_bwd():
            x = perturbed_solve(v, B, plan, eps, path="sparse")
            return torch.autograd.grad(x, (v, B), G)

        fwd_bwd()
        torch.cuda.synchronize()
        f_ms, _ = _events(torch, fwd, 3)
        fb_ms, _ = _events(torch, fwd_bwd, 3)
        # the same per Jacobian, one Jacobian per call (the plain path), on the first 8
        JP = 8

        def plain_fwd_bwd():
            for s_ in range(JP):
                vs = v[s_:s_ + 1].detach().requires_grad_(True)
                Bs = B[s_:s_ + 1].detach().requires_grad_(True)
                xs = perturbed_solve(vs, Bs, plan, eps, path="sparse")
                torch.autograd.grad(xs, (vs, Bs), G[s_:s_ + 1])

        plain_fwd_bwd()
        torch.cuda.synchronize()
        p_ms, _ = _events(torch, plain_fwd_bwd, 2)
        out["n601_adjoint_64rhs"] = {"jacobians": J, "K": len(eps), "nrhs": R, "path": "sparse (split steps)",
                                     "forward_ms": f_ms, "backward_ms": fb_ms - f_ms,
                                     "forward_rhs_solves_per_s": J * len(eps) * R / (f_ms / 1e3),
                                     "plain_fwd_bwd_ms_per_jacobian": p_ms / JP,
                                     "batched_fwd_bwd_ms_per_jacobian": fb_ms / J,
                                     "batched_speedup": (p_ms / JP) / (fb_ms / J)}
        print(f"[bench] n601 adjoint 64 rhs: fwd {f_ms:.3f} ms, bwd {fb_ms - f_ms:.3f} ms; plain {p_ms / JP:.3f} ms "
              f"per Jacobian vs batched {fb_ms / J:.3f}", file=sys.stderr, flush=True)
    if want("fig1_symmetric_nodes"):
        # the paper's own scheme (Fig. 1 analogue): nodes +-alpha*eps, alpha = 1..m, eps = 2e-3, on 25
        # scenarios of the 300-bus network, with D = I and with a Gaussian diagonal D (max |d_i| = 1);
        # error against LAPACK's pivoted solve and the device residual, per number of solves 2m
        TS = 25
        ipf, ixf, valsf, bsf = W.scenario_batch(300, TS)
        nf = len(ipf) - 1
        pf = psp.Plan(ipf, ixf)
        vf, bf = torch.from_numpy(valsf).to(dev), torch.from_numpy(bsf).to(dev)
        xstar = [np.linalg.solve(W.to_dense(nf, ipf, ixf, valsf[s_]), bsf[s_]) for s_ in range(TS)]
        dg = np.random.default_rng(1311).standard_normal(nf)
        dg /= np.abs(dg).max()
        fig = {"eps": 2e-3, "scenarios": TS, "n": nf}
        for dname, dvec in (("identity", None), ("gaussian", torch.from_numpy(dg).to(dev))):
            rows_ = {}
            for m in range(1, 6):
                nodes = np.array([sg * a_ * 2e-3 for a_ in range(1, m + 1) for sg in (1.0, -1.0)])
                xf, _ = psp.solve_batched(pf, vf, nodes, bf, path="sparse", d=dvec)
                rnf, bnf = psp.residual(pf, vf, bf, xf)
                xfn = xf.cpu().numpy()
                e_ = np.array([np.abs(xfn[s_] - xstar[s_]).max() / np.abs(xstar[s_]).max() for s_ in range(TS)])
                r_ = (rnf / bnf).cpu().numpy().ravel()
                rows_[str(2 * m)] = {"err_median": float(np.median(e_)), "err_max": float(np.nanmax(e_)),
                                     "res_median": float(np.median(r_)), "res_max": float(np.nanmax(r_))}
            fig[dname] = rows_
        out["fig1_symmetric_nodes"] = fig
        print("[bench] symmetric nodes (median err by solves): " + ", ".join(
            f"{k}: I {fig['identity'][k]['err_median']:.1e} / G {fig['gaussian'][k]['err_median']:.1e}"
            for k in fig["identity"]), file=sys.stderr, flush=True)
    if want("uneven_512"):
        # uneven batch: 512 Jacobians of five networks (n = 61 .. 2709), one psp_solve_group call
        groups = W.uneven_batch(512)
        items, paths_u, flops_u, sizes = [], {}, 0.0, {}
        for N, ipu, ixu, valsu, bsu in groups:
            pu = psp.Plan(ipu, ixu)
            vu, bu = torch.from_numpy(valsu).to(dev), torch.from_numpy(bsu).to(dev)
            psp.tune(pu, vu, eps, bu)
            paths_u[len(ipu) - 1] = psp.tune_choice(pu, int(valsu.shape[0]), len(eps), 1)
            sizes[len(ipu) - 1] = int(valsu.shape[0])
            flops_u += valsu.shape[0] * len(eps) * sparse_flops(pu.info(), len(ipu) - 1)
            items.append((pu, vu, bu))
        grp = psp.Group([(p_, v_.shape[0]) for p_, v_, _ in items], eps)
        gin = [(v_, b_) for _, v_, b_ in items]
        grp.run(gin)
        torch.cuda.synchronize()
        g_ms, outs_u = _events(torch, lambda: grp.run(gin), 3)
        graph_u, outs_g = grp.capture(gin)
        grp.replay(graph_u)
        torch.cuda.synchronize()
        gr_ms, _ = _events(torch, lambda: grp.replay(graph_u), 5)
        same = all(torch.equal(a[0], b_[0]) for a, b_ in zip(outs_u, outs_g))
        best = min(g_ms, gr_ms)
        # recovered x against a partially pivoted sparse LU (SuperLU), every Jacobian of every item
        import scipy.sparse as sps
        import scipy.sparse.linalg as spla
        acc_u = {}
        for (N, ipu, ixu, valsu, bsu), o_ in zip(groups, outs_u):
            nu, xu = len(ipu) - 1, o_[0].cpu().numpy()
            e_ = []
            for s_ in range(valsu.shape[0]):
                xs_ = spla.splu(sps.csr_matrix((valsu[s_], ixu, ipu), shape=(nu, nu)).tocsc()).solve(bsu[s_])
                e_.append(np.abs(xu[s_] - xs_).max() / np.abs(xs_).max())
            e_ = np.array(e_)
            acc_u[nu] = {"above_1e-9": int((e_ > 1e-9).sum()), "max": float(np.nanmax(e_)),
                         "median": float(np.median(e_))}
        # the same group with the error test on every item (psp_group_run_adaptive)
        grp.run_adaptive(gin, tol=tol)
        torch.cuda.synchronize()
        ga_ms, outs_a = _events(torch, lambda: grp.run_adaptive(gin, tol=tol), 3)
        graph_a, _ = grp.capture_adaptive(gin, tol=tol)
        grp.replay(graph_a)
        torch.cuda.synchronize()
        gra_ms, _ = _events(torch, lambda: grp.replay(graph_a), 5)
        acc_a, resc_a = {}, {}
        for (N, ipu, ixu, valsu, bsu), o_ in zip(groups, outs_a):
            nu, xu = len(ipu) - 1, o_[0].cpu().numpy()
            e_ = np.array([np.abs(xu[s_] - (xs_ := spla.splu(sps.csr_matrix((valsu[s_], ixu, ipu), shape=(nu, nu))
                                                            .tocsc()).solve(bsu[s_]))).max() / np.abs(xs_).max()
                           for s_ in range(valsu.shape[0])])
            acc_a[nu] = {"above_1e-9": int((e_ > 1e-9).sum()), "max": float(np.nanmax(e_)),
                         "median": float(np.median(e_))}
            resc_a[nu] = int((o_[3].cpu().numpy() != 1.0).sum())
        best_a = min(ga_ms, gra_ms)
        out["uneven_512"] = {"jacobians_by_n": sizes, "K": len(eps), "path_by_n": paths_u, "ms_per_call": best,
                             "eager_ms": g_ms, "graph_ms": gr_ms, "graph_bitwise_equal": bool(same),
                             "solves_per_s": 512 * len(eps) / (best / 1e3),
                             "sparse_tflops": flops_u / (best / 1e3) / 1e12,
                             "rel_err_vs_pivoted_by_n": acc_u,
                             "nodes": "1e-3 * 2^-k for every item (no error test)",
                             "error_test": {"tol": tol, "ms_per_call": best_a, "eager_ms": ga_ms,
                                            "graph_ms": gra_ms, "rescaled_by_n": resc_a,
                                            "rel_err_vs_pivoted_by_n": acc_a}}
        print(f"[bench] uneven 512: eager {g_ms:.3f} ms, graph {gr_ms:.3f} ms; with the error test eager "
              f"{ga_ms:.3f} ms, graph {gra_ms:.3f} ms; above 1e-9: fixed "
              f"{sum(v['above_1e-9'] for v in acc_u.values())}, error test {sum(v['above_1e-9'] for v in acc_a.values())}",
              file=sys.stderr, flush=True)
    if want("newton_pf_512"):
        # Newton-Raphson power flows (Sec. IV's setting): 512 scenarios of the 300-bus network with 69
        # generator buses, flat start, at most 20 iterations, K = 5; one psp_pf_newton call
        NS = 512
        case = W.pf_case(300)
        scn = W.pf_scenarios(case, NS)
        plan_pf = psp.Plan(case.indptr, case.indices)
        pfm = psp.PowerFlow(plan_pf, case.y_indptr, case.y_indices, case.g, case.b, case.pv)
        x0d, spd, ptd = (torch.from_numpy(a).to(dev) for a in (scn.x0, scn.spec, scn.part))
        pfm.newton(x0d, spd, ptd, eps, max_iter=20)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            xn, itn, stn, fnn = pfm.newton(x0d, spd, ptd, eps, max_iter=20)
        torch.cuda.synchronize()
        nr_ms = (time.perf_counter() - t0) * 1e3 / reps
        ev_ms, (Fj, Jj, _) = _events(torch, lambda: pfm.eval(x0d, spd, ptd), 20)
        so_ms, _ = _events(torch, lambda: psp.solve_batched(plan_pf, Jj, eps, Fj), 5)
        itn, stn = itn.cpu().numpy(), stn.cpu().numpy()
        at_target = int(np.sum(np.abs(xn.cpu().numpy() - scn.x_target).max(axis=1) <= 1e-8))
        out["newton_pf_512"] = {"buses": 300, "n": case.n, "generator_buses": int(case.pv.sum()), "scenarios": NS,
                                "K": len(eps), "tol": 1e-9, "max_iter": 20, "ms_per_call": nr_ms,
                                "power_flows_per_s": NS / (nr_ms / 1e3),
                                "iterations_hist": {str(k): int(v) for k, v in enumerate(np.bincount(itn)) if v},
                                "converged": int(np.sum(stn == 0)), "at_own_target": at_target,
                                "eval_kernel_ms": ev_ms, "solve_ms": so_ms}
        print(f"[bench] newton 512 x 300-bus: {nr_ms:.2f} ms ({int(itn.max())} iterations max), eval {ev_ms * 1e3:.1f} us, "
              f"solve {so_ms:.3f} ms, converged {int(np.sum(stn == 0))}, at target {at_target}", file=sys.stderr, flush=True)
    if want("n20001_32rhs"):
        # 10,000-bus network, n = 20,001, K = 4, 32 RHS: forward, transposed solve and gradient
        from paper_2311_11833_amd.workloads import make_network, make_state, jacobian, seed_state
        import scipy.sparse as sps
        import scipy.sparse.linalg as spla
        net = make_network(10000)
        vm, va, p = make_state(10000, seed_state(10000, 0))
        Jc = jacobian(net, vm, va, p)
        eps4 = W.large_eps()
        tp0 = time.perf_counter()
        plan4 = psp.Plan(Jc.indptr, Jc.indices)
        plan4.ensure(dev)
        torch.cuda.synchronize()
        plan4_ms = (time.perf_counter() - tp0) * 1e3
        v4 = torch.from_numpy(Jc.data[None]).to(dev)
        # its own generator, so that the right-hand sides do not depend on which extras ran first
        B4 = torch.from_numpy(np.random.default_rng(20001).standard_normal((1, Jc.n, 32))).to(dev)
        F = psp.Factors(plan4, v4, eps4, path="sparse", nrhs_cap=32)
        torch.cuda.synchronize()
        fac_ms, F = _events(torch, lambda: psp.Factors(plan4, v4, eps4, path="sparse", nrhs_cap=32), 3)
        sol_ms, Xk = _events(torch, lambda: F.solve(B4), 3)
        tr_ms, Lk = _events(torch, lambda: F.solve(B4, transpose=True), 3)
        gr_ms, _ = _events(torch, lambda: F.grad_values(Lk, Xk), 3)
        X = F.combine(Xk)
        rn, bn = psp.residual(plan4, v4, B4, X, keep_r=True)[:2]
        info = plan4.info()
        # error of the 32 recovered solutions against a partially pivoted sparse LU (SuperLU)
        A4 = sps.csr_matrix((Jc.data, Jc.indices, Jc.indptr), shape=(Jc.n, Jc.n)).tocsc()
        xs4 = spla.splu(A4, permc_spec="COLAMD").solve(B4[0].cpu().numpy())
        e4 = np.abs(X[0].cpu().numpy() - xs4).max(axis=0) / np.abs(xs4).max(axis=0)
        n4, nt = Jc.n, int(getattr(info, "tail_n", 0))
        fac_flops = len(eps4) * info.flops_sparse_factor
        fac_bytes = len(eps4) * (n4 + 2 * info.nnz_l) * 8
        out["n20001_32rhs"] = {"n": Jc.n, "nnz": int(info.nnz), "nnz_l": int(info.nnz_l), "K": len(eps4), "nrhs": 32,
                               "eps": [float(e) for e in eps4], "plan_create_upload_ms": plan4_ms,
                               "factor_ms": fac_ms, "solve_ms": sol_ms, "transposed_solve_ms": tr_ms,
                               "grad_values_ms": gr_ms, "path": "sparse_tail (split calls)",
                               "levels_total": int(info.nlev[0]), "sparse_levels": int(info.tail_fac_levels),
                               "dense_tail_columns": nt, "dense_tail_panels": (nt + 31) // 32,
                               "factor_us_per_level_or_panel": fac_ms * 1e3 / max(1, info.tail_fac_levels + (nt + 31) // 32),
                               "factor_tflops": fac_flops / (fac_ms / 1e3) / 1e12,
                               "factor_fp64_frac": fac_flops / (fac_ms / 1e3) / PEAK_FP64,
                               "factor_gbs_algorithmic": fac_bytes / (fac_ms / 1e3) / 1e9,
                               "residual_rel_max": float((rn / bn).max()),
                               "rel_err_vs_pivoted": {"rhs": 32, "above_1e-9": int((e4 > 1e-9).sum()),
                                                      "max": float(e4.max()), "median": float(np.median(e4)),
                                                      "reference": "SuperLU partial pivoting (scipy splu)"}}
        print(f"[bench] n20001: factor {fac_ms:.2f} ms, solve {sol_ms:.2f} ms, trans {tr_ms:.2f} ms, grad {gr_ms:.2f} ms, "
              f"err max {e4.max():.2e}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--jacobians", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-10, help="error-test tolerance of the adaptive call")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="length of the oracle's timed sample (passes over the batch are repeated)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-system-per-launch timing")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay timing")
    ap.add_argument("--no-paths", action="store_true", help="time only the step-schedule path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three 256 MiB device copies (the reference kernel for HBM counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary configurations (adjoint, node schemes, uneven batch, Newton loop, "
                         "20,001 unknowns)")
    ap.add_argument("--extras", default=None,
                    help="comma-separated secondary configurations to run (n601_adjoint_64rhs, "
                         "fig1_symmetric_nodes, uneven_512, newton_pf_512, n20001_32rhs); default all")
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
    tp = time.perf_counter()
    plan = psp.Plan(ip, ix)
    pinfo = plan.info()
    plan.ensure(dev)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - tp) * 1e3
    vals_d = torch.from_numpy(vals).to(dev)
    b_d = torch.from_numpy(bs).to(dev)
    systems = S * K
    print(f"[bench] inputs ready n={n} jacobians={S} K={K} plan {plan_ms:.1f} ms ({time.time() - t0:.1f}s)",
          file=sys.stderr, flush=True)

    st = torch.cuda.current_stream()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            out = fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            out = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, out

    def graph_timed(fn, steps, warmup):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            out = fn()
        ms, _ = timed(g.replay, steps, warmup)
        return ms, out

    # ---- the fixed nodes 1e-3 * 2^-k on every numeric path (one fused call each; the autotuner's timing)
    chosen, tuner_ms = psp.tune(plan, vals_d, eps, b_d)
    torch.cuda.synchronize()
    tuned = psp.tune_choice(plan, S, K, 1)
    print(f"[bench] tuner: {tuner_ms} -> {tuned}", file=sys.stderr, flush=True)
    results = {}
    for p in (["sparse_steps"] if args.no_paths else
              ["dense", "sparse_batched", "sparse_grouped", "sparse_lds", "sparse_steps"]):
        if p not in tuner_ms and p != "sparse_steps":
            continue
        ms, (x, info) = timed(lambda: psp.solve_batched(plan, vals_d, eps, b_d, path=p), args.steps, args.warmup)
        results[p] = dict(ms=ms, x=x, info=info)
        print(f"[bench] fixed nodes, {p}: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # ---- headline: Alg. 1 with its error test deciding the node size per Jacobian (psp_solve_adaptive):
    # the batch at the fixed nodes, the estimate from the perturbed solutions, the rescaled second
    # solve of the Jacobians above tol -- one call, no host synchronisation
    def adaptive():
        return psp.solve_adaptive(plan, vals_d, eps, b_d, tol=args.tol)

    ad_ms, ad_out = timed(adaptive, args.steps, args.warmup)
    print(f"[bench] adaptive (error test + rescale): {ad_ms:.3f} ms/step", file=sys.stderr, flush=True)
    ad_graph_ms, graph_equal = None, None
    if not args.no_graph:
        ad_graph_ms, g_out = graph_timed(adaptive, args.steps, args.warmup)
        graph_equal = bool(all(torch.equal(a.nan_to_num(7.0), b.nan_to_num(7.0)) for a, b in zip(g_out, ad_out)))
        print(f"[bench] adaptive graph replay: {ad_graph_ms:.3f} ms/step", file=sys.stderr, flush=True)
    ms = min(ad_ms, ad_graph_ms) if ad_graph_ms is not None else ad_ms
    value = systems / (ms / 1e3)
    xa, ia, esta, sca = (t.cpu().numpy() for t in ad_out)
    rescaled = int((sca != 1.0).sum())

    def flops_of(p):
        return dense_flops(n) if p == "dense" else sparse_flops(pinfo, n)

    # roofline of the dominant kernel: steps_kernel, one launch per fixed-node call, timed with HIP
    # events on the launch stream; algorithmic sparse flops per system x 2560 systems per launch
    steps_ms = results["sparse_steps"]["ms"]
    achieved = flops_of("sparse_steps") * systems / (steps_ms / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": measured_traffic("sparse_steps"),
                "kernel": KERNELS["sparse_steps"], "kernel_ms": steps_ms,
                "flops_per_system": flops_of("sparse_steps"), "systems_per_launch": systems,
                "hbm_bytes_algorithmic": S * (pinfo.nnz + 2 * n) * 8,
                "hbm_gbs_algorithmic": S * (pinfo.nnz + 2 * n) * 8 / (steps_ms / 1e3) / 1e9}
    # the bound that applies: the schedule's dependency depth (barrier steps one after another per
    # workgroup, K systems per workgroup, workgroups resident per CU); ns per step per workgroup
    if pinfo.steps > 0 and pinfo.steps_per_cu > 0:
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        slots = cus * pinfo.steps_per_cu
        per_jac = tuned["steps_mode"] == 1 or (tuned["steps_mode"] == -1 and S >= slots)
        wgs, sys_wg = (S, len(eps)) if per_jac else (S * len(eps), 1)
        rounds = -(-wgs // slots)                          # rounds of resident workgroups
        roofline["dependency_bound"] = {
            "barrier_steps_per_system": int(pinfo.steps), "systems_per_workgroup": sys_wg,
            "workgroups_per_cu": int(pinfo.steps_per_cu), "workgroup_rounds": int(rounds),
            "ns_per_step_per_workgroup": steps_ms * 1e6 / (rounds * sys_wg * pinfo.steps)}
    roofline_dense = None
    if "dense" in results:
        a_d = dense_flops(n) * systems / (results["dense"]["ms"] / 1e3)
        tr_d = measured_traffic("dense")
        roofline_dense = {"bound": "mfma", "achieved": a_d / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                          "frac": a_d / PEAK_FP64, "traffic": tr_d, "kernel": KERNELS["dense"],
                          "flops_per_system": dense_flops(n), "solves_per_s": systems / (results["dense"]["ms"] / 1e3),
                          "hbm_gbs_measured": tr_d / (results["dense"]["ms"] / 1e3) / 1e9 if tr_d else None}
    paths = {}
    for p, rr in results.items():
        paths[p] = {"ms_per_step": rr["ms"], "solves_per_s": systems / (rr["ms"] / 1e3),
                    "tflops": flops_of(p) * systems / (rr["ms"] / 1e3) / 1e12}
    xs_ = [rr["x"] for rr in results.values()]
    paths["all_paths_bitwise_equal"] = bool(all(torch.equal(xs_[0], x) for x in xs_[1:]))

    # ---- errors of every recovered solution against a partially pivoted LAPACK solve, and the
    # device error test (relative residual)
    xstar = np.stack([np.linalg.solve(W.to_dense(n, ip, ix, vals[s_]), bs[s_]) for s_ in range(S)])

    def err_summary(xx):
        e_ = np.abs(xx - xstar).max(axis=1) / np.abs(xstar).max(axis=1)
        e_ = np.where(np.isfinite(e_), e_, np.inf)
        return {"jacobians": S, "above_1e-9": int(np.sum(e_ > 1e-9)), "max": float(e_.max()),
                "median": float(np.median(e_))}

    err_ad = err_summary(xa)
    err_fixed = err_summary(results["sparse_steps"]["x"].cpu().numpy())
    rn, bn = psp.residual(plan, vals_d, b_d, ad_out[0])
    rel_res = (rn / bn).cpu().numpy()
    print(f"[bench] errors vs pivoted, all {S}: adaptive {err_ad['above_1e-9']} above 1e-9 (max {err_ad['max']:.2e}), "
          f"fixed nodes {err_fixed['above_1e-9']} (max {err_fixed['max']:.2e}); rescaled {rescaled}",
          file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain:
        # one system per launch: 5 Jacobians x K single-system calls (batch 1, K 1: the fused
        # factor+solve launch and its one-term combine), stream-ordered, no graph; median of 20
        J = 5

        def plain_seq():
            for s_ in range(J):
                for k_ in range(K):
                    psp.solve_batched(plan, vals_d[s_:s_ + 1], eps[k_:k_ + 1], b_d[s_:s_ + 1], path="sparse_steps")

        plain_seq()
        torch.cuda.synchronize()
        reps = []
        for _ in range(20):
            pm, _ = timed(plain_seq, 1, 0)
            reps.append(pm)
        pms = float(np.median(reps))
        plain = {"solves_per_s": J * K / (pms / 1e3), "systems": J * K, "ms_median_of_20": pms,
                 "launches": 2 * J * K, "path": "sparse_steps (batch 1, K 1 per call)",
                 "batched_speedup_fixed_nodes": (systems / (steps_ms / 1e3)) / (J * K / (pms / 1e3)),
                 "batched_speedup_adaptive": value / (J * K / (pms / 1e3))}
        print(f"[bench] plain: {pms:.3f} ms for {J * K} systems", file=sys.stderr, flush=True)

    only = None if args.extras is None else set(args.extras.split(","))
    extra = None if args.no_extra else extra_configs(psp, W, torch, dev, only, args.tol)

    cpu = None
    if not args.no_cpu:
        # the oracle's adaptive solve (the same rule, plain C and Python), timed on the host cores at
        # one thread and at all threads over about cpu_seconds each, bitwise-compared with the GPU
        from oracle import oracle as O
        sym = O.symbolic(n, ip, ix)
        cpu = {"unit": "solves/s", "kind": "oracle"}
        for label, thr in (("1_thread", 1), ("all_threads", os.cpu_count() or 1)):
            O.set_threads(thr)
            cnt = S if thr > 1 else min(S, 64)
            t = time.perf_counter()
            xo, io, eo, so = O.adaptive_batch(n, ip, ix, vals[:cnt], sym, eps, bs[:cnt], args.tol)
            dt = time.perf_counter() - t
            passes = 1
            while dt < args.cpu_seconds / 2 and passes < 1000:
                O.adaptive_batch(n, ip, ix, vals[:cnt], sym, eps, bs[:cnt], args.tol)
                passes += 1
                dt = time.perf_counter() - t
            cpu[label] = {"value": passes * cnt * K / dt, "cores": thr,
                          "sample": f"{passes} passes of the oracle's adaptive solve over {cnt} Jacobians x K={K}, "
                                    f"{dt:.1f} s wall",
                          "bitwise_equal_to_gpu": bool(np.array_equal(xo, xa[:cnt]) and np.array_equal(so, sca[:cnt]))}
        cpu["value"] = cpu["all_threads"]["value"]
        cpu["cores"] = cpu["all_threads"]["cores"]
        cpu["sample"] = cpu["all_threads"]["sample"]
        cpu["bitwise_equal_to_gpu"] = cpu["all_threads"]["bitwise_equal_to_gpu"]

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n601_batched: 300-bus network, 512 scenarios x K=5, error test + rescale",
                   "network_buses": N, "n": n, "nnz": int(pinfo.nnz), "jacobians": S, "K": K,
                   "systems_per_step": systems, "nrhs": 1, "path": "sparse_steps (psp_solve_adaptive)",
                   "timed_as": "graph replay" if ad_graph_ms is not None and ad_graph_ms <= ad_ms else "eager calls",
                   "eps": [float(e) for e in eps], "tol": args.tol, "ordering": "minimum degree"},
        "roofline": roofline,
        "roofline_dense": roofline_dense,
        "cpu_baseline": cpu,
        "rel_err_vs_pivoted": err_ad,
        "rel_err_vs_pivoted_fixed_nodes": err_fixed,
        "rescaled_jacobians": rescaled,
        "recovered_solutions_per_s": S / (ms / 1e3),
        "eager_ms_per_step": ad_ms,
        "graph_ms_per_step": ad_graph_ms,
        "graph_bitwise_equal": graph_equal,
        "fixed_nodes_ms_per_step": steps_ms,
        "fixed_nodes_solves_per_s": systems / (steps_ms / 1e3),
        "plan_create_upload_ms": plan_ms,
        "plain": plain,
        "paths": paths,
        "tuner_ms": tuner_ms,
        "tuned_choice": tuned,
        "info_nonzero": int(np.count_nonzero(ia)),
        "residual_rel_all": {"max": float(rel_res.max()), "median": float(np.median(rel_res)),
                             "jacobians": int(rel_res.size), "above_1e-9": int(np.sum(rel_res > 1e-9)),
                             "kernel": "residual_kernel (device)"},
        "extra": extra,
    }
    print(json.dumps(out))
    if args.copy_calibration:
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
