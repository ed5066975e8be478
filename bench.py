#!/usr/bin/env python3
"""Time to 1e-5 tolerance of the MaxCut SDP hot path on one MI355X.

Workload (one "step"): the plain float64 method (ALM + L-BFGS with H0 = I and
the exact line search) solving the 1e7-node Chung-Lu MaxCut SDP (exponent 2.5,
mean degree 8, 4e7 edges, unit weights, C = -L/4, diag(X) = 1, rank 24) from a
seeded unit-row starting factor until err1 <= 1e-5 and |err3| <= 1e-5.  The
problem, the starting factor and the workspace are resident in HBM before the
timed region; the timed region is the solve.  The problem is built with the
library's degree node order (nodes relabelled inside the library for locality
of the SpMM gather; the starting factor and the result stay in the graph's
labels); the comparison path f64_input_order solves the input order.  Beside
it, untimed by the step but timed on its own: float32 + learned warm start on
the same graph, and the same with the row-block H0 of the L-BFGS direction
(features and MLP inference counted in their time), with the model committed
beside the library.

The whole run keeps to a wall-clock budget (--budget, counted from the start of
the process, generation and upload included): warm-ups are short capped solves,
as many timed solves run as fit (at least one; `steps` reports the executed
count), every solve carries a time limit, and the comparison path and the CPU
baseline run only in the time left.

The JSON line carries the SpMM roofline (algorithmic bytes per launch over the
launch duration measured with HIP events on the solve's stream) and the CPU
oracle's time on a bounded sample of the same workload family.
"""

import argparse
import json
import math
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-5 tol: plain FP64 vs FP32+learned warm start; SpMM/SDDMM HBM GB/s"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "cl_10m": (["cl_10m"], "maxcut n=1e7 Chung-Lu beta=2.5 mean degree 8 (4e7 edges), unit weights, C=-L/4, "
                           "diag(X)=1, rank 24"),
    "pair_1m": (["er_1m_pm1", "cl_1m_pm1"],
                "maxcut n=1e6 pair: Erdos-Renyi 5e6 edges + Chung-Lu beta=2.5 mean degree 10 (5e6 edges), "
                "weights uniform in {-1,+1}, C=-L/4, diag(X)=1, rank 20"),
    "er_1k": (["er_1k"], "maxcut n=1e3 Erdos-Renyi 5e3 edges, unit weights, C=-L/4, diag(X)=1, rank 10"),
    "cl_50m": (["cl_50m"], "maxcut n=5e7 Chung-Lu beta=2.5 mean degree 4 (1e8 edges), unit weights, C=-L/4, "
                           "diag(X)=1, rank 26 (held out from the warm-start training graphs)"),
}
DEFAULT_PATHS = "f32_warm,f32_precond_warm"
ALL_PATHS = ["f32_warm", "f32_precond_warm", "f32", "f32_precond", "f32_bf16in", "f64_precond", "f64_input_order",
             "f64_dynrank", "f64_reopt", "f64_reopt2", "f32_dynrank_precond"]
DYNRANK_LD = {0: 30, 1: 32}       # row stride with room for the grown rank (FP64, FP32)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed solves at most (as many as fit the budget run)")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up solves, each capped at --warmup-iters")
    ap.add_argument("--warmup-iters", type=int, default=20)
    ap.add_argument("--budget", type=float, default=540.0,
                    help="wall-clock budget of the whole run in seconds, from process start")
    ap.add_argument("--workload", default="cl_10m", choices=sorted(WORKLOADS))
    ap.add_argument("--instances", default=None, help="comma list of named instances (overrides --workload)")
    ap.add_argument("--paths", default=DEFAULT_PATHS,
                    help="comparison paths run after the timed steps in the time left (comma list of: "
                         + ", ".join(ALL_PATHS) + ")")
    ap.add_argument("--path-limit", type=float, default=None,
                    help="time limit of each comparison-path solve in seconds (default: the budget left)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--cert", action="store_true", help="dual certificate of every result (untimed)")
    ap.add_argument("--cert-iters", type=int, default=600)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--short", type=int, default=0,
                    help="profiling aid: cap each solve at this many L-BFGS iterations (first ALM step only)")
    ap.add_argument("--completion", action="store_true",
                    help="instead of the MaxCut step: time the matrix-completion kernels (SDDMM constraint map, "
                         "gradient SpMM) and 300 L-BFGS iterations at n1 = n2 = 5e5, m = 1e7, rank 16")
    ap.add_argument("--completion-solve", type=float, default=0.0,
                    help="with --completion: also solve to 1e-5 at the factor rank and at the planted rank, in "
                         "float64 and float32, each with this time limit in seconds")
    ap.add_argument("--general-dense", action="store_true",
                    help="instead of the MaxCut step: the general path with C stored dense (n = 8192, every "
                         "upper-triangle entry N(0, 1), diag(X) = 1, rank 24): the C - A*(y) SpMM, whose dense "
                         "product runs on float64 matrix cores, and a solve to 1e-5, in float64")
    ap.add_argument("--general", action="store_true",
                    help="instead of the MaxCut step: time the general-problem kernels (compressed constraint map, "
                         "C - A*(y) SpMM) and a full solve of a general SDP with n = 1e6 (diag(X) = 1 plus 1000 "
                         "side constraints, 5e6 random objective entries, rank 16)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy three times (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(f"[bench {time.perf_counter() - T_START:7.1f}s]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); nothing here uses a "
              "second GPU, so run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2407_15049_amd import lrsdp as L
    from synth import init_factor, maxcut_instance

    dev = torch.device("cuda", 0)
    ctx = L.Context(0)
    if args.completion:
        return completion_bench(args, ctx, dev)
    if args.general:
        return general_bench(args, ctx, dev)
    if args.general_dense:
        return general_dense_bench(args, ctx, dev)

    def left():
        return args.budget - (time.perf_counter() - T_START)

    if args.instances:
        names = args.instances.split(",")
        known = {tuple(v[0]): (k, v[1]) for k, v in WORKLOADS.items()}
        wl_name, wl_desc = known.get(tuple(names), (",".join(names), ",".join(names)))
    else:
        names, wl_desc = WORKLOADS[args.workload]
        wl_name = args.workload
    runs = []
    for name in names:
        t0 = time.perf_counter()
        inst = maxcut_instance(name)
        t1 = time.perf_counter()
        n, r = inst["n"], inst["rank"]
        # nodes relabelled by degree inside the library (R, y stay in the graph's labels)
        prob = L.Problem.maxcut(n, inst["u"], inst["v"], inst["w"], node_order=L.ORDER_DEGREE)
        t2 = time.perf_counter()
        prob.upload(ctx)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        R0 = init_factor(n, r, inst["seed"] + 1)
        ld = L.padded_ld(r, L.F64)
        R0d = torch.zeros((n, ld), dtype=torch.float64, device=dev)
        R0d[:, :r] = torch.from_numpy(R0).to(dev)
        del R0
        opts = L.default_options(prec=L.F64, rank=r, ld=ld, profile=1, verbose=int(args.verbose))
        if args.short:
            opts.max_outer, opts.max_inner = 1, args.short
        # R, y and the workspace of the float64 path are allocated at its first solve
        per = {L.F64: dict(opts=opts, R0=R0d, R=None, y=None, ws=None)}
        info = prob.info
        runs.append(dict(name=name, inst=inst, prob=prob, per=per, n=n, r=r, nnz=info.nnz,
                         setup=dict(generate_s=round(t1 - t0, 2), build_s=round(t2 - t1, 2),
                                    upload_s=round(t3 - t2, 2))))
        log(f"{name}: n={n} nnz={info.nnz} max_row={info.max_row_nnz} generate {t1 - t0:.1f}s "
            f"build {t2 - t1:.1f}s upload {t3 - t2:.1f}s")
    torch.cuda.synchronize()

    def solve(run, prec, opts=None, limit=None, R_init=None, y_init=None, ws=None):
        """One solve of `run` in `prec` from its starting factor (or R_init / y_init),
        stopped by the solver's own time limit when `limit` is given."""
        p = run["per"][prec]
        if p["R"] is None:
            p["R"] = torch.empty_like(p["R0"])
            p["y"] = torch.zeros(run["n"], dtype=torch.float64, device=dev)
            p["ws"] = torch.empty(L.workspace_bytes(run["prob"], p["opts"]), dtype=torch.uint8, device=dev)
        o = opts if opts is not None else p["opts"]
        if limit is not None:
            o.time_limit_s = max(1.0, limit)
        if ws is None and p["ws"].numel() < L.workspace_bytes(run["prob"], o):
            # options that need more workspace (row-block H0): a larger buffer, allocated outside the timing
            p["ws"] = None
            p["ws"] = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
        p["R"].copy_(p["R0"] if R_init is None else R_init)
        if y_init is None:
            p["y"].zero_()
        else:
            p["y"].copy_(y_init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = L.solve(ctx, run["prob"], p["R"], p["y"], o, workspace=p["ws"] if ws is None else ws)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, rc, res

    # ---- warm-up: short capped solves (kernels loaded, clocks up)
    warm_opts = {}
    for w in range(args.warmup):
        for run in runs:
            p = run["per"][L.F64]
            o = L.default_options(prec=L.F64, rank=run["r"], ld=p["opts"].ld, max_outer=1,
                                  max_inner=args.warmup_iters)
            warm_opts[run["name"]] = o
            dt, rc, res = solve(run, L.F64, opts=o)
            log(f"warm-up {w} {run['name']}: {res.inner} iterations {dt:.2f}s")

    # ---- timed steps: full float64 solves, as many as fit
    reserve_cpu = 0.0 if args.no_cpu_baseline else args.cpu_seconds + 15.0
    enabled = [q for q in args.paths.split(",") if q] if args.paths else []
    step_times, recs = [], {run["name"]: [] for run in runs}
    for s in range(args.steps):
        if step_times:
            # keep room for the comparison path (about half a float64 solve) and the CPU sample
            need = step_times[-1] + (0.5 * step_times[0] if enabled else 0.0) + reserve_cpu + 10.0
            if need > left():
                log(f"budget: {left():.0f}s left, a further step needs about {need:.0f}s; {s} step(s) timed")
                break
        limit = left() - reserve_cpu - 10.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for run in runs:
            dt, rc, res = solve(run, L.F64, limit=limit / len(runs))
            recs[run["name"]].append((dt, rc, res))
            log(f"step {s} {run['name']}: {dt:.2f}s rc {rc} outer {res.outer} inner {res.inner} "
                f"obj {res.obj:.10e} err1 {res.err1:.2e} err3 {res.err3:.2e}")
        torch.cuda.synchronize()
        step_times.append(time.perf_counter() - t0)
    ms_per_step = 1000.0 * sum(step_times) / len(step_times) if step_times else None
    converged = all(rc == L.OK for v in recs.values() for _, rc, _ in v)

    # ---- SpMM roofline from the HIP events of the timed solves
    allres = [res for v in recs.values() for _, _, res in v]
    spmm_ms = sum(res.spmm_ms for res in allres)
    spmm_n = sum(res.spmm_launches for res in allres)
    spmm_bytes = sum(res.spmm_bytes * res.spmm_launches for res in allres)
    achieved = (spmm_bytes / 1e9) / (spmm_ms / 1e3) if spmm_ms > 0 else None
    traffic = measured_traffic(wl_name)

    paths = {"f64": {}}
    for run in runs:
        if not recs[run["name"]]:
            continue
        dt, rc, res = recs[run["name"]][-1]
        rec = dict(seconds=round(dt, 3), converged=rc == L.OK, outer=res.outer, inner=res.inner, obj=res.obj,
                   err1=res.err1, err1_inf=res.err1_inf, err3=res.err3,
                   ms_per_iter=round(1e3 * dt / max(res.inner, 1), 3),
                   spmm_us=round(1e3 * res.spmm_ms / max(res.spmm_launches, 1), 2),
                   all_seconds=[round(d, 3) for d, _, _ in recs[run["name"]]])
        paths["f64"][run["name"]] = rec

    copy_gbs = copy_ceiling(torch, dev, args.copy_calibration) if step_times else None

    comparison_paths(args, ctx, dev, L, runs, paths, enabled, left, reserve_cpu, solve, log)
    if args.cert:   # the FP64 step's multipliers (the comparison paths certify their own)
        for run in runs:
            rec = paths["f64"].get(run["name"])
            if rec and run["per"][L.F64]["y"] is not None and left() > reserve_cpu + 20:
                rec.update(cert_of(args, ctx, dev, L, run, run["per"][L.F64]["y"], rec["obj"]))

    cpu = None
    if not args.no_cpu_baseline and step_times:
        cpu = cpu_baseline(runs, recs, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(ms_per_step / 1000.0, 3) if ms_per_step else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": len(step_times),
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 1) if ms_per_step else None,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl_desc, "name": wl_name, "instances": names, "tol": 1e-5,
                   "path": "plain FP64 ALM + L-BFGS (H0 = I), exact line search",
                   "node_order": "degree (relabelled inside the library; R and y in the graph's labels)",
                   "lbfgs_mem": runs[0]["per"][L.F64]["opts"].lbfgs_mem, "converged": converged,
                   "steps_requested": args.steps, "warmup_iters": args.warmup_iters, "budget_s": args.budget,
                   "setup": {run["name"]: run["setup"] for run in runs}},
        "step_seconds": [round(t, 3) for t in step_times],
        "roofline": {
            "kernel": "spmm (MaxCut, line-search epilogue)",
            "bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
            "traffic_note": ("HBM-side bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the stored "
                             "counter summary of this workload; it counts L2 misses, MALL hits included"
                             if traffic else "no counter summary matching the current SpMM sources"),
            "launches": spmm_n,
            "avg_us": round(1e3 * spmm_ms / max(spmm_n, 1), 2),
            "alg_bytes_per_launch": {run["name"]: recs[run["name"]][-1][2].spmm_bytes for run in runs
                                     if recs[run["name"]]},
            "copy_ceiling_gbs": copy_gbs,
        },
        "cpu_baseline": cpu,
        "paths": paths,
        "wall_s": round(time.perf_counter() - T_START, 1),
    }
    print(json.dumps(out), flush=True)


def copy_ceiling(torch, dev, calibration_copies):
    """Read + write bytes of a 1 GiB device-to-device copy over its HIP-event time
    (median of 10): the box's copy ceiling.  With calibration_copies, three more
    untimed copies for the counter calibration of a profiled run."""
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev)
    for _ in range(3 if calibration_copies else 1):
        b.copy_(a)
    times = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    del a, b
    gbs = round(2.0 * (1 << 30) / 1e9 / sorted(times)[len(times) // 2], 1)
    log(f"copy ceiling: {gbs} GB/s")
    return gbs


def comparison_paths(args, ctx, dev, L, runs, paths, enabled, left, reserve_cpu, solve, log):
    """Untimed-by-the-step paths on the same graphs, each one solve with a time
    limit from what is left of the budget."""
    import torch
    if not enabled:
        return

    def budget_for_path():
        b = left() - reserve_cpu - 10.0
        return min(b, args.path_limit) if args.path_limit else b

    def record(path, run, dt, rc, res, extra=None, y=None):
        o64 = paths["f64"].get(run["name"], {}).get("obj")
        rec = dict(seconds=round(dt, 3), converged=rc == L.OK, outer=res.outer, inner=res.inner, obj=res.obj,
                   err1=res.err1, err3=res.err3, obj_rel_vs_f64=abs(res.obj - o64) / abs(o64) if o64 else None,
                   ms_per_iter=round(1e3 * dt / max(res.inner, 1), 3),
                   spmm_us=round(1e3 * res.spmm_ms / max(res.spmm_launches, 1), 2))
        rec.update(extra or {})
        if args.cert and y is not None and not args.short:
            rec.update(cert_of(args, ctx, dev, L, run, y, res.obj))
        paths.setdefault(path, {})[run["name"]] = rec
        log(f"{path} {run['name']} {dt:.2f}s rc {rc} outer {res.outer} inner {res.inner} obj {res.obj:.10e}")

    def ensure_f32(run):
        if L.F32 in run["per"]:
            return run["per"][L.F32]
        n, r = run["n"], run["r"]
        ld = L.padded_ld(r, L.F32)
        o = L.default_options(prec=L.F32, rank=r, ld=ld, profile=1, verbose=int(args.verbose))
        R0 = torch.zeros((n, ld), dtype=torch.float32, device=dev)
        R0[:, :r] = run["per"][L.F64]["R0"][:, :r].to(torch.float32)
        run["per"][L.F32] = dict(opts=o, R0=R0, R=torch.empty_like(R0),
                                 y=torch.zeros(n, dtype=torch.float64, device=dev),
                                 ws=torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev))
        return run["per"][L.F32]

    def opts_for(run, prec, **kw):
        p = run["per"][prec]
        o = L.default_options(prec=prec, rank=run["r"], ld=p["opts"].ld, profile=1,
                              verbose=int(args.verbose), **kw)
        if args.short:
            o.max_outer, o.max_inner = 1, args.short
        return o

    model = None
    for path in enabled:
        if path not in ALL_PATHS:
            raise SystemExit(f"unknown path {path}")
        for run in runs:
            if budget_for_path() < 20.0:
                paths.setdefault(path, {})[run["name"]] = dict(skipped=f"budget: {left():.0f}s left")
                log(f"{path} {run['name']}: skipped, {left():.0f}s left")
                continue
            lim = budget_for_path()
            if path in ("f32_warm", "f32_precond_warm"):
                from paper_2407_15049_amd import warmstart as W
                if model is None:
                    model = W.load_model(dev)
                if model is None:
                    paths.setdefault(path, {})[run["name"]] = dict(skipped="no trained warm-start model in the tree")
                    continue
                p = ensure_f32(run)
                o = opts_for(run, L.F32, precond=1 if path == "f32_precond_warm" else 0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()                 # features + inference count toward the solve
                y0, sigma0 = W.warm_start(ctx, run["prob"], model)
                o.sigma0 = sigma0
                dt, rc, res = solve(run, L.F32, opts=o, limit=lim - (time.perf_counter() - t0), y_init=y0)
                dt = time.perf_counter() - t0
                record(path, run, dt, rc, res, dict(sigma0=sigma0, model=model.meta.get("name")), y=p["y"])
            elif path in ("f32", "f32_precond", "f32_bf16in"):
                p = ensure_f32(run)
                kw = dict(precond=1) if path == "f32_precond" else {}
                if path == "f32_bf16in":
                    o = L.default_options(prec=L.F32_BF16IN, rank=run["r"], ld=p["opts"].ld, profile=1,
                                          refresh_every=25)
                    ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
                    dt, rc, res = solve(run, L.F32, opts=o, limit=lim, ws=ws)
                    del ws
                else:
                    dt, rc, res = solve(run, L.F32, opts=opts_for(run, L.F32, **kw), limit=lim)
                record(path, run, dt, rc, res, y=p["y"])
            elif path in ("f64_precond", "f64_reopt", "f64_reopt2"):
                kw = {"f64_precond": dict(precond=1), "f64_reopt": dict(reopt=1), "f64_reopt2": dict(reopt=2)}[path]
                o = opts_for(run, L.F64, **kw)
                ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
                dt, rc, res = solve(run, L.F64, opts=o, limit=lim, ws=ws)
                del ws
                extra = dict(reopt_rounds=res.reopt_rounds) if "reopt" in path else None
                record(path, run, dt, rc, res, extra, y=run["per"][L.F64]["y"])
            elif path in ("f64_dynrank", "f32_dynrank_precond"):
                prec = L.F64 if path == "f64_dynrank" else L.F32
                if prec == L.F32:
                    ensure_f32(run)
                ld = DYNRANK_LD[0 if prec == L.F64 else 1]
                o = L.default_options(prec=prec, rank=run["r"], ld=ld, profile=1, rank_max=ld,
                                      verbose=int(args.verbose), precond=1 if prec == L.F32 else 0)
                o.time_limit_s = max(1.0, lim)
                ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
                R = torch.zeros((run["n"], ld), dtype=L.elem_dtype(prec), device=dev)
                R[:, :run["r"]] = run["per"][prec]["R0"][:, :run["r"]]
                y = torch.zeros(run["n"], dtype=torch.float64, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, res = L.solve(ctx, run["prob"], R, y, o, workspace=ws)
                torch.cuda.synchronize()
                record(path, run, time.perf_counter() - t0, rc, res, dict(rank_final=res.rank_final), y=y)
                del ws, R
            elif path == "f64_input_order":
                # the same graph built in the caller's node order (no relabelling by degree)
                inst, n = run["inst"], run["n"]
                prob2 = L.Problem.maxcut(n, inst["u"], inst["v"], inst["w"]).upload(ctx)
                o = opts_for(run, L.F64)
                o.time_limit_s = max(1.0, lim)
                ws = torch.empty(L.workspace_bytes(prob2, o), dtype=torch.uint8, device=dev)
                R = run["per"][L.F64]["R0"].clone()
                y = torch.zeros(n, dtype=torch.float64, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, res = L.solve(ctx, prob2, R, y, o, workspace=ws)
                torch.cuda.synchronize()
                record(path, run, time.perf_counter() - t0, rc, res, y=y)
                del prob2, ws, R, y


def cert_of(args, ctx, dev, L, run, y, obj):
    """Dual estimate of the multipliers y by block Lanczos (outside every timed
    region): lambda_min is a Ritz value, the bound subtracts its residual."""
    import torch
    torch.cuda.synchronize()
    work = torch.empty(L.certify_workspace_bytes(run["prob"], args.cert_iters), dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    c = L.certify(ctx, run["prob"], y, max_iter=args.cert_iters, tol=1e-8 * abs(obj) / run["n"], work=work)
    dt = time.perf_counter() - t0
    gap = (obj - c.dual_bound) / (1.0 + abs(obj) + abs(c.dual_bound))
    out = dict(lambda_min=c.lambda_min, lambda_max_ritz=c.lambda_max, cert_resid=c.resid,
               cert_resid_rel=c.resid / max(abs(c.lambda_min), abs(c.lambda_max), 1e-300),
               dual_bound_est=c.dual_bound, gap_est=gap, err2=c.err2, cert_iters=c.iters, cert_status=c.status,
               cert_s=round(dt, 3))
    if run["n"] <= L.PROOF_MAX_N:
        # small problems: prove the bound (host Cholesky of S - shift I) a little below the estimate
        shift = c.lambda_lb - 1e-7 * max(abs(c.lambda_min), abs(c.lambda_max), 1.0)
        t0 = time.perf_counter()
        p = L.certify_dense(run["prob"], y.cpu().numpy(), shift)
        out.update(proof_status=p.status, proof_lambda_lb=p.lambda_lb, proof_dual_bound=p.dual_bound,
                   proof_gap=(obj - p.dual_bound) / (1.0 + abs(obj) + abs(p.dual_bound)) if p.status == 0 else None,
                   proof_s=round(time.perf_counter() - t0, 3))
    return out


TRAFFIC_PROFILES = {
    "cl_10m": "spmm_maxcut_traffic_cl_10m_f64.md",
}
SPMM_SOURCES = [os.path.join(ROOT, "paper_2407_15049_amd", "csrc", f)
                for f in ("spmm_maxcut.hip", "device.h", "kernels.h")]


def measured_traffic(workload):
    """HBM bytes per SpMM launch from the committed counter summary of this
    workload, or None when there is none or the SpMM sources changed since the
    counters were taken."""
    import hashlib
    if workload not in TRAFFIC_PROFILES:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", TRAFFIC_PROFILES[workload])).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("source_sha256: ", "traffic_bytes_per_launch: ")))
    h = hashlib.sha256()
    for f in SPMM_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch"])


COMPLETION = dict(n1=500_000, n2=500_000, k=5, per_row=20, rank=16, seed=15051)


def completion_bench(args, ctx, dev):
    """Kernel bandwidth of the completion hot path (SDDMM constraint map, gradient
    SpMM) with HIP events on the library's stream, and the time of 300 L-BFGS
    iterations of the solve, in float64 and float32."""
    import numpy as np
    import torch

    from paper_2407_15049_amd import lrsdp as L
    from synth.graphs import completion_instance, gaussian_factor

    cfg = COMPLETION
    t0 = time.perf_counter()
    i, j, M, U, V = completion_instance(cfg["n1"], cfg["n2"], cfg["k"], cfg["per_row"], cfg["seed"])
    prob = L.Problem.completion(cfg["n1"], cfg["n2"], i, j, M).upload(ctx)
    n, m, r = prob.info.n, prob.info.m, cfg["rank"]
    log(f"completion n={n} m={m} setup {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.current_stream(dev)
    out = {}
    reps = 20
    for prec, name in [(L.F64, "f64"), (L.F32, "f32")]:
        ld = L.padded_ld(r, prec)
        w = 8 if prec == L.F64 else 4
        R = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=dev)
        R[:, :r] = torch.from_numpy(gaussian_factor(n, r, 1.0 / math.sqrt(r), cfg["seed"] + 1)).to(dev, R.dtype)
        y = torch.from_numpy(np.random.default_rng(cfg["seed"] + 2).standard_normal(m) * 0.1).to(dev)
        acon = torch.empty(m, dtype=torch.float64, device=dev)
        Y = torch.empty_like(R)

        def timed(fn):
            for _ in range(3):
                fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(reps):
                fn()
            ev[1].record(stream)
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]) * 1e3 / reps      # us per launch

        t_sdd = timed(lambda: L.k_constraint(ctx, prob, prec, R, R, acon))
        t_spmm = timed(lambda: L.k_spmm(ctx, prob, prec, R, y, Y))
        b_sdd = 4.0 * (cfg["n1"] + 1) + 4.0 * m + n * ld * w + 8.0 * m
        b_spmm = 4.0 * (n + 2) + 4.0 * m + 8.0 * m + 16.0 * m + 2.0 * n * ld * w
        opts = L.default_options(prec=prec, rank=r, ld=ld, max_iter_total=300, max_inner=300, max_outer=1,
                                 eta0=1e-12)          # no early inner stop: 300 full iterations
        R0 = R.clone()
        y0 = torch.zeros(m, dtype=torch.float64, device=dev)
        ws = torch.empty(L.workspace_bytes(prob, opts), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc, res = L.solve(ctx, prob, R0, y0, opts, workspace=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        out[name] = dict(
            sddmm_us=round(t_sdd, 2), sddmm_alg_bytes=b_sdd, sddmm_gbs=round(b_sdd / t_sdd / 1e3, 1),
            sddmm_frac=round(b_sdd / t_sdd / 1e3 / HBM_PEAK_GBS, 4),
            spmm_us=round(t_spmm, 2), spmm_alg_bytes=b_spmm, spmm_gbs=round(b_spmm / t_spmm / 1e3, 1),
            spmm_frac=round(b_spmm / t_spmm / 1e3 / HBM_PEAK_GBS, 4),
            iters=res.inner, ms_per_iter=round(1e3 * dt / max(res.inner, 1), 3), err1=res.err1)
        log(f"completion {name}: {out[name]}")
        del R, Y, R0, ws
    solves = completion_solves(args, ctx, dev, L, prob, cfg, U, V) if args.completion_solve > 0 else None
    copy_gbs = copy_ceiling(torch, dev, args.copy_calibration)
    print(json.dumps({
        "metric": "completion kernels: SDDMM / SpMM algorithmic GB/s and L-BFGS ms per iteration",
        "unit": "GB/s", "n_gpus": 1, "dtype": "f64,f32", "data": "synthetic",
        "config": {"workload": "matrix completion n1=n2=5e5 (X of order 1e6), m=1e7 samples (20 per row), "
                               "planted rank 5, factor rank 16", **cfg},
        "kernels": out, "solves": solves, "copy_ceiling_gbs": copy_gbs}), flush=True)


def completion_solves(args, ctx, dev, L, prob, cfg, U, V):
    """Time to 1e-5 of the completion SDP at the factor rank and at the planted
    rank, float64 and float32, from the seeded Gaussian start; with the
    recovery error of the planted M = U V^T on 100,000 seeded positions (most
    of them unobserved): ||(R_top R_bot^T - M)_S|| / ||M_S||."""
    import numpy as np
    import torch
    from synth.graphs import gaussian_factor
    n, m = prob.info.n, prob.info.m
    g = np.random.default_rng(cfg["seed"] + 7)
    si = g.integers(0, cfg["n1"], 100_000)
    sj = g.integers(0, cfg["n2"], 100_000)
    want = np.einsum("ij,ij->i", U[si], V[sj])
    res_all = {}
    for r in (cfg["rank"], cfg["k"]):
        for prec, name in [(L.F64, "f64"), (L.F32, "f32")]:
            ld = L.padded_ld(r, prec)
            R = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=dev)
            R[:, :r] = torch.from_numpy(gaussian_factor(n, r, 1.0 / math.sqrt(r), cfg["seed"] + 1)).to(dev, R.dtype)
            y = torch.zeros(m, dtype=torch.float64, device=dev)
            opts = L.default_options(prec=prec, rank=r, ld=ld)
            opts.time_limit_s = args.completion_solve
            ws = torch.empty(L.workspace_bytes(prob, opts), dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rc, res = L.solve(ctx, prob, R, y, opts, workspace=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            Rh = R[:, :r].double().cpu().numpy()
            got = np.einsum("ij,ij->i", Rh[si], Rh[cfg["n1"] + sj])
            rec = float(np.linalg.norm(got - want) / np.linalg.norm(want))
            key = f"{name}_rank{r}"
            res_all[key] = dict(seconds=round(dt, 3), converged=rc == L.OK, outer=res.outer, inner=res.inner,
                                obj=res.obj, err1=res.err1, err3=res.err3,
                                ms_per_iter=round(1e3 * dt / max(res.inner, 1), 3), recovery_rel_err=rec)
            log(f"completion solve {key}: {res_all[key]}")
            del R, y, ws
    return res_all


GENERAL = dict(n=1_000_000, c_nnz=5_000_000, extra=1000, per_con=5, rank=16, seed=15052)


def general_instance(cfg):
    """Triplets of the general benchmark SDP: a symmetric objective with c_nnz
    N(0, 1) entries at uniform positions, diag(X) = 1, and `extra` side
    constraints on `per_con` off-diagonal positions each with N(0, 1)
    coefficients and right-hand side 0 (X = I is feasible)."""
    import numpy as np
    g = np.random.Generator(np.random.PCG64(cfg["seed"]))
    n = cfg["n"]
    c_row = g.integers(0, n, cfg["c_nnz"]).astype(np.int32)
    c_col = g.integers(0, n, cfg["c_nnz"]).astype(np.int32)
    c_val = g.standard_normal(cfg["c_nnz"])
    k = np.repeat(np.arange(n, n + cfg["extra"], dtype=np.int32), cfg["per_con"])
    rr = g.integers(0, n, k.size).astype(np.int32)
    cc = ((rr + 1 + g.integers(0, n - 1, k.size)) % n).astype(np.int32)     # off the diagonal
    diag = np.arange(n, dtype=np.int32)
    a_con = np.concatenate([diag, k])
    a_row = np.concatenate([diag, rr])
    a_col = np.concatenate([diag, cc])
    a_val = np.concatenate([np.ones(n), g.standard_normal(k.size)])
    m = n + cfg["extra"]
    b = np.concatenate([np.ones(n), np.zeros(cfg["extra"])])
    return c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b


def general_bench(args, ctx, dev):
    """Kernel bandwidth of the general-problem path (compressed outer product +
    constraint rows, C - A*(y) SpMM on Omega) with HIP events on the library's
    stream, and a full solve to 1e-5, in float64 and float32."""
    import numpy as np
    import torch

    from paper_2407_15049_amd import lrsdp as L
    from synth import init_factor

    cfg = GENERAL
    t0 = time.perf_counter()
    prob = L.Problem.general(cfg["n"], *general_instance(cfg)).upload(ctx)
    inf = prob.info
    n, m, r, nnz_s = inf.n, inf.m, cfg["rank"], inf.nnz
    nom = (nnz_s + n) // 2                  # positions: each off-diagonal one is stored twice, all n diagonals once
    nnz_a = n + cfg["extra"] * cfg["per_con"]
    log(f"general n={n} m={m} |Omega|={nom} symmetric nnz={nnz_s} setup {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.current_stream(dev)
    out = {}
    reps = 20
    for prec, name in [(L.F64, "f64"), (L.F32, "f32")]:
        ld = L.padded_ld(r, prec)
        w = 8 if prec == L.F64 else 4
        R = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=dev)
        R[:, :r] = torch.from_numpy(init_factor(n, r, cfg["seed"] + 1)).to(dev, R.dtype)
        y = torch.from_numpy(np.random.default_rng(cfg["seed"] + 2).standard_normal(m) * 0.1).to(dev)
        acon = torch.empty(m, dtype=torch.float64, device=dev)
        Y = torch.empty_like(R)

        def timed(fn):
            for _ in range(3):
                fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(reps):
                fn()
            ev[1].record(stream)
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]) * 1e3 / reps      # us per launch

        t_map = timed(lambda: L.k_constraint(ctx, prob, prec, R, R, acon))
        t_spmm = timed(lambda: L.k_spmm(ctx, prob, prec, R, y, Y))
        # algorithmic bytes: every array once, R read once
        b_map = 8.0 * nom + 8.0 * nom + n * ld * w + 4.0 * (m + 1) + 12.0 * nnz_a + 8.0 * nom + 8.0 * m
        b_spmm = (4.0 * (n + 1) + 8.0 * nnz_s + 8.0 * nom + 4.0 * (nom + 1) + 12.0 * nnz_a + 8.0 * m
                  + 2.0 * n * ld * w)
        opts = L.default_options(prec=prec, rank=r, ld=ld, time_limit_s=120.0)
        R0 = R.clone()
        y0 = torch.zeros(m, dtype=torch.float64, device=dev)
        ws = torch.empty(L.workspace_bytes(prob, opts), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc, res = L.solve(ctx, prob, R0, y0, opts, workspace=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        out[name] = dict(
            map_us=round(t_map, 2), map_alg_bytes=b_map, map_gbs=round(b_map / t_map / 1e3, 1),
            map_frac=round(b_map / t_map / 1e3 / HBM_PEAK_GBS, 4),
            spmm_us=round(t_spmm, 2), spmm_alg_bytes=b_spmm, spmm_gbs=round(b_spmm / t_spmm / 1e3, 1),
            spmm_frac=round(b_spmm / t_spmm / 1e3 / HBM_PEAK_GBS, 4),
            solve_s=round(dt, 3), converged=rc == L.OK, outer=res.outer, iters=res.inner,
            ms_per_iter=round(1e3 * dt / max(res.inner, 1), 3), obj=res.obj, err1=res.err1, err3=res.err3)
        log(f"general {name}: {out[name]}")
        del R, Y, R0, ws
    print(json.dumps({
        "metric": "general SDP: compressed constraint map / C - A*(y) SpMM algorithmic GB/s and time to 1e-5",
        "unit": "GB/s", "n_gpus": 1, "dtype": "f64,f32", "data": "synthetic",
        "config": {"workload": "general SDP n=1e6: 5e6 random N(0,1) objective entries, diag(X)=1 plus 1000 "
                               "side constraints on 5 off-diagonal positions each (b = 0), rank 16", **cfg},
        "kernels": out}), flush=True)


GENERAL_DENSE = dict(n=8192, rank=24, seed=15053)


def general_dense_bench(args, ctx, dev):
    """The general path with C stored dense: HIP-event time of lrsdp_k_spmm
    (dense product W = C V on float64 matrix cores, then the sparse part and the
    split-k finish) and a float64 solve to 1e-5.  The instance is the SDP
    relaxation of a dense +-spin problem: C with every upper-triangle entry
    N(0, 1), diag(X) = 1."""
    import numpy as np
    import torch

    from paper_2407_15049_amd import lrsdp as L
    from synth import init_factor

    cfg = GENERAL_DENSE
    n, r = cfg["n"], cfg["rank"]
    t0 = time.perf_counter()
    g = np.random.Generator(np.random.PCG64(cfg["seed"]))
    c_row, c_col = np.triu_indices(n)
    c_val = g.standard_normal(c_row.size)
    diag = np.arange(n, dtype=np.int32)
    prob = L.Problem.general(n, c_row.astype(np.int32), c_col.astype(np.int32), c_val, n, diag, diag, diag,
                             np.ones(n), np.ones(n), c_storage=L.C_DENSE).upload(ctx)
    del c_row, c_col, c_val
    assert prob.info.c_dense == 1
    log(f"general dense n={n} setup {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.current_stream(dev)
    prec, ld = L.F64, L.padded_ld(r, L.F64)
    R = torch.zeros((n, ld), dtype=torch.float64, device=dev)
    R[:, :r] = torch.from_numpy(init_factor(n, r, cfg["seed"] + 1)).to(dev)
    y = torch.from_numpy(np.random.default_rng(cfg["seed"] + 2).standard_normal(n) * 0.1).to(dev)
    Y = torch.empty_like(R)
    for _ in range(3):
        L.k_spmm(ctx, prob, prec, R, y, Y)
    reps = 50
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(reps):
        L.k_spmm(ctx, prob, prec, R, y, Y)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_spmm = ev[0].elapsed_time(ev[1]) * 1e3 / reps
    # algorithmic: C once (n^2 float64), V read, W and Y written once; flops 2 n^2 r
    b_spmm = 8.0 * n * n + 3.0 * 8.0 * n * ld
    flops = 2.0 * n * n * r
    opts = L.default_options(prec=prec, rank=r, ld=ld, time_limit_s=120.0)
    if args.short:
        opts.max_outer, opts.max_inner = 1, args.short
    y0 = torch.zeros(n, dtype=torch.float64, device=dev)
    ws = torch.empty(L.workspace_bytes(prob, opts), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, res = L.solve(ctx, prob, R, y0, opts, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    out = dict(spmm_us=round(t_spmm, 2), spmm_alg_bytes=b_spmm, spmm_gbs=round(b_spmm / t_spmm / 1e3, 1),
               spmm_frac=round(b_spmm / t_spmm / 1e3 / HBM_PEAK_GBS, 4),
               spmm_tflops=round(flops / t_spmm / 1e6, 2), solve_s=round(dt, 3), converged=rc == L.OK,
               outer=res.outer, iters=res.inner, ms_per_iter=round(1e3 * dt / max(res.inner, 1), 3),
               obj=res.obj, err1=res.err1, err3=res.err3)
    log(f"general dense f64: {out}")
    print(json.dumps({
        "metric": "general SDP with dense C: C - A*(y) SpMM (dense product on matrix cores) and time to 1e-5",
        "unit": "GB/s", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "general SDP n=8192, C dense with N(0,1) upper-triangle entries, diag(X)=1, "
                               "rank 24, C stored dense", **cfg},
        "kernels": {"f64": out}}), flush=True)


def cpu_baseline(runs, recs, target_s):
    """The oracle (numpy/scipy, float64) timed on the host on a bounded sample of
    the workload: per instance, L-BFGS iterations of its first ALM subproblem
    for about target_s seconds in total, on the instance itself when it has at
    most 2e7 stored entries, else on a graph of the same family with a tenth of
    the nodes and edges (time per iteration scaled by the ratio of stored
    entries).  Time per iteration times the iterations of the GPU float64
    solve, summed over the instances: the unit of the step."""
    from threadpoolctl import threadpool_limits

    from oracle.alm import Options, alm_solve
    from oracle.problem import maxcut_problem
    from synth import MAXCUT_CONFIGS, chung_lu_edges, erdos_renyi_edges, init_factor, pm1_weights

    threads = max(1, min(os.cpu_count() or 1, 16))
    total, parts, util = 0.0, [], []
    with threadpool_limits(limits=threads):
        for run in runs:
            inst = run["inst"]
            n, u, v, w, scale, what = inst["n"], inst["u"], inst["v"], inst["w"], 1.0, "the instance itself"
            if run["nnz"] > 20_000_000:
                kind, n0, m0, beta, wk, rank, seed = MAXCUT_CONFIGS[run["name"]]
                n, m = n0 // 10, m0 // 10
                u, v = chung_lu_edges(n, m, beta, seed + 1) if kind == "cl" else erdos_renyi_edges(n, m, seed + 1)
                w = None if wk == "unit" else pm1_weights(m, seed + 7920)
                what = f"a graph of the same family with n={n}, {m} edges"
            t0 = time.perf_counter()
            op = maxcut_problem(n, u, v, w)
            R0 = init_factor(n, inst["rank"], inst["seed"] + 1)
            if n != inst["n"]:
                scale = run["nnz"] / float(op.C.nnz)
            build = time.perf_counter() - t0
            t1 = time.perf_counter()
            alm_solve(op, R0, opts=Options(max_outer=1, max_inner=1))
            one = time.perf_counter() - t1
            k = max(2, int(target_s / len(runs) / max(one, 1e-6)))
            t2, c2 = time.perf_counter(), time.process_time()
            res = alm_solve(op, R0, opts=Options(max_outer=1, max_inner=1 + k))
            wall = time.perf_counter() - t2
            util.append((time.process_time() - c2) / max(wall, 1e-9))
            per_iter = max(wall - one, 1e-9) / max(res.inner - 1, 1) * scale
            gres = recs[run["name"]][-1][2]
            est = per_iter * gres.inner
            total += est
            log(f"cpu oracle {run['name']}: {res.inner} iterations in {wall:.1f}s on {what} "
                f"({per_iter:.3f}s per iteration at full size), estimate for {gres.inner} iterations: {est:.0f}s "
                f"(problem build {build:.1f}s)")
            parts.append(f"{run['name']}: {res.inner - 1} iterations after the first ({wall - one:.1f}s) on {what}"
                         + (f", scaled by the stored-entry ratio {scale:.2f}" if scale != 1.0 else "")
                         + f", times the GPU FP64 solve's {gres.inner} iterations")
            del op
    return {
        "value": round(total, 1),
        "unit": "s",
        "cores": threads,
        "cpu_util": round(sum(util) / len(util), 2),
        "kind": "oracle",
        "sample": ("oracle L-BFGS iterations of the first ALM subproblem (numpy/scipy float64; BLAS pool of "
                   f"{threads} threads, scipy's sparse products on one; cpu_util = process CPU seconds per wall "
                   "second), per instance: " + "; ".join(parts) + "; problem builds not included"),
    }


if __name__ == "__main__":
    main()
