#!/usr/bin/env python3
"""Time to 1e-5 tolerance of the MaxCut SDP hot path on one MI355X.

Workload (one "step"): the 1e6-node MaxCut SDP pair -- an Erdos-Renyi graph
and a Chung-Lu power-law graph (exponent 2.5, mean degree 10), 5e6 edges
each, weights uniform in {-1, +1}, C = -L/4, diag(X) = 1, rank 20 -- each
solved from a seeded unit-row starting factor until err1 <= 1e-5 and
|err3| <= 1e-5 with the plain float64 method.  Problems, starting factors and
workspaces are resident in HBM before the timed region; the timed region is
the solves themselves.  The float32 path is run after the timed region and
reported beside it.

The JSON line carries the SpMM roofline (algorithmic bytes per launch over the
launch duration measured with HIP events on the solve's stream) and the CPU
oracle's time on a bounded sample of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-5 tol: plain FP64 vs FP32+learned warm start; SpMM/SDDMM HBM GB/s"
HBM_PEAK_GBS = 8000.0
WORKLOAD = ("maxcut n=1e6 pair: Erdos-Renyi 5e6 edges + Chung-Lu beta=2.5 mean degree 10 (5e6 edges), "
            "weights uniform in {-1,+1}, C=-L/4, diag(X)=1, rank 20")
INSTANCES = ["er_1m_pm1", "cl_1m_pm1"]
ALL_PATHS = ["f64_degsort", "f64_precond", "f64_dynrank", "f64_reopt", "f64_reopt2", "f32", "f32_precond",
             "f32_bf16in", "f32_warm", "f32_precond_warm", "f32_dynrank_precond"]
DYNRANK_LD = {0: 30, 1: 32}       # row stride with room for the grown rank (FP64, FP32)
OTHER_WORKLOADS = {
    "cl_10m": "maxcut n=1e7 Chung-Lu beta=2.5 mean degree 8 (4e7 edges), unit weights, C=-L/4, diag(X)=1, rank 24",
    "er_1k": "maxcut n=1e3 Erdos-Renyi 5e3 edges, unit weights, C=-L/4, diag(X)=1, rank 10",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the float32 / warm-start / bf16 paths")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm start")
    ap.add_argument("--no-bf16", action="store_true", help="skip the bfloat16-input path")
    ap.add_argument("--no-precond", action="store_true", help="skip the row-block H0 paths")
    ap.add_argument("--paths", default=",".join(ALL_PATHS),
                    help="untimed comparison paths to run after the timed step (comma list)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--instances", default=",".join(INSTANCES))
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--short", type=int, default=0,
                    help="profiling aid: cap each solve at this many L-BFGS iterations (first ALM step only)")
    ap.add_argument("--completion", action="store_true",
                    help="instead of the MaxCut step: time the matrix-completion kernels (SDDMM constraint map, "
                         "gradient SpMM) and 300 L-BFGS iterations at n1 = n2 = 5e5, m = 1e7, rank 16")
    ap.add_argument("--general", action="store_true",
                    help="instead of the MaxCut step: time the general-problem kernels (compressed constraint map, "
                         "C - A*(y) SpMM) and a full solve of a general SDP with n = 1e6 (diag(X) = 1 plus 1000 "
                         "side constraints, 5e6 random objective entries, rank 16)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy three times (counter calibration)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "spmm_maxcut_traffic_pair_1m_f64.md")
SPMM_SOURCES = [os.path.join(ROOT, "paper_2407_15049_amd", "csrc", f)
                for f in ("spmm_maxcut.hip", "device.h", "kernels.h")]


def measured_traffic():
    """HBM bytes per SpMM launch from the committed counter summary, or None when
    the SpMM sources changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
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
    names = args.instances.split(",")
    runs = []
    for name in names:
        t0 = time.perf_counter()
        inst = maxcut_instance(name)
        n, r = inst["n"], inst["rank"]
        prob = L.Problem.maxcut(n, inst["u"], inst["v"], inst["w"]).upload(ctx)
        R0 = init_factor(n, r, inst["seed"] + 1)
        per = {}
        for prec in ([L.F64] if args.no_f32 else [L.F64, L.F32]):
            ld = L.padded_ld(r, prec)
            opts = L.default_options(prec=prec, rank=r, ld=ld, profile=1, verbose=int(args.verbose))
            if args.short:
                opts.max_outer, opts.max_inner = 1, args.short
            R0d = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=dev)
            R0d[:, :r] = torch.from_numpy(R0).to(dev, R0d.dtype)
            per[prec] = dict(
                opts=opts, R0=R0d, R=torch.empty_like(R0d),
                y=torch.zeros(n, dtype=torch.float64, device=dev),
                ws=torch.empty(L.workspace_bytes(prob, opts), dtype=torch.uint8, device=dev))
        info = prob.info
        runs.append(dict(name=name, inst=inst, prob=prob, per=per, n=n, r=r, nnz=info.nnz))
        log(f"{name}: n={n} nnz={info.nnz} max_row={info.max_row_nnz} setup {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()

    def solve(run, prec):
        p = run["per"][prec]
        p["R"].copy_(p["R0"])
        p["y"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = L.solve(ctx, run["prob"], p["R"], p["y"], p["opts"], workspace=p["ws"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != L.OK and not args.short:
            raise RuntimeError(f"{run['name']} prec {prec} did not converge: {res.as_dict()}")
        return dt, res

    cert_ws = {}

    def cert_of(run, y, obj):
        """Dual certificate of the multipliers y (outside every timed region)."""
        if run["name"] not in cert_ws:
            cert_ws[run["name"]] = torch.empty(L.certify_workspace_bytes(run["prob"], 600), dtype=torch.uint8,
                                               device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = L.certify(ctx, run["prob"], y, max_iter=600, tol=1e-8 * abs(obj) / run["n"],
                      work=cert_ws[run["name"]])
        dt = time.perf_counter() - t0
        gap = (obj - c.dual_bound) / (1.0 + abs(obj) + abs(c.dual_bound))
        return dict(lambda_min=c.lambda_min, cert_resid=c.resid, dual_bound=c.dual_bound, cert_gap=gap,
                    err2=c.err2, cert_iters=c.iters, cert_s=round(dt, 4))

    for w in range(args.warmup):
        for run in runs:
            dt, res = solve(run, L.F64)
            log(f"warmup {w} {run['name']} f64 {dt:.3f}s outer {res.outer} inner {res.inner}")

    step_times, recs = [], {run["name"]: [] for run in runs}
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for run in runs:
            dt, res = solve(run, L.F64)
            recs[run["name"]].append((dt, res))
        torch.cuda.synchronize()
        step_times.append(time.perf_counter() - t0)
        log(f"step {s}: {step_times[-1]:.3f}s")
    ms_per_step = 1000.0 * sum(step_times) / len(step_times) if step_times else None

    # SpMM roofline from the HIP events of the timed solves
    spmm_ms = sum(res.spmm_ms for v in recs.values() for _, res in v)
    spmm_n = sum(res.spmm_launches for v in recs.values() for _, res in v)
    spmm_bytes = sum(res.spmm_bytes * res.spmm_launches for v in recs.values() for _, res in v)
    achieved = (spmm_bytes / 1e9) / (spmm_ms / 1e3) if spmm_ms > 0 else None
    traffic = measured_traffic()

    enabled = [p for p in args.paths.split(",") if p] if args.paths else []
    drop = set()
    if args.no_precond:
        drop |= {"f64_precond", "f32_precond", "f32_precond_warm"}
    if args.no_f32:
        drop |= {p for p in ALL_PATHS if p.startswith("f32")}
    if args.no_bf16:
        drop.add("f32_bf16in")
    if args.no_warm:
        drop |= {"f32_warm", "f32_precond_warm"}
    enabled = [p for p in enabled if p not in drop]
    paths = {"f64": {}}
    for run in ([] if not step_times else runs):
        dt, res = recs[run["name"]][-1]
        rec = dict(seconds=round(dt, 4), outer=res.outer, inner=res.inner, obj=res.obj, err1=res.err1,
                   err3=res.err3, spmm_us=round(1e3 * res.spmm_ms / max(res.spmm_launches, 1), 2))
        if not args.short:
            rec.update(cert_of(run, run["per"][L.F64]["y"], res.obj))
            log(f"f64 {run['name']} certificate: lambda_min {rec['lambda_min']:.3e} gap {rec['cert_gap']:.2e} "
                f"({rec['cert_iters']} steps, {rec['cert_s']}s)")
        paths["f64"][run["name"]] = rec

    def record(path, run, dt, res, extra=None, y=None):
        o64 = paths["f64"].get(run["name"], {}).get("obj")
        rec = dict(seconds=round(dt, 4), outer=res.outer, inner=res.inner, obj=res.obj, err1=res.err1,
                   err3=res.err3, obj_rel_vs_f64=abs(res.obj - o64) / abs(o64) if o64 else None,
                   spmm_us=round(1e3 * res.spmm_ms / max(res.spmm_launches, 1), 2))
        rec.update(extra or {})
        if y is not None and not args.short:
            rec.update(cert_of(run, y, res.obj))
        paths.setdefault(path, {})[run["name"]] = rec
        log(f"{path} {run['name']} {dt:.3f}s outer {res.outer} inner {res.inner} obj {res.obj:.8e}"
            + (f" cert gap {rec['cert_gap']:.2e}" if "cert_gap" in rec else ""))

    def solve_with(run, prec, **kw):
        """One untimed-by-the-step solve of `run` in `prec` with extra options."""
        p = run["per"][prec]
        o = L.default_options(prec=prec, rank=run["r"], ld=p["opts"].ld, profile=1, verbose=int(args.verbose), **kw)
        ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
        p["R"].copy_(p["R0"])
        p["y"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = L.solve(ctx, run["prob"], p["R"], p["y"], o, workspace=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del ws
        return dt, rc, res

    if "f64_degsort" in enabled:
        # the same graphs with nodes relabelled by decreasing degree (hubs first):
        # the locality counterpart of the random labels of the timed step; the
        # starting factor is permuted with the nodes, so the solve is the same
        # problem up to the order of summation
        import numpy as np
        for run in runs:
            inst, n = run["inst"], run["n"]
            deg = np.bincount(inst["u"], minlength=n) + np.bincount(inst["v"], minlength=n)
            order = np.argsort(-deg, kind="stable")            # new node k is old node order[k]
            new_id = np.empty(n, dtype=np.int64)
            new_id[order] = np.arange(n)
            prob2 = L.Problem.maxcut(n, new_id[inst["u"]], new_id[inst["v"]], inst["w"]).upload(ctx)
            p = run["per"][L.F64]
            o = L.default_options(prec=L.F64, rank=run["r"], ld=p["opts"].ld, profile=1, verbose=int(args.verbose))
            ws = torch.empty(L.workspace_bytes(prob2, o), dtype=torch.uint8, device=dev)
            R = p["R0"][torch.from_numpy(order).to(dev)].contiguous()
            y = torch.zeros(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, res = L.solve(ctx, prob2, R, y, o, workspace=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            y_orig = y[torch.from_numpy(new_id).to(dev)].contiguous()     # back to the original labels
            record("f64_degsort", run, dt, res, dict(converged=rc == L.OK), y=y_orig)
            del prob2, ws, R, y, y_orig
    if "f64_precond" in enabled:
        # row-block H0 for Algorithm 1 (an extension; the timed step keeps H0 = I)
        for run in runs:
            dt, rc, res = solve_with(run, L.F64, precond=1)
            record("f64_precond", run, dt, res, dict(converged=rc == L.OK), y=run["per"][L.F64]["y"])
    def solve_dynrank(run, prec, **kw):
        """Dynamic rank (appendix A.1): start at the workload's rank, grow in place
        up to the stride DYNRANK_LD."""
        ld = DYNRANK_LD[0 if prec == L.F64 else 1]
        o = L.default_options(prec=prec, rank=run["r"], ld=ld, profile=1, rank_max=ld,
                              verbose=int(args.verbose), **kw)
        ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
        R = torch.zeros((run["n"], ld), dtype=L.elem_dtype(prec), device=dev)
        R[:, :run["r"]] = run["per"][prec]["R0"][:, :run["r"]]
        y = run["per"][prec]["y"]
        y.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = L.solve(ctx, run["prob"], R, y, o, workspace=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del ws, R
        return dt, rc, res, y

    if "f64_dynrank" in enabled:
        for run in runs:
            dt, rc, res, y = solve_dynrank(run, L.F64)
            record("f64_dynrank", run, dt, res, dict(converged=rc == L.OK, rank_final=res.rank_final), y=y)
    for path, level in (("f64_reopt", 1), ("f64_reopt2", 2)):
        # re-optimisation (Section 4.1): rounds stop at err1 <= tol; C scaled by
        # 0.1 per extra round until |err3| <= tol (and err2 <= tol at level 2)
        if path in enabled:
            for run in runs:
                dt, rc, res = solve_with(run, L.F64, reopt=level)
                extra = dict(converged=rc == L.OK, reopt_rounds=res.reopt_rounds)
                if level == 2:
                    extra["reopt_err2"] = res.err2
                record(path, run, dt, res, extra, y=run["per"][L.F64]["y"])
    if "f32" in enabled:
        for run in runs:
            dt, res = solve(run, L.F32)
            record("f32", run, dt, res, y=run["per"][L.F32]["y"])
    if "f32_precond" in enabled:
        for run in runs:
            dt, rc, res = solve_with(run, L.F32, precond=1)
            record("f32_precond", run, dt, res, dict(converged=rc == L.OK), y=run["per"][L.F32]["y"])
    if "f32_bf16in" in enabled:
        # bfloat16 gathered operand (float32 iterate, exact gradient every 25 iterations)
        for run in runs:
            p = run["per"][L.F32]
            o = L.default_options(prec=L.F32_BF16IN, rank=run["r"], ld=p["opts"].ld, profile=1, refresh_every=25)
            ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
            p["R"].copy_(p["R0"])
            p["y"].zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, res = L.solve(ctx, run["prob"], p["R"], p["y"], o, workspace=ws)
            torch.cuda.synchronize()
            record("f32_bf16in", run, time.perf_counter() - t0, res, dict(converged=rc == L.OK), y=p["y"])
            del ws
    if "f32_dynrank_precond" in enabled:
        for run in runs:
            dt, rc, res, y = solve_dynrank(run, L.F32, precond=1)
            record("f32_dynrank_precond", run, dt, res, dict(converged=rc == L.OK, rank_final=res.rank_final), y=y)
    warm_paths = [w for w in ("f32_warm", "f32_precond_warm") if w in enabled]
    if warm_paths:
        from paper_2407_15049_amd import warmstart as W
        t0 = time.perf_counter()
        data = W.make_training_set(ctx, log=log)
        t1 = time.perf_counter()
        params, hist = W.train(ctx, data, steps=400, lr=3e-3, log=log)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del data
        warm_info = dict(train_graphs=len(W.TRAIN_SPECS), label_solves_s=round(t1 - t0, 2),
                         train_s=round(t2 - t1, 2), loss_first=hist[0][1], loss_last=hist[-1][1])
        for wp in warm_paths:
            for run in runs:
                p = run["per"][L.F32]
                o = L.default_options(prec=L.F32, rank=run["r"], ld=p["opts"].ld, profile=1,
                                      precond=1 if wp == "f32_precond_warm" else 0,
                                      verbose=int(args.verbose))
                ws = torch.empty(L.workspace_bytes(run["prob"], o), dtype=torch.uint8, device=dev)
                p["R"].copy_(p["R0"])
                torch.cuda.synchronize()
                t0 = time.perf_counter()           # features + inference count toward the solve
                y0, sigma0 = W.warm_start(ctx, run["prob"], params)
                p["y"].copy_(y0)
                o.sigma0 = sigma0
                rc, res = L.solve(ctx, run["prob"], p["R"], p["y"], o, workspace=ws)
                torch.cuda.synchronize()
                record(wp, run, time.perf_counter() - t0, res, dict(sigma0=sigma0, converged=rc == L.OK), y=p["y"])
                del ws
            paths[wp]["model"] = warm_info

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device-to-device copies")
        del a, b

    # copy ceiling of the box: a 1 GiB device-to-device copy, read + write bytes
    # over its HIP-event time (median of 10)
    copy_gbs = None
    if step_times:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        stream = torch.cuda.current_stream(dev)
        for _ in range(3):
            b.copy_(a)
        times = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.copy_(a)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        copy_gbs = round(2.0 * (1 << 30) / 1e9 / sorted(times)[len(times) // 2], 1)
        log(f"copy ceiling: {copy_gbs} GB/s")
        del a, b

    cpu = None
    if not args.no_cpu_baseline and step_times:
        cpu = cpu_baseline(runs, recs, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(ms_per_step / 1000.0, 4) if ms_per_step else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2) if ms_per_step else None,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD if names == INSTANCES else
                   "; ".join(OTHER_WORKLOADS.get(nm, nm) for nm in names), "instances": names, "tol": 1e-5, "path": "plain FP64 ALM + L-BFGS",
                   "lbfgs_mem": runs[0]["per"][L.F64]["opts"].lbfgs_mem},
        "roofline": {
            "kernel": "spmm (MaxCut, line-search epilogue)",
            "bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
            "traffic_gbs": round(traffic / 1e9 / (spmm_ms / 1e3 / spmm_n), 1) if traffic and spmm_n else None,
            "launches": spmm_n,
            "avg_us": round(1e3 * spmm_ms / max(spmm_n, 1), 2),
            "alg_bytes_per_launch": {run["name"]: recs[run["name"]][-1][1].spmm_bytes for run in runs
                                     if recs[run["name"]]},
            "copy_ceiling_gbs": copy_gbs,
        },
        "cpu_baseline": cpu,
        "paths": paths,
    }
    print(json.dumps(out), flush=True)


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
    i, j, M, _, _ = completion_instance(cfg["n1"], cfg["n2"], cfg["k"], cfg["per_row"], cfg["seed"])
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
    print(json.dumps({
        "metric": "completion kernels: SDDMM / SpMM algorithmic GB/s and L-BFGS ms per iteration",
        "unit": "GB/s", "n_gpus": 1, "dtype": "f64,f32", "data": "synthetic",
        "config": {"workload": "matrix completion n1=n2=5e5 (X of order 1e6), m=1e7 samples (20 per row), "
                               "planted rank 5, factor rank 16", **cfg},
        "kernels": out}), flush=True)


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


def cpu_baseline(runs, recs, target_s):
    """Oracle (numpy/scipy FP64, one thread) L-BFGS iterations on every instance
    for about target_s seconds in total; time per iteration times the
    iterations the GPU FP64 solve of that instance took, summed over the
    instances (the same unit as the step)."""
    from threadpoolctl import threadpool_limits

    from oracle.alm import Options, alm_solve
    from oracle.problem import maxcut_problem
    from synth import init_factor

    total, parts = 0.0, []
    with threadpool_limits(limits=1):
        for run in runs:
            inst = run["inst"]
            t0 = time.perf_counter()
            op = maxcut_problem(inst["n"], inst["u"], inst["v"], inst["w"])
            R0 = init_factor(inst["n"], inst["rank"], inst["seed"] + 1)
            build = time.perf_counter() - t0
            t1 = time.perf_counter()                       # calibrate on 2 iterations
            alm_solve(op, R0, opts=Options(max_outer=1, max_inner=2))
            per_iter = (time.perf_counter() - t1) / 2
            k = max(2, int(target_s / len(runs) / max(per_iter, 1e-6)))
            t2 = time.perf_counter()
            res = alm_solve(op, R0, opts=Options(max_outer=1, max_inner=k))
            sample_s = time.perf_counter() - t2
            per_iter = sample_s / max(res.inner, 1)
            gres = recs[run["name"]][-1][1]
            est = per_iter * gres.inner
            total += est
            log(f"cpu oracle {run['name']}: {res.inner} iterations in {sample_s:.1f}s ({per_iter:.3f}s/iter), "
                f"estimate for {gres.inner} iterations: {est:.0f}s (problem build {build:.1f}s)")
            parts.append(f"{run['name']}: {res.inner} iterations in {sample_s:.1f}s, scaled to the GPU FP64 "
                         f"solve's {gres.inner} iterations / {gres.outer} ALM steps")
            del op
    return {
        "value": round(total, 1),
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("oracle L-BFGS iterations of the first ALM subproblem (numpy/scipy, one thread), per "
                   "instance: " + "; ".join(parts) + "; oracle problem builds not included"),
    }


if __name__ == "__main__":
    main()
