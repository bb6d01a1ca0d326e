"""Benchmark: Tucker-ALS (HOOI) decompositions of a 1080p multi-exposure stereo stack on one MI355X.

A step is one whole decomposition through the C ABI: T-HOSVD start + 20 HOOI sweeps + the
exact-residual fit, on a 1080 x 1920 x 3 x 14 FP32 Y'CbCr stack (2 views x 7 exposures) with
ranks (256, 384, 3, 8).  The input is resident in HBM before the timed region.  The reported
value is whole-job HOOI sweeps per second: 20 * steps / elapsed.

Also reported (one JSON line on stdout):
  roofline      the dominant single-kernel stage, algorithmic bytes or flops per launch divided by
                its mean launch time, timed with HIP events on the launch stream during the timed
                steps, against the MI355X peak (HBM 8 TB/s, FP32 MFMA 157.3 TFLOP/s,
                FP64 MFMA 78.6 TFLOP/s);
  stages        every stage (ms per launch, achieved rate), from the first timed step, which times
                every stage; the later timed steps time the dominant stage only, since each timed
                stage's pair of events leaves the device idle for a few microseconds;
  cpu_baseline  the FP64 CPU oracle on the same tensor, timed on the host cores: the whole job
                (T-HOSVD + the same sweeps; the precision variants add their refinement sweep)
                for the 1080p stack, with the GPU result's errors against it (relative
                reconstruction and core-norm differences, fit difference, largest principal-angle
                sine per factor); T-HOSVD plus a sample of sweeps, scaled to the job, for 4K.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0}   # MI355X dense


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_work(dims, ranks, precision="fp32"):
    """Algorithmic work of one launch of each single-kernel stage of a tree sweep.

    Returns {stage: (kind, amount)} with kind 'hbm' (bytes) or a matrix-core type 'f32', 'f64',
    'bf16', 'f16', 'fp8' (flops).  Bytes are the reads of the input and writes of the output
    once; flops are 2 * MACs (the Gram counts the lower triangle it computes: s^2 K).  In FP32
    every product runs on the FP32 matrix cores: with one orthogonal-iteration step per sweep (the
    default) the gram stages time the two products W = Y x_n U^T and Y_(n) W_(n)^T (mode 2 forms W
    from the mode-1 tensor, contracting over s1) with their split sums.  In reduced precision every contraction runs in the 16-bit
    type (FP8: the two products over X in FP8, the rest in BF16) and the two full-tensor passes
    are priced by their bytes (X in the storage type, outputs in the 16-bit type, T34 rows padded
    to a multiple of 8).
    """
    s0, s1, s2, s3 = dims
    r0, r1, r2, r3 = ranks
    r23, L = r2 * r3, s2 * s3
    if precision == "fp32":
        return {
            "pass_a": ("hbm", 4 * (s0 * s1 * L + s0 * s1 * r23)),
            "ttm_y1": ("f32", 2 * r1 * s1 * (s0 * r23)),
            "gram_1": ("f32", 4 * s0 * r0 * (r1 * r23)),
            # Y2 = T1 x_3 U3^T x_4 U4^T: the fibre kernel on T1 (pass C1 runs before mode 2)
            "ttm_y2": ("hbm", 4 * (r0 * s1 * L + r0 * s1 * r23)),
            # mode 2: W = Y1 x_1 U1^T from the mode-1 tensor (contracted over s1), then Y2_(2) W_(2)^T
            "gram_2": ("f32", 2 * r0 * s0 * (r1 * r23) + 2 * s1 * r1 * (r0 * r23)),
            "pass_c1": ("f32", 2 * r0 * s0 * (s1 * L)),
            "ttm_c2": ("f32", 2 * r1 * s1 * (r0 * L)),
        }
    ex = 1 if precision == "fp8" else 2
    it = "bf16" if precision in ("bf16", "fp8") else "f16"
    r23p = (r23 + 7) // 8 * 8
    return {
        "pass_a": ("hbm", ex * s0 * s1 * L + 2 * s0 * s1 * r23p),
        "ttm_y1": (it, 2 * r1 * s1 * (s0 * r23p)),
        "gram_1": (it, s0 * s0 * (r1 * r23p)),
        "ttm_y2": (it, 2 * r0 * s0 * (s1 * r23p)),
        "gram_2": (it, s1 * s1 * (r0 * r23p)),
        "pass_c1": ("hbm", ex * s0 * s1 * L + 2 * r0 * s1 * L),
        "ttm_c2": (it, 2 * r1 * s1 * (r0 * L)),
    }


def roofline_of(kind, amount, ms):
    if kind == "hbm":
        achieved = amount / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    achieved = amount / (ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[kind]
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "mfma_type": kind}


def cpu_baseline(x32, ranks, sweeps_job, sample_sweeps, gpu_result=None, oracle_sweeps=None, start="thosvd"):
    """FP64 oracle on the host.

    sample_sweeps > 0: T-HOSVD + `sample_sweeps` sweeps, scaled to a sweeps_job job.
    sample_sweeps == 0: the whole job (T-HOSVD + oracle_sweeps sweeps, default sweeps_job) is run and
    timed; with gpu_result (core, factors, fit of the GPU's last decomposition, host arrays) the
    GPU's errors against this oracle result are reported beside the time: relative reconstruction
    difference, relative core-norm difference, fit difference and the largest principal-angle sine
    of every factor (rotation-invariant; computed in core space)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    x = x32.astype(np.float64)
    if sample_sweeps == 0:
        n_or = oracle_sweeps if oracle_sweeps is not None else sweeps_job
        t0 = time.perf_counter()
        o = oracle.hooi(x, ranks, n_or, start=start)
        t_job = time.perf_counter() - t0
        out = {"value": round(n_or / t_job, 4), "unit": "sweeps/s", "cores": cores, "kind": "oracle",
               "sample": f"the whole job: {'T-HOSVD' if start == 'thosvd' else 'ST-HOSVD'} + {n_or} sweeps "
                         f"of the FP64 oracle on the full tensor "
                         f"({t_job:.2f} s)", "job_s": round(t_job, 3)}
        if gpu_result is not None:
            m = oracle.compare(gpu_result, dict(core=o.core, factors=o.factors, fit=o.fits[-1]))
            out["errors_vs_oracle"] = {
                "recon_rel": float(f"{m['recon']:.3e}"), "core_norm_rel": float(f"{m['core_norm']:.3e}"),
                "fit_abs": float(f"{m['fit']:.3e}"), "sin_theta_max": [float(f"{v:.3e}") for v in m["sin_theta"]],
                "oracle_fit": round(o.fits[-1], 10), "oracle_sweeps": n_or}
        return out
    t0 = time.perf_counter()
    fac, _ = oracle.thosvd_factors(x, ranks)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(sample_sweeps):
        for n, r in enumerate(ranks):
            fac[n], _, _ = oracle.hooi_update(x, fac, n, r)
    t_sweep = (time.perf_counter() - t0) / sample_sweeps
    t_job = t_init + sweeps_job * t_sweep
    return {"value": round(sweeps_job / t_job, 4), "unit": "sweeps/s", "cores": cores, "kind": "oracle",
            "sample": f"T-HOSVD ({t_init:.2f} s) + {sample_sweeps} sweep(s) ({t_sweep:.2f} s each) of the FP64 "
                      f"oracle on the full tensor; {sweeps_job}-sweep job time extrapolated",
            "init_s": round(t_init, 3), "sweep_s": round(t_sweep, 3)}


def measured_traffic(stage):
    """HBM bytes per launch of a stage kernel from the committed counter summary, or None when the
    kernel's source has changed since the counters were taken (or no summary exists)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_stack1080.txt")
    if not os.path.exists(path):
        return None
    for ln in open(path):
        f = ln.split()
        if len(f) == 6 and f[0] == "traffic" and f[1] == stage:
            src = os.path.join(ROOT, "paper_2104_04726_amd", "csrc", f[4])
            if not os.path.exists(src):
                return None
            digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            if digest != f[5]:
                return None
            return {"fetch_bytes": int(f[2]), "write_bytes": int(f[3]), "total_bytes": int(f[2]) + int(f[3]),
                    "source": "profiles/hbm_traffic_stack1080.txt (FETCH_SIZE x2.0, WRITE_SIZE x1.0 from a "
                              "1 GiB copy calibration)"}
    return None


def _gen_stack(args):
    from synth import make_stereo_stack
    H, W, seed = args
    return make_stereo_stack(H, W, 7, "ycbcr", seed)


def serve(args):
    """Served execution: Poisson-arriving requests of mixed resolution and exposure count (the
    serving configuration), BF16 sweeps + 1 FP32 refinement, admitted by HBM budget with several
    requests on the GPU at once.  Tensors: one seeded E = 7 stack per resolution; a request with
    E = 3 or 5 exposures uses the middle exposures of each view, which is exactly the stack the
    generator makes for that E (same radiance field and exposure scale)."""
    import concurrent.futures as cf
    import threading
    import numpy as np
    import torch
    import paper_2104_04726_amd as tk
    from synth import serving_requests

    reqs = serving_requests(args.requests, 0.025, 3)
    sizes = sorted({(q["H"], q["W"]) for q in reqs})
    log(f"generating {len(sizes)} base stacks")
    with cf.ProcessPoolExecutor(max_workers=min(4, len(sizes))) as ex:
        base = dict(zip(sizes, ex.map(_gen_stack, [(H, W, 3000 + i) for i, (H, W) in enumerate(sizes)])))
    cells = {}
    for (H, W), x7 in base.items():
        for E in (3, 5, 7):
            lo = (7 - E) // 2
            x = np.concatenate([x7[..., v * 7 + lo: v * 7 + lo + E] for v in range(2)], axis=-1)
            cells[(H, W, E)] = torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
    del base
    iters = 10

    def run(srv, items, open_loop):
        t0 = time.perf_counter()
        ids = [None] * len(items)

        def submitter():
            for k, q in enumerate(items):
                if open_loop:
                    d = q["t_arrive"] - (time.perf_counter() - t0)
                    if d > 0:
                        time.sleep(d)
                ids[k] = srv.submit(cells[(q["H"], q["W"], q["E"])], q["ranks"], iters, precision=args.serve_precision,
                                    refine_sweeps=1 if args.serve_precision != "fp32" else 0, tag=k)
        th = threading.Thread(target=submitter)
        th.start()
        out = []
        for k in range(len(items)):
            while ids[k] is None:
                time.sleep(0.0005)
            out.append(srv.wait(ids[k]))
        th.join()
        wall = time.perf_counter() - t0
        return out, wall

    def summary(res, wall):
        lat = np.array([r.latency for r in res]) * 1e3
        bad = [r for r in res if r.status != 0]
        if bad:
            raise RuntimeError(f"{len(bad)} requests failed: {bad[0].error}")
        span = max(r.t_finish for r in res) - min(r.t_submit for r in res)
        return {"requests": len(res), "decomp_per_s": round(len(res) / span, 3), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2), "mean_ms": round(float(lat.mean()), 2),
                "wall_s": round(wall, 3)}

    # warm-up (kernels loaded, memory pool primed) on one request of every size
    with tk.Server(0, slots=args.slots, use_graphs=not args.no_serve_graphs) as srv:
        warm = [dict(H=H, W=W, E=7, ranks=(H // 4, W // 4, 3, 13), t_arrive=0.0) for (H, W) in sizes]
        run(srv, warm, open_loop=False)
        log(f"open loop: {len(reqs)} requests, Poisson 40/s, {args.slots} slots")
        res_open, wall_open = run(srv, reqs, open_loop=True)
        open_sum = summary(res_open, wall_open)
        log(f"  {open_sum}")
        nsat = min(len(reqs), args.saturated)
        log(f"saturated: {nsat} requests submitted at once")
        res_sat, wall_sat = run(srv, reqs[:nsat], open_loop=False)
        sat_sum = summary(res_sat, wall_sat)
        log(f"  {sat_sum}")
        st = srv.stats()
    # grouped burst: requests of one class submitted at once, run with and without grouped launches
    # of their reduced-precision products (groups form from consecutive requests of one class)
    bH, bW = sizes[len(sizes) // 2]
    burst = [dict(H=bH, W=bW, E=5, ranks=(bH // 4, bW // 4, 3, 9), t_arrive=0.0)] * args.burst
    burst_sum = {}
    for key, grouped, graphs in (("alone", False, not args.no_serve_graphs), ("alone_no_graphs", False, False),
                                 ("grouped", True, False)):
        with tk.Server(0, slots=args.slots, use_graphs=graphs, group_requests=4 if grouped else 0) as srv:
            run(srv, burst[:args.slots], open_loop=False)
            res_b, wall_b = run(srv, burst, open_loop=False)
            bst = srv.stats()
        burst_sum[key] = dict(summary(res_b, wall_b), grouped_requests=bst["grouped_requests"],
                              group_launches=bst["group_launches"], grouped_products=bst["grouped_products"])
        log(f"burst {key}: {burst_sum[key]}")
    # baseline: the same requests one after another in plain FP32 (10 sweeps), on a stratified
    # sample of one request per (resolution, exposures) cell
    ctx = tk.Context(0)
    times = []
    for (H, W, E), xh in sorted(cells.items()):
        xd = xh.cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.decompose(xd, (H // 4, W // 4, 3, 2 * E - 1), iters)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        del xd
    ctx.close()
    seq_rate = 1.0 / float(np.mean(times))
    out = {
        "metric": "served decompositions/s (p50/p99 latency)",
        "value": open_sum["decomp_per_s"],
        "unit": "decompositions/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": args.serve_precision,
        "data": "synthetic",
        "config": {"workload": f"serving: {len(reqs)} Poisson requests (mean 40/s), 640x480..2560x1440 x 3 x 2E, "
                               f"E in 3/5/7, ranks (H/4, W/4, 3, 2E-1), {iters} {args.serve_precision} sweeps"
                               + (" + 1 FP32 refinement" if args.serve_precision != "fp32" else ""),
                   "slots": args.slots, "budget_bytes": st["budget_bytes"],
                   "peak_admitted_bytes": st["peak_admitted_bytes"], "peak_running": st["peak_running"]},
        "open_loop": open_sum,
        "saturated": sat_sum,
        "grouped_burst": dict(burst_sum, workload=f"{args.burst} requests {bH}x{bW}x3x10 at once, ranks "
                                                  f"({bH // 4}, {bW // 4}, 3, 9), {iters} {args.serve_precision} sweeps"),
        "group_stats": {"grouped_requests": st["grouped_requests"], "group_launches": st["group_launches"]},
        "sequential_fp32_baseline": {"decomp_per_s": round(seq_rate, 3),
                                     "sample": f"{len(times)} requests, one per (resolution, E) cell, plain FP32, "
                                               f"{iters} sweeps, one at a time"},
    }
    print(json.dumps(out), flush=True)


def copy_probe(nbytes=1 << 30, reps=3):
    """A plain elementwise kernel that reads and writes nbytes each (y = -x, FP32): what the HBM
    byte counters report for it calibrates them against a known algorithmic traffic."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "reps": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=None, help="sweeps per decomposition (default: the workload's)")
    ap.add_argument("--cpu-sample-sweeps", type=int, default=None,
                    help="oracle sweeps timed for the CPU baseline and scaled to the job; 0 runs the whole "
                         "oracle job and reports the GPU result's errors against it (default: 0 for "
                         "stack1080, 2 for stack2160)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="stack1080", choices=["stack1080", "stack2160"],
                    help="stack1080: 1080p Y'CbCr, 20 sweeps (the default measurement); stack2160: 4K IPT, 15 sweeps")
    ap.add_argument("--init-iters", type=int, default=20,
                    help="cold-start orthogonal-iteration steps of the T-HOSVD start")
    ap.add_argument("--start", default="thosvd", choices=["thosvd", "sthosvd"],
                    help="initialisation: truncated HOSVD (default) or the sequentially truncated HOSVD")
    ap.add_argument("--pp-tol", type=float, default=0.0,
                    help="pairwise-perturbation sweeps once the factors settle to this subspace distance (0: off)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16", "fp8"],
                    help="operand precision of the sweeps (reduced precision adds one FP32 refinement sweep)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="launch choices from the built-in heuristics instead of measuring them during the warm-up")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each sweep as a HIP graph on a side stream (no per-stage timers)")
    ap.add_argument("--serve", action="store_true", help="run the served-execution benchmark instead")
    ap.add_argument("--no-serve-graphs", action="store_true", help="serving slots launch kernel by kernel")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--saturated", type=int, default=128)
    ap.add_argument("--burst", type=int, default=32, help="requests of one class in the grouped-burst comparison")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--serve-precision", default="bf16", choices=["fp32", "bf16", "fp16", "fp8"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain elementwise copy of 1 GiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.serve:
        serve(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the decomposition runs on a "
              "single GPU and is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2104_04726_amd as tk
    from synth import make_stereo_stack, STACK_CONFIGS

    cfg = STACK_CONFIGS[args.workload]
    H, W, E, ranks = cfg["H"], cfg["W"], cfg["E"], tuple(cfg["ranks"])
    sweeps = args.sweeps if args.sweeps is not None else cfg["sweeps"]
    log(f"generating {H}x{W}x3x{2 * E} stack (seed {cfg['seed']})")
    x32 = make_stereo_stack(H, W, E, cfg["colorspace"], cfg["seed"])
    dims = x32.shape
    x = torch.from_numpy(x32).to("cuda:0")
    torch.cuda.synchronize()

    if args.graphs:
        side = torch.cuda.Stream()
        ctx = tk.Context(0, stream=side, timing=False, precision=args.precision, refine_sweeps=1,
                         init_iters=args.init_iters, use_graphs=True, start=args.start, pp_tol=args.pp_tol,
                         autotune=not args.no_autotune)
    else:
        ctx = tk.Context(0, timing=True, precision=args.precision, refine_sweeps=1, init_iters=args.init_iters,
                         start=args.start, pp_tol=args.pp_tol, autotune=not args.no_autotune)
    for i in range(args.warmup):
        r = ctx.decompose(x, ranks, sweeps)
        log(f"warmup {i}: fit {r.fit:.8f} sweeps {r.sweeps} init {r.stats['init_ms']:.2f} ms "
            f"sweeps {r.stats['sweeps_ms']:.2f} ms")
    torch.cuda.synchronize()
    work = stage_work(dims, ranks, args.precision)

    def dominant_of(st):
        # the roofline object describes one kernel: the single-kernel stage with the largest total
        # time (in FP32 the mode-update stages run two products and a split sum)
        single = [n for n in st if n in work and (args.precision != "fp32" or not n.startswith("gram"))]
        return max(single, key=lambda n: st[n][0]) if single else None

    dominant, breakdown, base_ms = None, {}, 0.0
    if not args.no_autotune:
        log("autotuner choices:\n" + tk.autotune_table().rstrip())
    stage_tot = {}
    init_ms = sweeps_ms = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = ctx.decompose(x, ranks, sweeps)
        if i == 0 and r.stats["stages"]:
            # every stage timed on the first step; the dominant one only from then on
            breakdown, base_ms = r.stats["stages"], r.stats["sweeps_ms"]
            dominant = dominant_of(breakdown)
            if dominant:
                ctx.set_timing(True, [dominant])
        for name, (ms, calls) in r.stats["stages"].items():
            a = stage_tot.setdefault(name, [0.0, 0])
            a[0] += ms
            a[1] += calls
        init_ms += r.stats["init_ms"]
        sweeps_ms += r.stats["sweeps_ms"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = sweeps * args.steps / elapsed
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.2f} sweeps/s, fit {r.fit:.8f}, "
        f"second CholeskyQR passes {r.stats.get('orth_second_passes')}")

    stages = {}
    for name, (ms, calls) in sorted(breakdown.items()):
        per = ms / calls
        entry = {"ms_per_launch": round(per, 4), "launches": calls, "share": round(ms / (base_ms or 1), 4)}
        if name in work:
            entry.update(roofline_of(*work[name], per))
        stages[name] = entry
    roof = None
    if dominant and dominant in stage_tot:
        kind, amount = work[dominant]
        roof = roofline_of(kind, amount, stage_tot[dominant][0] / stage_tot[dominant][1])
        traffic = measured_traffic(dominant) if (args.precision == "fp32" and args.workload == "stack1080") else None
        roof.update({"kernel": dominant, "traffic": traffic["total_bytes"] if traffic else None,
                     "traffic_unit": "bytes per launch", "traffic_detail": traffic,
                     "per_launch": f"{amount / 1e9:.3f} {'GB' if kind == 'hbm' else 'GFLOP'}"})

    out = {
        "metric": "HOOI sweeps/s",
        "value": round(value, 3),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp16": "f16", "fp8": "fp8_e4m3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {H}x{W}x3x{2 * E} FP32 {cfg['colorspace']} multi-exposure stereo stack, ranks "
                               f"{list(ranks)}, {'T-HOSVD' if args.start == 'thosvd' else 'ST-HOSVD'} start + "
                               f"{sweeps} HOOI sweeps per step"
                               + ("" if args.precision == "fp32" else
                                  f" ({args.precision} contractions, then 1 FP32 refinement sweep)"),
                   "precision": args.precision,
                   "sweeps_per_step": sweeps, "fit": round(r.fit, 9),
                   "orth_second_passes": r.stats.get("orth_second_passes"),
                   "pp_tol": args.pp_tol, "pp_sweeps": r.stats.get("pp_sweeps"), "autotune": not args.no_autotune,
                   "init_ms": round(init_ms / args.steps, 3), "sweeps_ms": round(sweeps_ms / args.steps, 3)},
        "roofline": roof,
        "stages": stages,
    }
    gpu_result = dict(core=r.core.cpu().numpy().astype(np.float64),
                      factors=[u.cpu().numpy().astype(np.float64) for u in r.factors], fit=r.fit)
    ctx.close()
    if not args.no_cpu_baseline:
        sample = args.cpu_sample_sweeps
        if sample is None:
            sample = 0 if args.workload == "stack1080" else 2
        log("timing the CPU oracle" + (" (whole job, errors of the GPU result against it)" if sample == 0 else
                                       " sample"))
        refine = 0 if args.precision == "fp32" else 1
        out["cpu_baseline"] = cpu_baseline(x32, ranks, sweeps, sample, gpu_result, sweeps + refine, args.start)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
