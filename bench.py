"""Benchmark: Tucker-ALS (HOOI) decompositions of a 1080p multi-exposure stereo stack on one MI355X.

A step is one whole decomposition through the C ABI: T-HOSVD start + 20 HOOI sweeps + the
exact-residual fit, on a 1080 x 1920 x 3 x 14 FP32 Y'CbCr stack (2 views x 7 exposures) with
ranks (256, 384, 3, 8).  The input is resident in HBM before the timed region.  The reported
value is whole-job HOOI sweeps per second: 20 * steps / elapsed.

Also reported (one JSON line on stdout):
  roofline      the dominant single-kernel stage, algorithmic bytes or flops per launch divided by
                its mean launch time, timed with HIP events on the launch stream during the timed
                steps, against the MI355X peak (HBM 8 TB/s, FP32 MFMA 157.3 TFLOP/s);
  stages        every timed stage (ms per launch, achieved rate);
  cpu_baseline  the FP64 CPU oracle on the same tensor: T-HOSVD plus a sample of sweeps, timed on
                the host cores and scaled to the same 20-sweep job.

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
FP32_MFMA_PEAK_TFLOPS = 157.3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_work(dims, ranks):
    """Algorithmic work of one launch of each single-kernel stage of a tree sweep.

    Returns {stage: (kind, amount)} with kind 'hbm' (bytes) or 'mfma' (flops).  Bytes are
    the reads of the input and writes of the output once; flops are 2 * MACs (the Gram counts
    the lower triangle it computes: s^2 K).
    """
    s0, s1, s2, s3 = dims
    r0, r1, r2, r3 = ranks
    r23, L = r2 * r3, s2 * s3
    return {
        "pass_a": ("hbm", 4 * (s0 * s1 * L + s0 * s1 * r23)),
        "ttm_y1": ("mfma", 2 * r1 * s1 * (s0 * r23)),
        "gram_1": ("mfma", s0 * s0 * (r1 * r23)),
        "ttm_y2": ("mfma", 2 * r0 * s0 * (s1 * r23)),
        "gram_2": ("mfma", s1 * s1 * (r0 * r23)),
        "pass_c1": ("mfma", 2 * r0 * s0 * (s1 * L)),
        "ttm_c2": ("mfma", 2 * r1 * s1 * (r0 * L)),
    }


def roofline_of(kind, amount, ms):
    if kind == "hbm":
        achieved = amount / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    achieved = amount / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4)}


def cpu_baseline(x32, ranks, sweeps_job, sample_sweeps):
    """FP64 oracle on the host: T-HOSVD + `sample_sweeps` sweeps, scaled to a sweeps_job job."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    x = x32.astype(np.float64)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--cpu-sample-sweeps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the decomposition is not "
              "sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2104_04726_amd as tk
    from synth import make_stereo_stack, STACK_CONFIGS

    cfg = STACK_CONFIGS["stack1080"]
    H, W, E, ranks = cfg["H"], cfg["W"], cfg["E"], tuple(cfg["ranks"])
    sweeps = args.sweeps
    log(f"generating {H}x{W}x3x{2 * E} stack (seed {cfg['seed']})")
    x32 = make_stereo_stack(H, W, E, cfg["colorspace"], cfg["seed"])
    dims = x32.shape
    x = torch.from_numpy(x32).to("cuda:0")
    torch.cuda.synchronize()

    ctx = tk.Context(0, timing=True)
    for i in range(args.warmup):
        r = ctx.decompose(x, ranks, sweeps)
        log(f"warmup {i}: fit {r.fit:.8f} sweeps {r.sweeps} init {r.stats['init_ms']:.2f} ms "
            f"sweeps {r.stats['sweeps_ms']:.2f} ms")
    torch.cuda.synchronize()
    stage_tot = {}
    init_ms = sweeps_ms = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = ctx.decompose(x, ranks, sweeps)
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
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.2f} sweeps/s, fit {r.fit:.8f}")

    work = stage_work(dims, ranks)
    stages = {}
    for name, (ms, calls) in sorted(stage_tot.items()):
        per = ms / calls
        entry = {"ms_per_launch": round(per, 4), "launches": calls, "share": round(ms / (sweeps_ms or 1), 4)}
        if name in work:
            entry.update(roofline_of(*work[name], per))
        stages[name] = entry
    dominant = max((n for n in stages if n in work), key=lambda n: stage_tot[n][0])
    kind, amount = work[dominant]
    roof = roofline_of(kind, amount, stage_tot[dominant][0] / stage_tot[dominant][1])
    roof.update({"kernel": dominant, "traffic": None,
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"stack1080: {H}x{W}x3x{2 * E} FP32 Y'CbCr multi-exposure stereo stack, ranks "
                               f"{list(ranks)}, T-HOSVD start + {sweeps} HOOI sweeps per step",
                   "sweeps_per_step": sweeps, "fit": round(r.fit, 9),
                   "init_ms": round(init_ms / args.steps, 3), "sweeps_ms": round(sweeps_ms / args.steps, 3)},
        "roofline": roof,
        "stages": stages,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(x32, ranks, sweeps, args.cpu_sample_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
