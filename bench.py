#!/usr/bin/env python3
"""Benchmark of the DoSample hot path on one MI355X.

Workload (the metric's configuration): Vegas in d = 8 with 128 bins per
dimension, 20 iterations of 10^7 points each, on the Genz oscillatory and
product-peak integrands (parameters: a_i = 9 r_i / sum r, r, u ~ U(0,1),
seed 1).  One step = both integrals run to completion, 4 x 10^8 integrand
evaluations, with FP32 evaluation and FP64 accumulation.  The same step in
all-FP64 is timed beside it.  Inputs are synthetic and resident on the device
(the points are generated on the device from Philox counters).

Prints one JSON line: value = integrand evaluations per second of the whole
job (FP32-evaluate path), plus the FP64 figure, a roofline object for the
DoSample kernel (event-timed inside the library on the stream it runs on) and
the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D, NBINS, NPTS, ITERS = 8, 128, 10**7, 20
FAMILIES = (1, 2)  # oscillatory, product peak
PEAK_VALU_SLOTS = 256 * 4 * 16 * 2.4e9  # VALU lane-op issue slots per second
# VALU issue slots per point of the FP32-evaluate DoSample loop at d = 8 (from
# the instruction mix of this build: 247 full-rate VALU instructions and 33
# 64-bit integer multiplies at a quarter of the issue rate)
SLOTS_PER_POINT = {1: 247 + 4 * 33, 2: 254 + 4 * 33}


def _step(cc, ctx, params, prec):
    ev = 0
    for fam in FAMILIES:
        a, u = params[fam]
        r = cc.vegas(fam, a, u, ctx=ctx, flags=prec, nbins=NBINS, nstart=NPTS,
                     maxeval=ITERS * NPTS, seed=1)
        if r["neval"] != ITERS * NPTS:
            raise RuntimeError("unexpected neval %d" % r["neval"])
        ev += r["neval"]
    return ev


def _timed(cc, ctx, params, prec, steps, warmup):
    import torch
    for _ in range(warmup):
        _step(cc, ctx, params, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = 0
    for _ in range(steps):
        ev += _step(cc, ctx, params, prec)
    torch.cuda.synchronize()
    return ev, time.perf_counter() - t0


def _kernel_rate(cc, ctx, params, prec):
    """Event-timed DoSample launches of one profiled step."""
    import ctypes as C

    class Stats(C.Structure):
        _fields_ = [("dosample_launches", C.c_longlong), ("dosample_ms", C.c_double),
                    ("refine_launches", C.c_longlong), ("refine_ms", C.c_double),
                    ("evals", C.c_longlong), ("rule_launches", C.c_longlong),
                    ("rule_ms", C.c_double), ("rule_evals", C.c_longlong)]

    fn = cc._lib.ccuba_stats_get
    fn.argtypes = [C.c_void_p, C.POINTER(Stats), C.c_int]
    st = Stats()
    fn(ctx.handle, C.byref(st), 1)
    ctx.config("profile", 1)
    per_fam = {}
    for fam in FAMILIES:
        a, u = params[fam]
        cc.vegas(fam, a, u, ctx=ctx, flags=prec, nbins=NBINS, nstart=NPTS,
                 maxeval=ITERS * NPTS, seed=1)
        fn(ctx.handle, C.byref(st), 1)
        per_fam[fam] = dict(launches=st.dosample_launches, ms=st.dosample_ms, evals=st.evals,
                            refine_ms=st.refine_ms)
    ctx.config("profile", 0)
    return per_fam


def _cpu_baseline(params, iters_sample=4):
    import oracle as O
    t0 = time.perf_counter()
    ev = 0
    for fam in FAMILIES:
        a, u = params[fam]
        r = O.vegas(O.genz(fam, a, u), D, nbins=NBINS, nstart=NPTS,
                    maxeval=iters_sample * NPTS, seed=1)
        ev += r["neval"]
    dt = time.perf_counter() - t0
    return dict(value=ev / dt, unit="evals/s", cores=1, kind="oracle",
                sample="first %d of 20 iterations (10^7 points each) of both integrals, "
                       "FP64, single thread: %d evals in %.1f s" % (iters_sample, ev, dt))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); no multi-GPU path exists",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1408_6373_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    params = {fam: W.genz_params(fam, D, 1) for fam in FAMILIES}
    ctx = cc.Context(device=0)

    ev32, t32 = _timed(cc, ctx, params, cc.FP32_EVAL, args.steps, args.warmup)
    value = ev32 / t32
    out = {
        "metric": "integrand evals/s (Vegas d=8, FP32 vs FP64) + p50/p99 solve latency",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "accumulate": "f64", "data": "synthetic",
        "config": {"workload": "vegas_d8_genz_oscillatory+product_peak_20x1e7_128bins",
                   "ndim": D, "nbins": NBINS, "points_per_iteration": NPTS,
                   "iterations": ITERS, "integrals_per_step": len(FAMILIES)},
    }
    if not args.no_fp64:
        ev64, t64 = _timed(cc, ctx, params, cc.FP64, args.steps, args.warmup)
        out["fp64"] = {"value": ev64 / t64, "unit": "evals/s",
                       "ms_per_step": 1e3 * t64 / args.steps,
                       "fp32_speedup": value / (ev64 / t64)}

    k = _kernel_rate(cc, ctx, params, cc.FP32_EVAL)
    ms = sum(v["ms"] for v in k.values())
    launches = sum(v["launches"] for v in k.values())
    evals = sum(v["evals"] for v in k.values())
    slots = sum(SLOTS_PER_POINT[f] * k[f]["evals"] for f in FAMILIES)
    avg_ms = ms / max(launches, 1)
    achieved = slots / (ms * 1e-3) / 1e12
    peak = PEAK_VALU_SLOTS / 1e12
    out["roofline"] = {
        "bound": "alu", "kernel": "vegas_dosample_kernel<float,float>",
        "achieved": achieved, "peak": peak, "unit": "T VALU-slots/s", "frac": achieved / peak,
        "traffic": None, "avg_launch_ms": avg_ms, "launches": launches,
        "kernel_evals_per_s": evals / (ms * 1e-3),
        "refine_ms_per_launch": sum(v["refine_ms"] for v in k.values()) / max(launches, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(params)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
