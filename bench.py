#!/usr/bin/env python3
"""Benchmark of the DoSample hot path on one MI355X.

Headline workload (the metric's configuration): Vegas in d = 8 with 128 bins
per dimension, 20 iterations of 10^7 points each, on the Genz oscillatory
and product-peak integrands (a_i = 9 r_i / sum r, r, u ~ U(0,1), seed 1).
One step = both integrals run to completion (4 x 10^8 integrand evaluations)
with FP32 evaluation and FP64 accumulation; the same step in all-FP64 is
timed beside it.  Inputs are synthetic; the points are generated on the
device from Philox counters, so nothing but the 2 x 8 Genz constants
crosses PCIe.

The JSON line also carries:
  roofline      the DoSample kernel's VALU issue rate (HIP events recorded by
                the library around each launch, on the stream it runs on)
                against the FP32 VALU issue peak;
  batch         4096 independent Vegas integrals (d 2..12, 10^4..10^6
                points, 10 iterations, FP32) in one persistent launch per
                iteration, launch settings autotuned on the batch itself
                (first call, untimed);
  cuhre         corner peak, d = 6, batches of 10^5 regions to epsrel 1e-6;
  serving       Poisson arrivals of Vegas (70%) and Cuhre (30%) requests,
                d 2..16, epsrel log-uniform in [1e-5, 1e-3], at 0.7 of the
                measured saturation rate: p50/p99 latency and evals/s;
  cpu_baseline  the CPU oracle on a bounded sample of the headline workload.
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D, NBINS, NPTS, ITERS = 8, 128, 10**7, 20
FAMILIES = (1, 2)  # oscillatory, product peak
FAMILY_KEYS = {1: "oscillatory", 2: "product_peak"}
# VALU issue peak: one wave64 instruction per SIMD per quad-cycle (16 lanes a
# clock): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-slots/s
PEAK_VALU = 256 * 4 * 16 * 2.4e9
# a transcendental holds the VALU for two quad-cycles (19.6 T measured)
PEAK_TRANS = PEAK_VALU / 2
PEAK_FP32_FLOPS = 157.3e12  # published dense FP32 vector rate (packed FMA)
PEAK_FP64_FLOPS = 78.6e12   # published FP64 vector rate


class Stats(C.Structure):
    _fields_ = [("dosample_launches", C.c_longlong), ("dosample_ms", C.c_double),
                ("refine_launches", C.c_longlong), ("refine_ms", C.c_double),
                ("evals", C.c_longlong), ("rule_launches", C.c_longlong),
                ("rule_ms", C.c_double), ("rule_evals", C.c_longlong),
                ("fold_ms", C.c_double), ("dosample_busy_ms", C.c_double)]


def _stats(cc, ctx, reset=True):
    fn = cc._lib.ccuba_stats_get
    fn.argtypes = [C.c_void_p, C.POINTER(Stats), C.c_int]
    st = Stats()
    fn(ctx.handle, C.byref(st), 1 if reset else 0)
    return st


_JOBS = {}


def _headline_jobs(cc, params, prec):
    """The step's integrals as one batch: every iteration samples both in one
    DoSample launch, and one fold and one refine launch finish both."""
    if prec not in _JOBS:
        specs = [dict(method=0, family=fam, a=params[fam][0], u=params[fam][1], flags=prec,
                      seed=1, stream_id=0, nstart=NPTS, maxeval=ITERS * NPTS, nbins=NBINS)
                 for fam in FAMILIES]
        _JOBS[prec] = cc.make_jobs(specs)
    return _JOBS[prec]


def _tune_cache():
    """The autotuner's cache file (CCUBA_TUNE_CACHE; a file in the temporary
    directory unless set)."""
    path = os.environ.get("CCUBA_TUNE_CACHE")
    if not path:
        import tempfile
        path = os.path.join(tempfile.gettempdir(), "ccuba_tune_cache.txt")
        os.environ["CCUBA_TUNE_CACHE"] = path
    return path


def _ensure_tuned():
    """Tune the headline batch in a child process (untimed, and outside any
    profiler that wraps a later run once the cache exists), so that this
    process's headline context finds its settings in the cache."""
    import subprocess
    path = _tune_cache()
    if os.path.exists(path) and ":batch:" in open(path).read():
        return
    subprocess.run([sys.executable, os.path.abspath(__file__), "--tune-only"], check=True,
                   stdout=subprocess.DEVNULL)


def _tuned_settings(ctx, prec):
    return {k: ctx.config_get(k, prec) for k in ("block", "blocks_per_cu", "ilp", "min_tile",
                                                 "hist64", "batch_streams")}


def _step(cc, ctx, params, prec):
    ev = 0
    for r in cc.vegas_batch(ctx, _headline_jobs(cc, params, prec)):
        if r["neval"] != ITERS * NPTS or r["status"] != 0:
            raise RuntimeError("unexpected result %r" % (r,))
        ev += r["neval"]
    return ev


def _timed(cc, ctx, params, prec, steps, warmup, warm_s=0.0):
    """W untimed warm-up steps, then more untimed steps until warm_s seconds
    have passed since the first (the GPU's clocks settle over the first tens
    of milliseconds of work: the steps of a cold start speed up by ~10% over
    the first 25 ms), then exactly `steps' timed steps."""
    import torch
    t_warm = time.perf_counter() + warm_s
    for _ in range(warmup):
        _step(cc, ctx, params, prec)
    while time.perf_counter() < t_warm:
        _step(cc, ctx, params, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = 0
    for _ in range(steps):
        ev += _step(cc, ctx, params, prec)
    torch.cuda.synchronize()
    return ev, time.perf_counter() - t0


def _counters():
    """The committed VALU counter summary, with each kernel's entry kept only
    while the sources it was taken on are unchanged."""
    path = os.path.join(ROOT, "profiles", "valu_counters.json")
    if not os.path.exists(path):
        return {}
    rec = json.load(open(path))
    ks = rec.get("kernels", {})
    out = {}
    if rec.get("kernel_source_sha256") == kernel_source_hash(rec.get("kernel_sources", [])):
        for k, v in ks.items():
            if k.startswith("dosample"):
                # the points the probe's step sampled in this kernel
                pts = rec.get("probe", {}).get(k + "_points")
                out[k] = dict(v, points=pts)
    if rec.get("cuhre_source_sha256") == kernel_source_hash(rec.get("cuhre_sources", [])):
        if "cuhre_rule" in ks:
            out["cuhre_rule"] = dict(ks["cuhre_rule"], evals=rec["probe"]["cuhre_evals"])
    return out


def _valu_fields(c, units, seconds, flops_peak):
    """Roofline fields from counter totals `c' over `units' points (or
    evaluations) and the live seconds those units take: VALU slot rate against
    the issue peak, FP32/FP64 FLOP rate, transcendental rate, dual issue."""
    k = c["counters"]
    g = lambda n: k.get(n, 0.0)
    lanes = 64.0
    slots = g("SQ_ACTIVE_INST_VALU") * lanes / units  # quad-cycle slots per unit
    instrs = g("SQ_INSTS_VALU") * lanes / units
    f32 = lanes * (2 * g("SQ_INSTS_VALU_FMA_F32") + g("SQ_INSTS_VALU_ADD_F32") +
                   g("SQ_INSTS_VALU_MUL_F32")) / units
    f64 = lanes * (2 * g("SQ_INSTS_VALU_FMA_F64") + g("SQ_INSTS_VALU_ADD_F64") +
                   g("SQ_INSTS_VALU_MUL_F64")) / units
    trans = lanes * (g("SQ_INSTS_VALU_TRANS_F32") + g("SQ_INSTS_VALU_TRANS_F64")) / units
    rate = units / seconds
    achieved = slots * rate
    # VALU busy over the counter run alone (rocprof's VALUBusy: busy
    # quad-cycles per CU over the active clocks of one XCD's 32 CUs)
    disp = max(c.get("dispatches", 1), 1)
    grbm = g("GRBM_GUI_ACTIVE") / disp / 8
    busy = (g("SQ_ACTIVE_INST_VALU") / disp) / (256 * grbm) if grbm > 0 else None
    out = {"achieved": achieved / 1e12, "frac": achieved / PEAK_VALU,
           "slots_per_unit": slots, "valu_instructions_per_unit": instrs,
           "valu_busy_counter_run": busy,
           "dual_issue_quad_cycle_frac": (g("SQ_ACTIVE_INST_VALU2") / g("SQ_ACTIVE_INST_VALU")
                                          if g("SQ_ACTIVE_INST_VALU") else None),
           "int32_per_unit": lanes * g("SQ_INSTS_VALU_INT32") / units,
           "int64_per_unit": lanes * g("SQ_INSTS_VALU_INT64") / units,
           "lds_per_unit": lanes * g("SQ_INSTS_LDS") / units,
           "fp32_flops_per_unit": f32, "fp64_flops_per_unit": f64,
           "trans_per_unit": trans,
           "trans_per_s": trans * rate, "trans_frac": trans * rate / PEAK_TRANS}
    if flops_peak == PEAK_FP32_FLOPS:
        out.update(fp32_tflops=f32 * rate / 1e12, fp32_flop_frac=f32 * rate / PEAK_FP32_FLOPS)
    else:
        out.update(fp64_tflops=f64 * rate / 1e12, fp64_flop_frac=f64 * rate / PEAK_FP64_FLOPS)
    return out


def _roofline(cc, ctx, params, prec):
    """Event-timed DoSample sampling launches of one profiled headline step.

    The library records HIP events on the stream each kernel runs on around
    the sampling kernel, the fold of its partial sums and the refine kernel
    of every iteration.  The step runs as the timed steps do: its two
    integrals as two halves on two streams, whose sampling launches overlap
    in time, so the library also reports the time during which at least one
    sampling launch ran (the union of their intervals, from the same
    events).  The sampling kernel is the dominant one and the roofline is its
    VALU issue rate: the VALU quad-cycles per point that rocprofv3's SQ
    counters measured on this kernel (SQ_ACTIVE_INST_VALU, committed under
    profiles/) x the step's points / that busy time, against one wave64
    instruction per SIMD per quad-cycle.  The slot model counted from the
    assembly (isa_slots.py) is reported beside it."""
    from paper_1408_6373_amd import isa_slots
    table = isa_slots.load() or {}
    _stats(cc, ctx)
    ctx.config("profile", 1)
    _step(cc, ctx, params, prec)
    st = _stats(cc, ctx)
    ctx.config("profile", 0)
    ms, fold_ms, refine_ms = st.dosample_ms, st.fold_ms, st.refine_ms
    busy = st.dosample_busy_ms
    evals, launches = st.evals, st.dosample_launches
    n = max(launches, 1)
    fp32 = prec == cc.FP32_EVAL
    # the instance at d = 8, 128 bins: 2 Philox blocks per point, power-of-two
    # bin count, d = 4 x blocks; histogram type and points per lane as set
    t = _tuned_settings(ctx, prec)
    h64, ilp = t["hist64"], t["ilp"]
    key = "%s%s_ilp%d_nb2_pow2_full" % ("f32" if fp32 else "f64", "h64" if h64 else "hfx", ilp)
    name = "vegas_dosample_kernel<%s,%s,%d,2,true,true>" % (
        "float" if fp32 else "double", "double" if h64 else "unsigned long long", ilp)
    model = 0.0
    for fam in FAMILIES:  # each integral contributes ITERS x NPTS points
        per = table.get(key, {}).get(FAMILY_KEYS[fam])
        model = None if (per is None or model is None) else model + per * ITERS * NPTS
    out = {"bound": "alu", "kernel": name, "launch": t, "unit": "T VALU-slots/s",
           "peak": PEAK_VALU / 1e12,
           "avg_launch_ms": ms / n, "launches": launches,
           "points_per_launch": evals / n,
           "busy_ms": busy, "launch_overlap": ms / busy if busy > 0 else None,
           "kernel_evals_per_s": evals / (busy * 1e-3),
           "fold_ms_per_launch": fold_ms / n,
           "refine_ms_per_launch": refine_ms / n,
           "achieved": None, "frac": None,
           "slot_model": None if model is None else {
               "slots_per_point": model / evals,
               "achieved": model / (busy * 1e-3) / 1e12,
               "frac": model / (busy * 1e-3) / PEAK_VALU}}
    c = _counters().get("dosample_fp32" if fp32 else "dosample_fp64")
    # counters taken on this precision and histogram type; when they were
    # taken on another instance (points per lane per trip), their slots per
    # point are scaled by the assembly counts of the two instances' loops
    scale = None
    if c and len(c.get("instances", [])) == 1:
        import re
        m = re.search(r"vegas_dosample_kernel<(\w+), ([\w ]+), (\d), 2, true, true>",
                      c["instances"][0])
        if m and (m.group(1) == "float") == fp32 and (m.group(2) == "double") == bool(h64):
            ckey = key.replace("_ilp%d_" % ilp, "_ilp%s_" % m.group(3))
            mk = [table.get(k, {}).get(FAMILY_KEYS[f]) for k in (key, ckey) for f in FAMILIES]
            scale = (1.0 if ckey == key else
                     None if None in mk else (mk[0] + mk[1]) / (mk[2] + mk[3]))
            out["counters_instance"] = c["instances"][0]
    if c and scale is not None:
        c = dict(c, counters={k: v * (scale if k.startswith("SQ_ACTIVE_INST_VALU") or
                                      k == "SQ_INSTS_VALU" else 1.0)
                              for k, v in c["counters"].items()})
        out["counters_isa_scale"] = scale
    else:
        c = None
    if c:
        # points of the counter run (one headline step)
        units = float(c.get("points") or ITERS * len(FAMILIES) * NPTS)
        out.update(_valu_fields(c, units, (busy * 1e-3) / evals * units,
                                PEAK_FP32_FLOPS if fp32 else PEAK_FP64_FLOPS))
        out["counters"] = "profiles/valu_counters.json"
    if fp32:
        out["traffic"] = _traffic(evals / n, t)
    return out


def _cuhre_roofline(st):
    """Cuhre's rule kernels: counter slots per evaluation x the evaluations per
    second that the library's HIP events measured around the rule launches of
    the cuhre leg."""
    c = _counters().get("cuhre_rule")
    if not c or st.rule_ms <= 0:
        return None
    rate = st.rule_evals / (st.rule_ms * 1e-3)
    out = {"bound": "alu", "kernel": "gm_rule_lane1_kernel<CORNER_PEAK,6> + gm_rule_lane_kernel<CORNER_PEAK,6> + gm_rule_kernel",
           "unit": "T VALU-slots/s", "peak": PEAK_VALU / 1e12, "evals_per_s": rate,
           "counters": "profiles/valu_counters.json"}
    out.update(_valu_fields(c, float(c["evals"]), c["evals"] / rate, PEAK_FP64_FLOPS))
    return out


# the sources the DoSample kernel is compiled from
KERNEL_SOURCES = ("vegas_sample.h", "vegas_sample_f32hfx.hip", "philox.h", "genz.h",
                  "engine.h", "vegas.h")


def kernel_source_hash(names=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_1408_6373_amd", "csrc", name), "rb").read())
    return h.hexdigest()


# the settings that shape a DoSample launch's tile plan (and so its bytes)
_PLAN_KEYS = ("block", "blocks_per_cu", "min_tile", "batch_streams")


def _traffic(points_per_launch, launch):
    """HBM bytes per DoSample launch from the committed PMC summary, if it was
    taken on the current kernel source, on launches of this size and with the
    same tile plan settings."""
    path = os.path.join(ROOT, "profiles", "vegas_dosample_d8_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    ppd = rec.get("dosample", {}).get("points_per_dispatch")
    if ppd is None or abs(ppd - points_per_launch) > 0.5:
        return None
    taken = rec.get("launch")
    if not taken or any(taken.get(k) != launch.get(k) for k in _PLAN_KEYS):
        return None
    return rec.get("bytes_per_launch")


def _read_pmc(path):
    """{kernel name: [counter value per dispatch]} from a rocprofv3 counter CSV."""
    import csv
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def summarize_pmc(fetch_csv, write_csv, out_path, commands, launch=None):
    """Write the HBM-traffic summary of the DoSample kernels of a
    --traffic-probe run: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, summed
    over the XCDs by rocprofv3), each scaled by what the same counter reads
    for the probe's 1 GiB device-to-device copy."""
    fetch, write = _read_pmc(fetch_csv), _read_pmc(write_csv)
    copy = "__amd_rocclr_copyBuffer"
    cf, cw = max(fetch.get(copy, [0])), max(write.get(copy, [0]))
    if cf <= 0 or cw <= 0:
        raise SystemExit("no 1 GiB copy dispatch in the counter files")
    gib = float(1 << 30)
    fs, ws = gib / (cf * 1024), gib / (cw * 1024)
    rec = {"what": "HBM bytes per dispatch of the FP32 DoSample kernels (one headline "
                   "step: Vegas d=8 oscillatory and product peak, 128 bins, 20 iterations "
                   "of 1e7 points each, launched as the tuned batch runs them) from "
                   "rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by the same counters on a "
                   "1 GiB device-to-device copy",
           "commands": commands,
           "copy_calibration": {"bytes": 1 << 30, "fetch_kib": cf, "write_kib": cw,
                                "fetch_scale": fs, "write_scale": ws}}
    for name, key in (("vegas_dosample_kernel", "dosample"), ("vegas_fold_kernel", "fold"),
                      ("vegas_fold2_kernel", "fold2")):
        fk = [v for k, vs in fetch.items() if name + "<" in k or name + "(" in k for v in vs]
        wk = [v for k, vs in write.items() if name + "<" in k or name + "(" in k for v in vs]
        if not fk or not wk:
            continue
        f_avg, w_avg = sum(fk) / len(fk), sum(wk) / len(wk)
        rec[key] = {"dispatches": len(fk), "fetch_kib": f_avg, "write_kib": w_avg,
                    "bytes": 1024 * (f_avg * fs + w_avg * ws)}
        if key == "dosample":  # the probe samples one headline step
            rec[key]["points_per_dispatch"] = ITERS * len(FAMILIES) * NPTS / len(fk)
    rec["kernel_sources"] = list(KERNEL_SOURCES)
    rec["kernel_source_sha256"] = kernel_source_hash()
    rec["bytes_per_launch"] = rec["dosample"]["bytes"]
    if launch:
        rec["launch"] = launch  # the tuned settings the probe ran with
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


# the kernels whose VALU counters the roofline uses: the headline DoSample
# instance in both precisions, and Cuhre's rule kernels
COUNTER_KERNELS = {
    # (a headline step launches one DoSample instance per precision)
    "dosample_fp32": "vegas_dosample_kernel<float",
    "dosample_fp64": "vegas_dosample_kernel<double",
    "cuhre_rule": "gm_rule",
}
# sources of the Cuhre rule kernels (the counter summary holds for them only
# while these are unchanged)
CUHRE_SOURCES = ("cuhre.hip", "genz.h", "engine.h")


def _read_counters(path):
    """{kernel name: {counter: [value per dispatch]}} from a rocprofv3 counter CSV."""
    import csv
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            d = out.setdefault(row["Kernel_Name"], {})
            d.setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    return out


def summarize_counters(csvs, out_path, commands, probe):
    """Write the VALU counter summary of --counter-probe runs: for each kernel
    of COUNTER_KERNELS, every counter's total over its dispatches and the
    dispatch count; `probe' is the probe's JSON line (its evaluation counts)."""
    rec = {"what": "rocprofv3 --pmc SQ counters of the DoSample kernels of one headline step "
                   "in each precision (Vegas d=8, oscillatory and product peak as one batch, 128 "
                   "bins, 2 x 1e7 points per launch, 20 launches) and of Cuhre's rule kernels "
                   "over one corner-peak d=6 run (batches of 1e5 regions to epsrel 1e-6); "
                   "counter values are totals over the dispatches (the SQ_ counters summed over "
                   "the shader engines by rocprofv3)",
           "commands": commands, "probe": probe, "kernels": {}}
    for path in csvs:
        for name, counters in _read_counters(path).items():
            for key, pat in COUNTER_KERNELS.items():
                if pat not in name:
                    continue
                k = rec["kernels"].setdefault(key, {"name": pat, "counters": {},
                                                    "dispatches": {}})
                for cn, vals in counters.items():
                    k["counters"][cn] = k["counters"].get(cn, 0.0) + sum(vals)
                    # dispatches of each matching kernel (the same in every pass)
                    k["dispatches"][name] = len(vals)
    for k in rec["kernels"].values():
        k["instances"] = sorted(k["dispatches"])
        k["dispatches"] = sum(k["dispatches"].values())
    rec["kernel_sources"] = list(KERNEL_SOURCES) + ["vegas_sample_f64.hip"]
    rec["kernel_source_sha256"] = kernel_source_hash(rec["kernel_sources"])
    rec["cuhre_sources"] = list(CUHRE_SOURCES)
    rec["cuhre_source_sha256"] = kernel_source_hash(CUHRE_SOURCES)
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def _union_ns(intervals):
    """Length of the union of (start, end) intervals."""
    total, hi, lo = 0, None, None
    for a, b in sorted(intervals):
        if hi is not None and a <= hi:
            hi = max(hi, b)
            continue
        if hi is not None:
            total += hi - lo
        lo, hi = a, b
    return total + (hi - lo if hi is not None else 0)


def summarize_stats(stats_csv, out_path, command, note):
    """Write a short text table from a rocprofv3 --stats kernel_stats.csv;
    with the run's kernel_trace.csv beside it, also each DoSample kernel's
    busy time: the union of its dispatches' intervals (launches on two
    streams overlap)."""
    import csv
    import glob
    rows = list(csv.DictReader(open(stats_csv, newline="")))
    traces = glob.glob(os.path.join(os.path.dirname(stats_csv), "*kernel_trace.csv"))
    with open(out_path, "w") as f:
        f.write("rocprofv3 kernel statistics (MI355X, gfx950)\n")
        f.write("command: %s\n%s\n\n" % (command, note))
        f.write("%-72s %7s %11s %11s %7s\n" % ("kernel", "calls", "avg_us", "total_ms", "pct"))
        for r in rows:
            name = r["Name"].replace("ccuba::", "")
            f.write("%-72s %7d %11.1f %11.2f %7.2f\n" % (
                name[:72], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
        if traces:
            iv = {}
            for r in csv.DictReader(open(traces[0], newline="")):
                if "vegas_dosample_kernel" in r["Kernel_Name"]:
                    iv.setdefault(r["Kernel_Name"], []).append(
                        (int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
            if not iv:
                return
            f.write("\nDoSample busy time (union of the dispatch intervals; calls overlap when "
                    "a batch runs as two halves on two streams)\n")
            f.write("%-72s %7s %11s %11s %9s\n" % ("kernel", "calls", "busy_ms", "sum_ms",
                                                   "overlap"))
            for name, v in sorted(iv.items()):
                u, t = _union_ns(v), sum(b - a for a, b in v)
                f.write("%-72s %7d %11.2f %11.2f %9.2f\n" % (
                    name.replace("ccuba::", "")[:72], len(v), u / 1e6, t / 1e6,
                    t / u if u else 0.0))


def _batch_leg(cc):
    import workloads as W
    jobs = W.batch_jobs(4096, seed=1000)
    specs = [dict(method=0, ndim=j["ndim"], family=j["family"], a=j["a"], u=j["u"],
                  seed=j["seed"], stream_id=j["stream_id"], nstart=j["nstart"],
                  maxeval=10 * j["nstart"], nbins=128, flags=cc.FP32_EVAL) for j in jobs]
    ctx = cc.Context(device=0)
    ctx.config("autotune", 1)
    prepared = cc.make_jobs(specs)  # argument marshalling, outside the timed call
    t0 = time.perf_counter()
    cc.vegas_batch(ctx, prepared)  # the first batch call tunes the launch on its jobs
    t_tune = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = cc.vegas_batch(ctx, prepared)
    dt = time.perf_counter() - t0
    tuned = {k: ctx.config_get(k) for k in ("blocks_per_cu", "ilp", "min_tile", "hist64",
                                            "batch_streams")}
    ctx.close()
    ev = sum(r["neval"] for r in res)
    return {"workload": "4096 Vegas integrals, d 2..12, 1e4..1e6 points x 10 iterations, FP32",
            "value": ev / dt, "unit": "evals/s", "seconds": dt, "evals": ev,
            "failed": sum(r["status"] != 0 for r in res), "autotuned": tuned,
            "first_call_with_tuning_s": t_tune}


def _caller_integrand_leg(cc):
    """Vegas of caller-evaluated integrands (ccuba_vegas_batched): a Gaussian at
    d = 8 written in torch on the GPU (points and values stay in HBM), and the
    same Gaussian in numpy on the host (points and values cross PCIe)."""
    import numpy as np
    import torch
    import workloads as W
    a, u = W.genz_params(W.GAUSSIAN, 8, 1)
    at = torch.tensor(np.asarray(a) ** 2, dtype=torch.float64, device="cuda")
    ut = torch.tensor(np.asarray(u), dtype=torch.float64, device="cuda")
    a2 = np.asarray(a) ** 2

    def fdev(x, f):
        f[:, 0] = torch.exp(-torch.sum(at * (x - ut) ** 2, dim=1))

    def fhost(x):
        return np.exp(-np.sum(a2 * (x - u) ** 2, axis=1))

    ctx = cc.Context(device=0)
    out = {"workload": "Vegas of a Gaussian d=8, 128 bins, FP64, ncomp 1: device integrand "
                       "(torch) 10 x 1e7 points in batches of 1e6; host integrand (numpy) "
                       "4 x 1e6 points in batches of 2.5e5", "unit": "evals/s"}
    for where, func, n, iters, nvec in (("device", fdev, 10**7, 10, 10**6),
                                        ("host", fhost, 10**6, 4, 250000)):
        kw = dict(ctx=ctx, where=where, nvec=nvec, nstart=n, maxeval=iters * n, nbins=128)
        cc.vegas_batched(func, 8, **dict(kw, maxeval=n))  # warm-up: allocations, torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cc.vegas_batched(func, 8, **kw)
        dt = time.perf_counter() - t0
        out[where] = {"value": r["neval"] / dt, "seconds": dt, "neval": r["neval"],
                      "nvec": nvec}
    # a device integrand given as source and compiled into DoSample: the
    # headline shape (d = 8, 128 bins, 20 x 1e7 points, FP32 evaluation)
    src = """
__device__ double ccuba_user(const double *x, int d, const double *a, const double *u) {
  double s = 0.0;
  for (int j = 0; j < d; ++j) { const double t = x[j] - u[j]; s = fma(a[j] * a[j], t * t, s); }
  return exp(-s);
}
__device__ float ccuba_user(const float *x, int d, const float *a, const float *u) {
  float s = 0.0f;
  for (int j = 0; j < d; ++j) { const float t = x[j] - u[j]; s = fmaf(a[j] * a[j], t * t, s); }
  return expf(-s);
}
"""
    kw = dict(ctx=ctx, flags=cc.FP32_EVAL, nbins=128, nstart=10**7, maxeval=20 * 10**7)
    t0 = time.perf_counter()
    cc.vegas_source(src, 8, a, u, **dict(kw, maxeval=10**7))  # compiles the kernel
    t_first = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = cc.vegas_source(src, 8, a, u, **kw)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    rb = cc.vegas(W.GAUSSIAN, a, u, **kw)
    dtb = time.perf_counter() - t0
    out["source"] = {"value": r["neval"] / dt, "seconds": dt, "neval": r["neval"],
                     "first_call_with_compile_s": t_first,
                     "builtin_gaussian_evals_per_s": rb["neval"] / dtb,
                     "workload": "Gaussian d=8 as device source, 128 bins, 20 x 1e7 points, "
                                 "FP32 evaluation"}
    ctx.close()
    out["value"] = out["device"]["value"]
    return out


def _cuhre_leg(cc, ctx):
    import workloads as W
    a, u = W.genz_params(W.CORNER_PEAK, 6, 1)
    kw = dict(epsrel=1e-6, maxeval=10**10, max_regions_per_batch=10**5)
    # warm-up runs for 0.1 s, then 11 timed runs; a run is ~0.6 ms, so the
    # median of several stands for it better than one
    t_warm = time.perf_counter() + 0.1
    while time.perf_counter() < t_warm:
        cc.cuhre(W.CORNER_PEAK, a, u, ctx=ctx, **kw)
    times = []
    for _ in range(11):
        t0 = time.perf_counter()
        r = cc.cuhre(W.CORNER_PEAK, a, u, ctx=ctx, **kw)
        times.append(time.perf_counter() - t0)
    times.sort()
    dt = times[len(times) // 2]
    # the rule kernel alone, event-timed in a separate profiled run
    _stats(cc, ctx)
    ctx.config("profile", 1)
    cc.cuhre(W.CORNER_PEAK, a, u, ctx=ctx, **kw)
    st = _stats(cc, ctx)
    ctx.config("profile", 0)
    return {"workload": "Cuhre corner peak d=6, batches of 1e5 regions, epsrel 1e-6, FP64",
            "value": r["neval"] / dt, "unit": "evals/s", "seconds": dt,
            "runs": len(times), "seconds_min": times[0], "seconds_max": times[-1],
            "neval": r["neval"],
            "nregions": r["nregions"], "fail": r["fail"],
            "rule_kernel_evals_per_s": st.rule_evals / max(st.rule_ms * 1e-3, 1e-12),
            "rule_launches": st.rule_launches, "roofline": _cuhre_roofline(st)}


SUAVE_NNEW, SUAVE_SPLIT, SUAVE_STEPS = 1 << 17, 64, 30


def _suave_maxeval(nnew, K, steps):
    """Budget of the root sampling plus `steps` steps (K regions split per step
    once that many exist)."""
    m, R = nnew, 1
    for _ in range(steps):
        k = min(K, R)
        m += 2 * k * nnew
        R += k
    return m


def _suave_leg(cc, ctx, cpu=True):
    import workloads as W
    a, u = W.genz_params(W.GAUSSIAN, 8, 1)
    kw = dict(nnew=SUAVE_NNEW, nsplit=SUAVE_SPLIT, nbins=128, flatness=25.0,
              maxeval=_suave_maxeval(SUAVE_NNEW, SUAVE_SPLIT, SUAVE_STEPS))
    cc.suave(W.GAUSSIAN, a, u, ctx=ctx, **kw)  # warm-up (buffers, code objects)
    best = None
    for _ in range(3):  # the call returns once its results are on the host
        t0 = time.perf_counter()
        r = cc.suave(W.GAUSSIAN, a, u, ctx=ctx, **kw)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    out = {"workload": "Suave Gaussian d=8, 128 bins, nnew=2^17 points per region, 64 splits "
                       "per step, flatness 25, 30 steps, FP64",
           "value": r["neval"] / best, "unit": "evals/s", "seconds": best,
           "neval": r["neval"], "nregions": r["nregions"],
           "rel_error": r["error"] / abs(r["integral"])}
    if cpu:  # the oracle on the first 4 steps of the same workload (about 4e6 points)
        import oracle as O
        okw = dict(kw, maxeval=_suave_maxeval(SUAVE_NNEW, SUAVE_SPLIT, 4))
        t0 = time.perf_counter()
        o = O.suave(O.genz(W.GAUSSIAN, a, u), 8, **okw)
        odt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": o["neval"] / odt, "unit": "evals/s", "cores": 1,
                             "kind": "oracle", "sample": "root + 4 steps (%d points)" % o["neval"]}
    return out


def _checkpoint_leg(cc, ctx):
    """Vegas at the headline shape (oscillatory d=8, 128 bins, 20 x 1e7 points,
    FP32 evaluation) without and with a state file written after every
    iteration, and started from a kept grid (gridno)."""
    import tempfile
    import workloads as W
    a, u = W.genz_params(W.OSCILLATORY, D, 1)
    kw = dict(ctx=ctx, flags=cc.FP32_EVAL, nbins=NBINS, nstart=NPTS, maxeval=ITERS * NPTS, seed=1)
    cc.vegas(W.OSCILLATORY, a, u, **kw)  # warm-up

    def best(**extra):
        t = None
        for _ in range(3):
            t0 = time.perf_counter()
            r = cc.vegas(W.OSCILLATORY, a, u, **dict(kw, **extra))
            dt = time.perf_counter() - t0
            t = dt if t is None else min(t, dt)
        return r, t

    plain, tp = best()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "vegas.state")
        t = None
        for _ in range(3):
            if os.path.exists(path):
                os.remove(path)
            t0 = time.perf_counter()
            r = cc.vegas(W.OSCILLATORY, a, u, statefile=path, **kw)
            dt = time.perf_counter() - t0
            t = dt if t is None else min(t, dt)
        ts, state_bytes = t, os.path.getsize(path)
    cc.vegas(W.OSCILLATORY, a, u, gridno=7, **kw)  # keeps its final grid in slot 7
    reused, tg = best(gridno=-7)
    return {"workload": "Vegas oscillatory d=8, 128 bins, 20 x 1e7 points, FP32 evaluation",
            "unit": "evals/s",
            "plain": {"value": plain["neval"] / tp, "seconds": tp},
            "statefile": {"value": plain["neval"] / ts, "seconds": ts,
                          "per_iteration_us": 1e6 * (ts - tp) / ITERS,
                          "file_bytes": state_bytes,
                          "rel_diff_from_plain": abs(r["integral"] - plain["integral"]) / abs(plain["integral"])},
            "gridno_reuse": {"value": reused["neval"] / tg, "seconds": tg,
                             "rel_error": reused["error"] / abs(reused["integral"]),
                             "plain_rel_error": plain["error"] / abs(plain["integral"])}}


DIV_NSEARCH, DIV_NITER, DIV_REGIONS, DIV_SPLIT = 1024, 64, 16384, 1024


def _divonne_leg(cc, ctx, cpu=True):
    import workloads as W
    a, u = W.genz_params(W.GAUSSIAN, 8, 1)
    kw = dict(nsearch=DIV_NSEARCH, niter=DIV_NITER, maxregions=DIV_REGIONS, nsplit=DIV_SPLIT)
    cc.divonne_partition(W.GAUSSIAN, a, u, ctx=ctx, **kw)  # warm-up
    best = None
    for _ in range(3):  # the call returns once its results are on the host
        t0 = time.perf_counter()
        r = cc.divonne_partition(W.GAUSSIAN, a, u, ctx=ctx, **kw)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    searches = 2 * r["nregions"] - 1
    out = {"workload": "Divonne partitioning phase, Gaussian d=8, 1024 search points and 64 "
                       "compass iterations per extremum, 1024 splits per step, to 16384 regions",
           "value": r["neval"] / best, "unit": "evals/s", "seconds": best,
           "region_searches_per_s": searches / best, "neval": r["neval"],
           "nregions": r["nregions"], "total_spread": r["total_spread"]}
    if cpu:  # the oracle on the same workload up to 4096 regions
        import oracle as O
        t0 = time.perf_counter()
        o = O.divonne_partition(O.genz(W.GAUSSIAN, a, u), 8, **dict(kw, maxregions=4096))
        odt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": o["neval"] / odt, "unit": "evals/s", "cores": 1,
                             "kind": "oracle",
                             "sample": "the same partition to 4096 regions (%d evaluations)"
                                       % o["neval"]}
    return out


def _serving_specs(cc, reqs):
    specs = []
    for r in reqs:
        if r["method"] == 0:
            specs.append(dict(method=0, ndim=r["ndim"], family=r["family"], a=r["a"], u=r["u"],
                              seed=r["seed"], stream_id=r["stream_id"], epsrel=r["epsrel"],
                              nstart=200000, nincrease=100000, maxeval=10**8, nbins=128,
                              flags=cc.FP32_EVAL))
        else:
            specs.append(dict(method=1, ndim=r["ndim"], family=r["family"], a=r["a"], u=r["u"],
                              epsrel=r["epsrel"], maxeval=10**8, max_regions_per_batch=10**5,
                              flags=0))
    return specs


def _serving_run(cc, W, n, rate):
    """n requests of the stream arriving at `rate' per second (Poisson), on a
    fresh context; returns the per-request results."""
    reqs = W.serving_requests(n, rate=rate, seed=7)
    specs = _serving_specs(cc, reqs)
    ctx = cc.Context(device=0)
    start = time.perf_counter()
    tickets = []
    for r, s in zip(reqs, specs):
        delay = start + r["arrival"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(cc.submit(ctx, s))
    cc.drain(ctx)
    res = [cc.poll(ctx, t) for t in tickets]
    ctx.close()
    return reqs, res


def _latency_rows(res):
    import numpy as np
    lat = np.array([r["t_done"] - r["t_submit"] for r in res]) * 1e3
    fail = np.array([r["fail"] for r in res])
    out = {}
    for key, m in (("all", np.ones(len(res), bool)), ("converged", fail == 0),
                   ("budget_capped", fail == 1)):
        if m.any():
            out[key] = {"count": int(m.sum()), "p50_ms": float(np.percentile(lat[m], 50)),
                        "p99_ms": float(np.percentile(lat[m], 99))}
    return out


def _serving_leg(cc, n, fracs=(0.3, 0.5, 0.7, 0.9)):
    import workloads as W
    # saturation throughput: every request queued at once
    ctx = cc.Context(device=0)
    specs = _serving_specs(cc, W.serving_requests(n, rate=1.0, seed=7))
    t0 = time.perf_counter()
    tickets = [cc.submit(ctx, s) for s in specs]
    cc.drain(ctx)
    t_sat = time.perf_counter() - t0
    for t in tickets:
        cc.poll(ctx, t)
    ctx.close()
    sat = n / t_sat
    rows = []
    for frac in fracs:  # Poisson arrivals at fractions of saturation
        reqs, res = _serving_run(cc, W, n, frac * sat)
        ev = sum(r["neval"] for r in res)
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        rows.append({"load": frac, "rate_per_s": frac * sat, "requests": n,
                     "latency": _latency_rows(res), "evals_per_s": ev / span,
                     "failed_status": sum(r["status"] != 0 for r in res)})
    head = next(r for r in rows if r["load"] == 0.7)
    return {"workload": "Poisson arrivals, 70%% Vegas (FP32) / 30%% Cuhre (FP64), d 2..16, "
                        "epsrel logU[1e-5,1e-3], maxeval 1e8, %d requests per load" % n,
            "saturation_per_s": sat, "rates": rows,
            "rate_per_s": head["rate_per_s"], "p50_ms": head["latency"]["all"]["p50_ms"],
            "p99_ms": head["latency"]["all"]["p99_ms"], "evals_per_s": head["evals_per_s"]}


def _host():
    """The host CPU's model name and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cores_available": avail}


def _cpu_baseline(cc, params, iters_sample=4, max_threads=16):
    """The oracle on the first `iters_sample` of the 20 iterations of both
    headline integrals (FP64): once in one thread, then as one independent
    oracle run per thread on all the cores the process may use (up to
    max_threads; the oracle is plain C behind ctypes, which releases the
    GIL).  The same sample is also run on the GPU in both precisions, and
    every result is compared with the single-thread oracle's (parity)."""
    import concurrent.futures as cf
    import oracle as O

    def one(fam):
        a, u = params[fam]
        return O.vegas(O.genz(fam, a, u), D, nbins=NBINS, nstart=NPTS,
                       maxeval=iters_sample * NPTS, seed=1)
    host = _host()
    t0 = time.perf_counter()
    ref = {fam: one(fam) for fam in FAMILIES}
    dt1 = time.perf_counter() - t0
    ev1 = sum(r["neval"] for r in ref.values())
    T = max(1, min(host["cores_available"] or 1, max_threads))
    fams = [FAMILIES[q % len(FAMILIES)] for q in range(T)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=T) as ex:
        runs = list(ex.map(one, fams))
    dtT = time.perf_counter() - t0
    evT = sum(r["neval"] for r in runs)
    # the GPU on the same sample: the headline batch path, both precisions
    parity = {}
    ctx = cc.Context(device=0)
    try:
        for prec, tag in ((cc.FP32_EVAL, "fp32_eval"), (cc.FP64, "fp64")):
            specs = [dict(method=0, family=fam, a=params[fam][0], u=params[fam][1], flags=prec,
                          seed=1, stream_id=0, nstart=NPTS, maxeval=iters_sample * NPTS,
                          nbins=NBINS) for fam in FAMILIES]
            for fam, r in zip(FAMILIES, cc.vegas_batch(ctx, specs)):
                o = ref[fam]
                parity.setdefault(FAMILY_KEYS[fam], {})[tag] = {
                    "integral_rel_diff": abs(r["integral"] - o["integral"]) / abs(o["integral"]),
                    "error_rel_diff": abs(r["error"] - o["error"]) / abs(o["error"]),
                    "prob_abs_diff": abs(r["prob"] - o["prob"])}
    finally:
        ctx.close()
    sample = ("first %d of 20 iterations (10^7 points each) of both integrals, FP64; %d threads "
              "each run the oracle on one of them (%d evals in %.1f s)"
              % (iters_sample, T, evT, dtT))
    return dict(value=evT / dtT, unit="evals/s", cores=T, kind="oracle", sample=sample,
                host=host,
                single_thread={"value": ev1 / dt1, "cores": 1, "evals": ev1, "seconds": dt1},
                parity_vs_fp64_oracle=parity)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--warm-seconds", type=float, default=0.25,
                    help="untimed headline steps continue for at least this long before "
                         "the timed ones (GPU clocks settle)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip batch/cuhre/serving legs")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--suave-only", action="store_true",
                    help="run only the Suave leg and print its JSON line (for profiling)")
    ap.add_argument("--divonne-only", action="store_true",
                    help="run only the Divonne-partition leg and print its JSON line")
    ap.add_argument("--cuhre-only", action="store_true",
                    help="run only the Cuhre leg and print its JSON line")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg and print its JSON line")
    ap.add_argument("--checkpoint-only", action="store_true",
                    help="run only the state-file / grid-reuse leg and print its JSON line")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for PMC runs: one 1 GiB device copy (calibration), then one FP32 "
                         "step of the headline workload; prints a JSON line")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT"),
                    help="write the traffic summary of two --traffic-probe counter runs")
    ap.add_argument("--probe-line", default="",
                    help="with --pmc-summary: a file holding the probe's JSON line (its "
                         "launch settings are recorded)")
    ap.add_argument("--tune-only", action="store_true",
                    help="autotune the headline batch in both precisions into the tune cache "
                         "(CCUBA_TUNE_CACHE) and exit")
    ap.add_argument("--counter-probe", action="store_true",
                    help="for PMC runs: one headline step in each precision and one Cuhre run "
                         "of the corner peak at d = 6; prints a JSON line")
    ap.add_argument("--counter-summary", nargs="+", metavar="ARG",
                    help="OUT PROBE_JSON CSV...: write the VALU counter summary of "
                         "--counter-probe runs")
    ap.add_argument("--stats-summary", nargs=2, metavar=("STATS_CSV", "OUT"),
                    help="write a text table of a rocprofv3 kernel_stats.csv")
    ap.add_argument("--command", default="", help="command recorded in a summary")
    ap.add_argument("--note", default="", help="note recorded in a stats summary")
    args = ap.parse_args()
    if args.pmc_summary:
        cmds = [c for c in args.command.split(";;") if c]
        probe = {}
        if args.probe_line:
            probe = json.loads([x for x in open(args.probe_line) if x.startswith("{")][0])
        print(json.dumps(summarize_pmc(*args.pmc_summary[:2], args.pmc_summary[2], cmds,
                                       probe.get("launch"))))
        return
    if args.stats_summary:
        summarize_stats(args.stats_summary[0], args.stats_summary[1], args.command, args.note)
        return
    if args.counter_summary:
        out, probe, csvs = args.counter_summary[0], args.counter_summary[1], args.counter_summary[2:]
        cmds = [c for c in args.command.split(";;") if c]
        rec = summarize_counters(csvs, out, cmds, json.load(open(probe)))
        print(json.dumps({k: v.get("dispatches") for k, v in rec["kernels"].items()}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); no multi-GPU path exists",
              file=sys.stderr)
        sys.exit(2)

    if not (args.tune_only or args.counter_probe or args.traffic_probe or args.suave_only or
            args.divonne_only or args.checkpoint_only or args.serving_only or
            args.cuhre_only):
        _ensure_tuned()

    import torch
    import paper_1408_6373_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    params = {fam: W.genz_params(fam, D, 1) for fam in FAMILIES}
    if args.traffic_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        _tune_cache()
        ctx = cc.Context(device=0)
        ctx.config("autotune", 1)  # the tuned settings, from the cache
        ev = _step(cc, ctx, params, cc.FP32_EVAL)
        launch = _tuned_settings(ctx, cc.FP32_EVAL)
        ctx.close()
        print(json.dumps({"traffic_probe": True, "copy_bytes": 1 << 30, "neval": ev,
                          "launch": launch}))
        return
    if args.tune_only:
        _tune_cache()
        ctx = cc.Context(device=0)
        ctx.config("autotune", 1)
        for prec in (cc.FP32_EVAL, cc.FP64):
            _step(cc, ctx, params, prec)
        print(json.dumps({p: _tuned_settings(ctx, p) for p in (cc.FP32_EVAL, cc.FP64)}))
        ctx.close()
        return
    if args.counter_probe:
        # the tuned headline settings, read from the cache that a plain run of
        # the benchmark (or --tune-only) wrote before; tuning here would add
        # its own DoSample dispatches to the counted ones
        path = _tune_cache()
        if not (os.path.exists(path) and ":batch:" in open(path).read()):
            print("bench.py --counter-probe: no tuned settings in %s; run bench.py --tune-only "
                  "first, outside the profiler" % path, file=sys.stderr)
            sys.exit(2)
        ctx = cc.Context(device=0)
        ctx.config("autotune", 1)
        ev32 = _step(cc, ctx, params, cc.FP32_EVAL)
        ev64 = _step(cc, ctx, params, cc.FP64)
        a, u = W.genz_params(W.CORNER_PEAK, 6, 1)
        r = cc.cuhre(W.CORNER_PEAK, a, u, ctx=ctx, epsrel=1e-6, maxeval=10**10,
                     max_regions_per_batch=10**5)
        ctx.close()
        print(json.dumps({"counter_probe": True, "dosample_fp32_points": ev32,
                          "dosample_fp64_points": ev64, "cuhre_evals": r["neval"],
                          "cuhre_regions": r["nregions"]}))
        return
    if args.serving_only:
        print(json.dumps({"serving": _serving_leg(cc, args.serving_requests)}))
        return
    ctx = cc.Context(device=0)
    if args.suave_only or args.divonne_only or args.checkpoint_only or args.cuhre_only:
        leg = ({"suave": _suave_leg(cc, ctx, cpu=False)} if args.suave_only else
               {"cuhre": _cuhre_leg(cc, ctx)} if args.cuhre_only else
               {"divonne_partition": _divonne_leg(cc, ctx, cpu=False)} if args.divonne_only
               else {"checkpoint": _checkpoint_leg(cc, ctx)})
        print(json.dumps(leg))
        ctx.close()
        return

    # the headline on its own context, with the launch settings the autotuner
    # picked for this batch (read from its cache)
    hctx = cc.Context(device=0)
    hctx.config("autotune", 1)
    ev32, t32 = _timed(cc, hctx, params, cc.FP32_EVAL, args.steps, args.warmup,
                       args.warm_seconds)
    value = ev32 / t32
    out = {
        "metric": "integrand evals/s (Vegas d=8, FP32 vs FP64) + p50/p99 solve latency",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "warm_seconds": args.warm_seconds,
        "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "accumulate": "f64", "data": "synthetic",
        "config": {"workload": "vegas_d8_genz_oscillatory+product_peak_20x1e7_128bins",
                   "ndim": D, "nbins": NBINS, "points_per_iteration": NPTS,
                   "iterations": ITERS, "integrals_per_step": len(FAMILIES)},
    }
    if not args.no_fp64:
        ev64, t64 = _timed(cc, hctx, params, cc.FP64, args.steps, args.warmup,
                           args.warm_seconds)
        out["fp64"] = {"value": ev64 / t64, "unit": "evals/s",
                       "ms_per_step": 1e3 * t64 / args.steps,
                       "fp32_speedup": value / (ev64 / t64)}
    out["launch"] = {"fp32": _tuned_settings(hctx, cc.FP32_EVAL),
                     "fp64": _tuned_settings(hctx, cc.FP64), "autotuned": True}
    out["roofline"] = _roofline(cc, hctx, params, cc.FP32_EVAL)
    if not args.no_fp64:
        out["fp64"]["roofline"] = _roofline(cc, hctx, params, cc.FP64)
    # the same counter slots over the whole timed step (sampling, folds,
    # refines and every gap): what the step as a whole makes of the VALU peak
    for ro, ev, t in ((out["roofline"], ev32, t32),) + (
            ((out["fp64"]["roofline"], ev64, t64),) if not args.no_fp64 else ()):
        if ro.get("slots_per_unit"):
            ro["step_achieved"] = ro["slots_per_unit"] * ev / t / 1e12
            ro["step_frac"] = ro["slots_per_unit"] * ev / t / PEAK_VALU
    hctx.close()
    if not args.no_extra:
        out["batch"] = _batch_leg(cc)
        out["caller_integrand"] = _caller_integrand_leg(cc)
        out["checkpoint"] = _checkpoint_leg(cc, ctx)
        out["cuhre"] = _cuhre_leg(cc, ctx)
        out["suave"] = _suave_leg(cc, ctx, cpu=not args.no_cpu_baseline)
        out["divonne_partition"] = _divonne_leg(cc, ctx, cpu=not args.no_cpu_baseline)
    ctx.close()
    if not args.no_extra:
        out["serving"] = _serving_leg(cc, args.serving_requests)
        out["p50_ms"] = out["serving"]["p50_ms"]
        out["p99_ms"] = out["serving"]["p99_ms"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(cc, params)
        out["parity"] = {"against": "the FP64 oracle on the cpu_baseline sample (4 of 20 "
                                    "iterations of both headline integrals)",
                         "results": out["cpu_baseline"]["parity_vs_fp64_oracle"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
