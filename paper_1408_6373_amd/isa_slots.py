"""VALU issue slots per sample point of the DoSample kernels, counted from the
gfx950 assembly of this build (a static model, beside the rocprofv3 counters
the benchmark reads).

The roofline of the Vegas DoSample kernel is the VALU issue rate: every
point is produced in registers, so HBM traffic is negligible and there is
no matrix contraction.  This script compiles the DoSample translation
units (``csrc/vegas_sample_*.hip``) to gfx950 assembly with the library's
flags, finds the per-point loop of each kernel instance and family, and
weighs its VALU instructions by the quad-cycles (4 clocks, one wave64
instruction on a 16-lane SIMD) they hold the VALU for, as the SQ counters
count them (SQ_ACTIVE_INST_VALU is SQ_INSTS_VALU plus one more quad-cycle
per transcendental on the headline kernel):

  * every VALU instruction, FP64 and 64-bit integer multiply-add included,
    1 slot (measured issue rates on MI355X with independent chains: FP32 FMA
    37.6 T, FP64 FMA 35.7 T, v_mad_u64_u32 31.2 T lane-ops/s, against
    39.3 T = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz)
  * transcendentals and v_mul_hi_u32                2 slots (19.6 T measured)

A loop's slots divided by the points it handles per trip (ILP) is the
work per point; times the points of a launch and divided by the launch's
duration and 39.3 T slots/s it is the fraction of the VALU issue peak.
(Simple 32-bit integer and bit operations can issue two per quad-cycle on
gfx950 -- v_add_u32 60.4 T, v_bitop3_b32 55.3 T measured -- so the peak is
not a hard ceiling for every mix.)

Usage: ``python paper_1408_6373_amd/isa_slots.py`` writes ``kernel_slots.json``
next to this file (also done by build.py) and prints it.
"""
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "kernel_slots.json")
FAMILIES = ["gaussian", "oscillatory", "product_peak", "corner_peak", "c0"]


def _weight(op):
    if op.startswith("v_mul_hi_") or any(t in op for t in ("v_exp_", "v_log_", "v_rcp_",
                                                            "v_rsq_", "v_sqrt_", "v_sin_",
                                                            "v_cos_")):
        return 2
    return 1


def _ops(lines):
    out = []
    for line in lines:
        t = line.strip()
        if not t or t.startswith((".", ";")) or t.endswith(":"):
            continue
        out.append(t.split()[0])
    return out


def _drop_fallback(lines):
    """The fixed-point histogram kernels send the rare v^2 that cannot be
    summed exactly in fixed point to an FP64 histogram; drop the basic blocks
    of that path (those holding its FP64 LDS adds), which a point takes only
    in that case, so that the count is the path every other point takes."""
    blocks, cur = [], []
    for l in lines:
        if re.match(r"^(\.LBB\w+:|; %bb\.)", l) and cur:
            blocks.append(cur)
            cur = []
        cur.append(l)
    if cur:
        blocks.append(cur)
    return [l for blk in blocks if not any("ds_add_f64" in x for x in blk) for l in blk]


def count(asm_text):
    """{kernel instance: {family: slots per point}} from gfx950 assembly.

    Each family's per-point loop follows an assembly comment that the kernel
    source places just before it ("ccuba sample_tile family F"); the loop is
    the largest backward-branch region between that comment and the next
    one that holds no comment itself (a backward branch, conditional or not,
    closes a loop region)."""
    res = {}
    for kern in re.findall(r"^(_ZN5ccuba21vegas_dosample_kernelI\w+):", asm_text, re.M):
        m = re.search(r"kernelI(\w)(\w)Li(\d)ELi(\d)ELb(\d)ELb(\d)E", kern)
        if not m:
            continue
        T, H, ilp, nb, pow2, full = m.groups()
        start = asm_text.index(kern + ":")
        body = asm_text[start:asm_text.index(".Lfunc_end", start)].splitlines()
        labels, marks = {}, []
        for i, l in enumerate(body):
            mm = re.match(r"^(\.LBB\w+):", l)
            if mm:
                labels[mm.group(1)] = i
            mm = re.search(r"ccuba sample_tile family (\d+)", l)
            if mm:
                marks.append((i, int(mm.group(1))))
        loops = []
        for i, l in enumerate(body):
            mm = re.match(r"\s+s_(?:cbranch_\w+|branch)\s+(\.LBB\w+)", l)
            if mm and mm.group(1) in labels and labels[mm.group(1)] < i:
                loops.append((labels[mm.group(1)], i))
        fam_slots = {}
        for q, (mline, fam) in enumerate(marks):
            nxt = marks[q + 1][0] if q + 1 < len(marks) else len(body)
            best = None
            for a, b in loops:
                if not (mline < a < nxt) or any(a <= ml <= b for ml, _ in marks):
                    continue
                lines = body[a:b + 1]
                if H == "y":
                    lines = _drop_fallback(lines)
                v = [o for o in _ops(lines) if o.startswith("v_")]
                if best is None or len(v) > len(best):
                    best = v
            if best:
                fam_slots[FAMILIES[fam]] = sum(_weight(o) for o in best) / int(ilp)
        key = "%s%s_ilp%s_nb%s%s%s" % ({"f": "f32", "d": "f64"}[T], {"y": "hfx", "d": "h64"}[H],
                                       ilp, nb, "_pow2" if pow2 == "1" else "",
                                       "_full" if full == "1" else "")
        res[key] = fam_slots
    return res


def _build_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_ccuba_build", os.path.join(HERE, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def compile_asm(hipcc=None, flags=None):
    """gfx950 assembly of every DoSample translation unit, concatenated."""
    import concurrent.futures as cf
    if hipcc is None or flags is None:
        B = _build_module()
        hipcc, flags = B.HIPCC, B.FLAGS
    srcs = sorted(os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))
                  if f.startswith("vegas_sample_") and f.endswith(".hip"))
    with tempfile.TemporaryDirectory() as td:
        def one(src):
            out = os.path.join(td, os.path.basename(src) + ".s")
            cmd = [hipcc, "-x", "hip"] + flags + ["--cuda-device-only", "-S", "-o", out, src]
            subprocess.run(cmd, check=True, capture_output=True)
            return open(out).read()
        with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
            return "\n".join(ex.map(one, srcs))


def write(hipcc=None, flags=None):
    data = count(compile_asm(hipcc, flags))
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    return data


def load():
    if not os.path.exists(OUT):
        return None
    with open(OUT) as f:
        return json.load(f)


if __name__ == "__main__":
    print(json.dumps(write(), indent=1, sort_keys=True))
