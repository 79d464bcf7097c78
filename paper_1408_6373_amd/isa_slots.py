"""VALU issue slots per sample point of the DoSample kernels, counted from the
gfx950 assembly of this build.

The roofline of the Vegas DoSample kernel is the VALU issue rate: every
point is produced in registers, so HBM traffic is negligible and there is
no matrix contraction.  This script compiles ``csrc/vegas.hip`` to gfx950
assembly with the library's flags, finds the per-point loop of each kernel
instance and family, and weighs its VALU instructions by their issue cost
relative to a full-rate FP32 operation (78.6 T lane-ops/s on MI355X = the
published 157.3 TFLOP/s FP32 vector peak / 2 flops per FMA):

  * FP32 / 32-bit integer operations              1 slot
  * FP64 operations (half rate)                   2 slots
  * 64-bit integer multiply-add, transcendentals  4 slots (quarter rate)

A loop's slots divided by the points it handles per trip (ILP) is the
work per point; times the points of a launch it is the launch's work.

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
    if op.startswith(("v_mad_u64_u32", "v_mad_i64_i32")):
        return 4
    if any(t in op for t in ("v_exp_", "v_log_", "v_rcp_", "v_rsq_", "v_sqrt_", "v_sin_",
                             "v_cos_")):
        return 4
    if "f64" in op:
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


def _family(ops, nested):
    has_exp = any(o.startswith("v_exp_") for o in ops)
    has_div = any(o.startswith("v_div_scale") for o in ops)
    if has_div:
        return "corner_peak" if nested else "product_peak"
    if has_exp:
        # C0 takes |x - u| (one v_and per dimension on the sign bit)
        n_and = sum(o.startswith("v_and_b32") for o in ops)
        return "c0" if n_and >= 4 else "gaussian"
    return "oscillatory"


def count(asm_text):
    """{kernel instance: {family: slots per point}} from gfx950 assembly."""
    res = {}
    for kern in re.findall(r"^(_ZN5ccuba21vegas_dosample_kernelI\w+):", asm_text, re.M):
        m = re.search(r"kernelI(\w)(\w)Li(\d)ELi(\d)ELb(\d)E", kern)
        if not m:
            continue
        T, H, ilp, nb, pow2 = m.groups()
        start = asm_text.index(kern + ":")
        body = asm_text[start:asm_text.index(".Lfunc_end", start)].splitlines()
        labels = {}
        for i, l in enumerate(body):
            mm = re.match(r"^(\.LBB\w+):", l)
            if mm:
                labels[mm.group(1)] = i
        loops = []
        for i, l in enumerate(body):
            mm = re.match(r"\s+s_cbranch_\w+\s+(\.LBB\w+)", l)
            if mm and mm.group(1) in labels and labels[mm.group(1)] < i:
                loops.append((labels[mm.group(1)], i))
        fam_slots = {}
        for a, b in loops:
            ops = _ops(body[a:b + 1])
            v = [o for o in ops if o.startswith("v_")]
            if len(v) < 80:
                continue
            # skip loops that contain another sampled loop (the outer tile loop)
            if sum(o.startswith("v_mad_u64_u32") for o in v) > 20 * int(nb) * int(ilp) + 8:
                continue
            nested = any(a < a2 and b2 < b for a2, b2 in loops)
            fam = _family(ops, nested)
            slots = sum(_weight(o) for o in v) / int(ilp)
            fam_slots.setdefault(fam, []).append(slots)
        key = "%s%s_ilp%s_nb%s%s" % ({"f": "f32", "d": "f64"}[T], {"f": "h32", "d": "h64"}[H],
                                     ilp, nb, "_pow2" if pow2 == "1" else "")
        res[key] = {f: max(v) for f, v in fam_slots.items()}
    return res


def _build_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_ccuba_build", os.path.join(HERE, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def compile_asm(hipcc=None, flags=None):
    if hipcc is None or flags is None:
        B = _build_module()
        hipcc, flags = B.HIPCC, B.FLAGS
    src = os.path.join(HERE, "csrc", "vegas.hip")
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "vegas.s")
        cmd = [hipcc, "-x", "hip"] + flags + ["--cuda-device-only", "-S", "-o", out, src]
        subprocess.run(cmd, check=True, capture_output=True)
        return open(out).read()


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
