"""Build ``libccuba.so`` (the HIP library behind include/ccuba.h) for gfx950.

Every source under ``csrc/`` is compiled by hipcc as HIP for gfx950 with FP
contraction off (every fused multiply-add is written out in the source) and
packed-FP32 instructions disabled, then linked into one shared library next
to this file.  Objects go to ``_build/`` at the repository root.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libccuba.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I" + INCLUDE, "-I" + CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-x", "hip"] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, msgs))
    return obj, msgs


def _slot_table():
    """VALU issue slots per point of each DoSample instance (roofline input)."""
    try:
        import importlib.util
        spec = importlib.util.spec_from_file_location("_ccuba_isa_slots",
                                                      os.path.join(HERE, "isa_slots.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.write(HIPCC, FLAGS)
        return None
    except Exception as e:  # the library itself is built; only the table is missing
        return "warning: kernel slot table not written: %s" % e


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    # the DoSample instances take longest: start them first
    srcs = sorted(sources(), key=lambda f: (not os.path.basename(f).startswith("vegas_sample_"), f))
    with cf.ThreadPoolExecutor(max_workers=1) as side:
        table = side.submit(_slot_table)  # its own assembly builds, alongside
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_compile, srcs))
        warn = table.result()
    if verbose:
        for (obj, msgs) in results:
            if msgs.strip():
                print(msgs)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if warn:
        print(warn, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
