"""Run the CPU test suite against the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer.

Builds ``oracle/liboracle_san.so`` (host code only: plain g++, nothing for the
GPU), then runs ``pytest -m "not gpu"`` in a child process with the ASan
runtime preloaded (the interpreter itself is not instrumented, so the runtime
has to come first in the process) and ``ORACLE_SANITIZE=1``, which makes the
oracle binding load the sanitized library.  Leak detection is off: the
interpreter's own allocations at exit are not the oracle's.  Any sanitizer
report aborts the run (``-fno-sanitize-recover=all``, ``halt_on_error``), so
the exit status is the outcome.

    python oracle/sanitize.py [extra pytest arguments]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def main(argv):
    sys.path.insert(0, HERE)
    import build as _build
    _build.build(sanitize=True)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], check=True,
                          capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-x",
           "-m", "not gpu", "-p", "no:cacheprovider"] + argv
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
