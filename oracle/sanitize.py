"""AddressSanitizer + UndefinedBehaviorSanitizer build of the C oracle, and a run of its CPU test
suite against that build.  Test infrastructure only (the oracle's own checker; no GPU, no product
code).  The build goes to oracle/_build_san; the suite runs in a child Python process with the
sanitizer runtime preloaded (Python itself is not instrumented, so leak detection is off) and
ORACLE_BUILD_DIR pointing there, and any sanitizer report aborts it.

    python -m oracle.sanitize      # build and run; exit status of the suite
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_DIR = os.path.join(HERE, "_build_san")
FLAGS = ("-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g")
# the oracle pins, minus the two reflection sweeps that take minutes unsanitized
SUITE = ["tests/test_oracle_core.py", "tests/test_oracle_nsbc.py", "tests/test_oracle_mrt.py",
         "tests/test_oracle_3d.py", "tests/test_oracle_mlp.py"]
DESELECT = "not gamma_sweep"


def runtime() -> str:
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("gcc has no AddressSanitizer runtime")
    return path


def build() -> str:
    import oracle
    oracle.build(extra_flags=FLAGS, build_dir=SAN_DIR)
    return SAN_DIR


def run_suite(timeout: float = 1200.0):
    """Run the oracle's CPU tests against the sanitizer build; returns (returncode, output)."""
    build()
    env = dict(os.environ)
    env.update({"LD_PRELOAD": runtime(), "ORACLE_BUILD_DIR": SAN_DIR,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "4"})
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", "-k", DESELECT, *SUITE]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


if __name__ == "__main__":
    rc, out = run_suite()
    print(out[-4000:])
    sys.exit(rc)
