"""The CPU suite again, with the host code of the library and the oracle
built under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed):
argument validation, database description and planning, workspace and
layout sizing, the pair planner, the status decoding, and the oracle's
recurrence and traceback.  Any sanitizer report fails the run."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# suites that drive native host code (the compile-only assembly checks and
# this file are left out)
SUITES = ["test_abi.py", "test_plan.py", "test_pair_plan.py", "test_oracle_pins.py", "test_oracle_align.py",
          "test_serve.py", "test_skew_schedule.py"]


@pytest.mark.skipif(not os.path.exists("/opt/rocm/llvm/bin/clang"), reason="clang not available")
def test_cpu_suite_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, HERE)
    import sanitize_build as sb
    lib = sb.build_library(str(tmp_path))
    orc = sb.build_oracle(str(tmp_path))
    env = dict(os.environ)
    env.update(LD_PRELOAD=sb.runtime(), SWDB_LIBRARY=lib, SWDB_ORACLE_LIBRARY=orc,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow", "-p", "no:cacheprovider"]
    cmd += [os.path.join(HERE, s) for s in SUITES]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
