"""Compile the CPU oracle (plain C, gcc) into ``oracle/liboracle.so``.

Test infrastructure: see ``oracle/__init__.py``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sw_oracle.c")
LIB = os.environ.get("SWDB_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")


def build(out: str = LIB, mutant: int = 0, quiet: bool = True, cc: str = "gcc", extra=()) -> str:
    """Build the oracle library; ``mutant`` > 0 plants one test-only mistake;
    ``cc`` / ``extra``: another C compiler and more flags."""
    tmp = out + ".tmp"
    cmd = [cc, "-std=c11", "-O2", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", f"-DORACLE_MUTANT={int(mutant)}"] + list(extra) + [SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + r.stdout + r.stderr)
    if not quiet and (r.stdout or r.stderr):
        sys.stderr.write(r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
