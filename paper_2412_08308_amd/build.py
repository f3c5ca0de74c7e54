"""Build the gfx950 library ``libswdb.so`` in-tree with hipcc.

Each kernel variant lives in its own translation unit; they are compiled in
parallel and linked into one shared library.  Every kernel is compiled for
gfx950 only.  Packed-fp32 instruction selection is disabled
(``-packed-fp32-ops``); the path has no floating point, the flag only keeps the
compiler away from those instruction forms.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswdb.so")
SOURCES = ["sw_k_i32p8.hip", "sw_k_i32p16.hip", "sw_k_i16.hip", "sw_k_i16p8.hip", "sw_k_rescore.hip", "sw_k_prep.hip", "sw_pair.hip",
           "sw_pair_flow.hip", "sw_runtime.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def build(out: str = LIB, extra=None, quiet: bool = True, jobs: int = 0, link_extra=None) -> str:
    """Compile every translation unit (in parallel) and link ``out``;
    ``extra`` / ``link_extra``: more compile / link flags."""
    extra = list(extra or [])
    link_extra = list(link_extra or [])
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="swdb_build_") as td:
        objs, procs, logs = [], [], []
        pending = list(SOURCES)
        while pending or procs:
            while pending and len(procs) < jobs:
                src = pending.pop(0)
                obj = os.path.join(td, os.path.basename(src) + ".o")
                cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
                procs.append((src, cmd, _run(cmd)))
                objs.append(obj)
            src, cmd, p = procs.pop(0)
            text, _ = p.communicate()
            if p.returncode != 0:
                for _, _, q in procs:
                    q.kill()
                raise RuntimeError(f"hipcc failed on {src}:\n" + " ".join(cmd) + "\n" + text)
            logs.append(text)
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + link_extra + objs + ["-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    if not quiet:
        sys.stderr.write("".join(logs))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
