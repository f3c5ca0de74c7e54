"""VALU instructions per DP cell in the hot loops of the search kernels.

Compiles ``csrc/sw_isa_probe.hip`` (each hot-loop variant alone in a kernel,
same flags as the library) to AMD assembly of this build, finds each kernel's
innermost loop -- one trip sweeps four subject columns of R query rows, i.e.
4*R cells per lane (8*R for the packed 16-bit variant, two subjects per lane) --
and counts its instructions by class.  The VALU count per cell is the ISA
operation count of the integer-VALU roofline.
"""
from __future__ import annotations

import collections
import json
import os
import re
import subprocess
import sys
import tempfile

from .build import CSRC, FLAGS, HIPCC, HERE

OUT = os.path.join(HERE, "isa_counts.json")

# key -> (mangled-name fragment, rows, cells per lane-column)
VARIANTS = {
    "i32_p8_lds_k1": ("isa_i32ILi32ELi1ELb1ELb0E", 32, 1),
    "i32_p8_lds_kn": ("isa_i32ILi32ELi1ELb1ELb1E", 32, 1),
    "i32_p8_glb_k1": ("isa_i32ILi32ELi1ELb0ELb0E", 32, 1),
    "i32_p8_glb_kn": ("isa_i32ILi32ELi1ELb0ELb1E", 32, 1),
    "i32_p16_lds_k1": ("isa_i32ILi32ELi2ELb1ELb0E", 32, 1),
    "i32_p16_glb_k1": ("isa_i32ILi32ELi2ELb0ELb0E", 32, 1),
    "i16_lds_k1": ("isa_i16ILi24ELi2ELb1ELb0E", 24, 2),
    "i16_lds_kn": ("isa_i16ILi24ELi2ELb1ELb1E", 24, 2),
    "i16_glb_k1": ("isa_i16ILi24ELi2ELb0ELb0E", 24, 2),
    "i16_glb_kn": ("isa_i16ILi24ELi2ELb0ELb1E", 24, 2),
    "i16_p8_lds_k1": ("isa_i16ILi24ELi1ELb1ELb0E", 24, 2),
    "i16_p8_lds_kn": ("isa_i16ILi24ELi1ELb1ELb1E", 24, 2),
    "i16_p8_glb_k1": ("isa_i16ILi24ELi1ELb0ELb0E", 24, 2),
    "i16_p8_glb_kn": ("isa_i16ILi24ELi1ELb0ELb1E", 24, 2),
    "rescore_i32_r24": ("isa_i32ILi24ELi2ELb0ELb1E", 24, 1),
    "rescore_i32_r24_p8": ("isa_i32ILi24ELi1ELb0ELb1E", 24, 1),
}


def _innermost_loop(lines):
    """Lines of the deepest loop (by the compiler's loop-depth comments)."""
    best = None
    for i, ln in enumerate(lines):
        m = re.search(r"Loop Header: Depth=(\d+)", ln)
        if not m:
            continue
        depth = int(m.group(1))
        j = i
        while j > 0 and not lines[j].startswith(".LBB"):
            j -= 1
        label = lines[j].split(":")[0]
        ends = [k for k, l in enumerate(lines) if re.search(r"s_c?branch\w*\s+" + re.escape(label) + r"\s*$", l)]
        if not ends:
            continue
        if best is None or depth > best[0]:
            best = (depth, j, max(ends))
    if best is None:
        return []
    return lines[best[1]:best[2] + 1]


def count(asm_text: str) -> dict:
    funcs = re.split(r"^(?=_Z\S+:)", asm_text, flags=re.M)
    out = {}
    for key, (frag, rows, per) in VARIANTS.items():
        body = next((f for f in funcs if f.startswith("_Z") and frag in f.split(":")[0]), None)
        if body is None:
            continue
        loop = _innermost_loop(body.split("\n"))
        ins = [l.strip().split()[0] for l in loop
               if l.strip() and not l.strip().startswith((".", ";")) and not l.strip().endswith(":")]
        c = collections.Counter(ins)
        cells = 4 * rows * per
        valu = sum(v for k, v in c.items() if k.startswith("v_"))
        out[key] = {
            "valu_per_cell": round(valu / cells, 4),
            "valu": valu, "cells": cells,
            "lds": sum(v for k, v in c.items() if k.startswith("ds_")),
            "vmem": sum(v for k, v in c.items() if k.startswith(("global_", "buffer_"))),
            "scratch": sum(v for k, v in c.items() if k.startswith("scratch_")),
            "salu": sum(v for k, v in c.items() if k.startswith("s_")),
        }
    return out


def run(out: str = OUT) -> dict:
    with tempfile.TemporaryDirectory(prefix="swdb_isa_") as td:
        asm = os.path.join(td, "probe.s")
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "--cuda-device-only", "-S",
                                 os.path.join(CSRC, "sw_isa_probe.hip"), "-o", asm]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("isa probe compile failed:\n" + r.stdout + r.stderr)
        res = count(open(asm).read())
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    return res


if __name__ == "__main__":
    json.dump(run(), sys.stdout, indent=1, sort_keys=True)
    print()
