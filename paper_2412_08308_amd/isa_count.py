"""VALU instructions per DP cell in the hot loops of the search kernels.

Compiles ``csrc/sw_isa_probe.hip`` (each hot-loop variant alone in a kernel,
same flags as the library), ``csrc/sw_pair.hip``, ``csrc/sw_pair_flow.hip``
and ``csrc/sw_k_rescore.hip`` to AMD assembly of this build, finds each
kernel's hot loop -- one trip sweeps four subject columns of R query rows,
i.e. 4*R cells per lane (8*R for the packed 16-bit variant, two subjects per
lane; 16 columns for the pair kernels) -- and counts its instructions by
class.  The VALU count per cell is the ISA operation count of the integer-VALU
roofline.
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
    # int32 rescore pass (csrc/sw_k_rescore.hip): 64 lanes x 24 rows, 16- / 8-bit profile
    # self-paired packed items (both halves of a lane on one subject's rows)
    "i16_self_lds": ("isa_i16_selfILi24ELi2ELb1E", 24, 2),
    "i16_self_glb": ("isa_i16_selfILi24ELi2ELb0E", 24, 2),
    "i16_p8_self_lds": ("isa_i16_selfILi24ELi1ELb1E", 24, 2),
    "i16_p8_self_glb": ("isa_i16_selfILi24ELi1ELb0E", 24, 2),
    "rescore_i32_r24": ("k_rescoreILi24ELi2E", 24, 1),
    "rescore_i32_r24_p8": ("k_rescoreILi24ELi1E", 24, 1),
    # probe of an 8-bit lane form (four subjects per lane, byte-wise saturating
    # arithmetic built from 32-bit operations; not part of the library)
    "i8x4_probe": ("isa_i8x4ILi16E", 16, 4),
    # single long pair (csrc/sw_pair.hip), score pass over skewed tiles: R rows
    # per lane, 8- / 16-bit profile; the loop of tiles inside the matrix
    "pair_r8_p8": ("k_pair_skewILi8ELi1E", 8, 1),
    "pair_r8_p16": ("k_pair_skewILi8ELi2E", 8, 1),
    "pair_r16_p8": ("k_pair_skewILi16ELi1E", 16, 1),
    "pair_r16_p16": ("k_pair_skewILi16ELi2E", 16, 1),
}
# pipelined pair pass (csrc/sw_pair_flow.hip): R rows per lane, 8- / 16-bit profile
for _R in (4, 6, 8, 10, 12, 16):
    for _ES in (1, 2):
        VARIANTS[f"flow_r{_R}_p{8 * _ES}"] = (f"k_pair_flowILi{_R}ELi{_ES}ELb0E", _R, 1)
_FLOW = [k for k in VARIANTS if k.startswith("flow_")]
# kernels with two copies of the hot loop (tiles at the matrix edge with a
# per-column predicate, tiles inside without): count the copy inside
INTERIOR = {"pair_r8_p8", "pair_r8_p16", "pair_r16_p8", "pair_r16_p16", *_FLOW}
# kernels whose first band has a copy of its own with no band above to read
# from: the loop counted is one that loads the row above (every other band's)
READS_ABOVE = set(_FLOW)
# subject columns one trip of the hot loop sweeps, where not four (the pair
# kernels unroll the 16 columns of a residue block)
TRIP_COLS = {"pair_r8_p8": 16, "pair_r8_p16": 16, "pair_r16_p8": 16, "pair_r16_p16": 16,
             **{k: 16 for k in _FLOW}}
SOURCES = ["sw_isa_probe.hip", "sw_pair.hip", "sw_pair_flow.hip", "sw_k_rescore.hip"]


def _hot_loop(lines, interior=False, reads_above=False):
    """Lines of the blocks of the hot loop: of the loops in the function, the
    one whose own blocks (its header block and every block the compiler
    annotates as directly inside it, wherever they are placed; not the blocks
    of loops nested in it) hold the most VALU instructions.  interior: of the
    loops holding at least 70% of that count, the one with the fewest.
    reads_above: of those, only the loops with the most vector-memory loads
    (the copy that reads the row above) count."""
    blocks = []            # (label, annotation, start, end)
    starts = [i for i, ln in enumerate(lines) if re.match(r"^\.LBB\w+:", ln)]
    for n, i in enumerate(starts):
        end = starts[n + 1] if n + 1 < len(starts) else len(lines)
        ann = [lines[i]]                     # the label line and the comment lines after it
        k = i + 1
        while k < end and lines[k].strip().startswith(";"):
            ann.append(lines[k])
            k += 1
        blocks.append((lines[i].split(":")[0], " ".join(ann), i, end))
    loops = []
    for hdr, ann, _, _ in blocks:
        m = re.search(r"Loop Header: Depth=(\d+)", ann)
        if not m:
            continue
        tag = "Header=" + hdr[2:] + " Depth=" + m.group(1)      # ".LBB1_2" -> "BB1_2"
        body = []
        for label, ann2, i, end in blocks:
            if label == hdr or tag in ann2:
                body.extend(lines[i:end])
        loops.append((sum(1 for l in body if l.strip().startswith("v_")), body))
    if not loops:
        return []
    top = max(v for v, _ in loops)
    if interior:
        cand = [lp for lp in loops if lp[0] >= 0.7 * top]
        if reads_above:
            loads = lambda lp: sum(1 for l in lp[1] if l.strip().startswith(("buffer_load", "global_load")))
            most = max(loads(lp) for lp in cand)
            cand = [lp for lp in cand if loads(lp) == most]
        return min(cand, key=lambda lp: lp[0])[1]
    return max(loops, key=lambda lp: lp[0])[1]


def count(asm_text: str) -> dict:
    funcs = re.split(r"^(?=_Z\S+:)", asm_text, flags=re.M)
    out = {}
    for key, (frag, rows, per) in VARIANTS.items():
        body = next((f for f in funcs if f.startswith("_Z") and frag in f.split(":")[0]), None)
        if body is None:
            continue
        loop = _hot_loop(body.split("\n"), key in INTERIOR, key in READS_ABOVE)
        ins = [l.strip().split()[0] for l in loop
               if l.strip() and not l.strip().startswith((".", ";")) and not l.strip().endswith(":")]
        c = collections.Counter(ins)
        cells = TRIP_COLS.get(key, 4) * rows * per
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
    res = {}
    with tempfile.TemporaryDirectory(prefix="swdb_isa_") as td:
        jobs = []
        for src in SOURCES:                 # the units compile in parallel
            asm = os.path.join(td, src + ".s")
            cmd = [HIPCC] + FLAGS + ["-x", "hip", "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", asm]
            jobs.append((src, asm, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                    text=True)))
        for src, asm, proc in jobs:
            log, _ = proc.communicate()
            if proc.returncode != 0:
                raise RuntimeError(f"{src} assembly failed:\n" + log)
            res.update(count(open(asm).read()))
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    return res


if __name__ == "__main__":
    json.dump(run(), sys.stdout, indent=1, sort_keys=True)
    print()
