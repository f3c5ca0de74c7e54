"""Checks on the gfx950 assembly of this build's own kernels (no GPU needed):
every DPP lane shift executes with the whole wave active.  A shift reads
another lane's register; the compiler may fold it into a select and run it
under a partial execution mask, where it would read lanes that did not take
part and return stale values (this happened once in the pair kernel)."""
import os
import re
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2412_08308_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
UNITS = ["sw_k_i32p8.hip", "sw_k_i32p16.hip", "sw_k_i16.hip", "sw_k_i16p8.hip", "sw_k_rescore.hip", "sw_pair.hip",
         "sw_pair_flow.hip"]


def _asm(unit, tmp_path):
    out = tmp_path / (unit + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-S", os.path.join(CSRC, unit), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


_BRANCH = re.compile(r"\s*s_(c)?branch\w*\s+(\.LBB\w+)\s*$")


def _full_mask_lines(body):
    """For every line of a kernel body, whether every path reaching it
    arrives with the whole wave active, judged from the nearest change of the
    execution mask before it on each path: a restore (s_or_b64 / s_mov_b64
    exec) or the kernel's entry counts as full, a saveexec as narrowed.  At a
    label the paths are its fall-through (unless the line before ends the
    flow) and every branch to it.  Solved as a greatest fixed point over the
    labels (all start full; a label becomes narrowed once some path into it
    arrives narrowed), so loops are decided by the paths into them."""
    block = []                      # label (or None: the entry) of each line
    local = []                      # the mask set in the line's block up to and including it, or None
    label, cur = None, None
    labels = {}
    for k, ln in enumerate(body):
        u = ln.strip()
        if u.startswith(".LBB") and u.split()[0].endswith(":"):
            label, cur = u.split(":")[0], None
            labels[label] = k
        block.append(label)
        if u.startswith(("s_or_b64 exec", "s_mov_b64 exec")):
            cur = True
        elif "saveexec" in u:
            cur = False
        local.append(cur)
    entry = {L: True for L in labels}

    def after(j):                       # the state just after line j
        if local[j] is not None:
            return local[j]
        return True if block[j] is None else entry[block[j]]

    def before(i):                      # the state just before line i
        if block[i] is not None and labels[block[i]] == i:
            return entry[block[i]]
        return True if i == 0 else after(i - 1)

    preds = {L: [] for L in labels}     # states flowing into each label
    for n, ln in enumerate(body):
        m = _BRANCH.match(ln)
        if m and m.group(2) in preds:
            preds[m.group(2)].append(lambda n=n: before(n))
    for L, k in labels.items():
        prev = next((q for q in range(k - 1, -1, -1)
                     if body[q].strip() and not body[q].strip().startswith(";")), None)
        if prev is not None and not body[prev].strip().startswith(("s_branch", "s_endpgm", "s_setpc")):
            preds[L].append(lambda k=k: after(k - 1))        # fall-through
    changed = True
    while changed:
        changed = False
        for L in labels:
            if entry[L] and not all(f() for f in preds[L]):
                entry[L] = False
                changed = True
    return [before(i) for i in range(len(body))]


def dpp_under_partial_exec(asm: str):
    """(kernel, line) of each DPP move that some path reaches with part of the
    wave masked off (see _full_mask_lines)."""
    found = []
    for name in re.findall(r"^(_ZN4swdb\w*):", asm, re.M):
        m = re.search(r"^" + re.escape(name) + r":.*?s_endpgm", asm, re.S | re.M)
        body = m.group(0).split("\n")
        full = _full_mask_lines(body)
        for i, line in enumerate(body):
            if "_dpp" in line and not full[i]:
                found.append((name, line.strip()))
    return found


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("unit", UNITS)
def test_dpp_shifts_run_with_full_wave(unit, tmp_path):
    asm = _asm(unit, tmp_path)
    assert "_dpp" in asm
    assert dpp_under_partial_exec(asm) == []


def test_scanner_flags_a_shift_in_a_branch():
    """The scanner itself: a shift after a saveexec (a partial mask) is reported."""
    asm = "\n".join(["_ZN4swdb1kEv:", "s_and_saveexec_b64 s[4:5], s[2:3]", "s_cbranch_execnz .LBB1_43",
                     ".LBB1_43:", "v_mov_b32_dpp v59, v59 wave_shr:1 row_mask:0xf bank_mask:0xf",
                     "s_or_b64 exec, exec, s[4:5]", "v_mov_b32_dpp v1, v1 wave_shr:1", "s_endpgm"])
    assert len(dpp_under_partial_exec(asm)) == 1


def test_dpp_check_follows_paths():
    """The checker flags a shift after a narrowing saveexec and a shift at a
    label that some branch reaches with a narrowed mask, and passes a loop
    header whose back edge restores the mask first."""
    narrowed = ("_ZN4swdb1aEv:\n s_and_saveexec_b64 s[0:1], vcc\n v_mov_b32_dpp v1, v1 wave_shr:1\n"
                " s_or_b64 exec, exec, s[0:1]\n s_endpgm\n")
    assert len(dpp_under_partial_exec(narrowed)) == 1
    loop_ok = ("_ZN4swdb1bEv:\n v_mov_b32 v1, 0\n.LBB0_1:\n v_mov_b32_dpp v1, v1 wave_shr:1\n"
               " s_and_saveexec_b64 s[0:1], vcc\n v_add_u32 v2, v1, v2\n s_or_b64 exec, exec, s[0:1]\n"
               " s_cbranch_scc1 .LBB0_1\n s_endpgm\n")
    assert dpp_under_partial_exec(loop_ok) == []
    loop_bad = ("_ZN4swdb1cEv:\n v_mov_b32 v1, 0\n.LBB0_1:\n v_mov_b32_dpp v1, v1 wave_shr:1\n"
                " s_and_saveexec_b64 s[0:1], vcc\n v_add_u32 v2, v1, v2\n s_cbranch_scc1 .LBB0_1\n"
                " s_or_b64 exec, exec, s[0:1]\n s_endpgm\n")
    assert len(dpp_under_partial_exec(loop_bad)) == 1


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_hot_loop_counts_are_sane(isa_counts):
    """The roofline's VALU-per-cell figures come from isa_count.py's choice of
    hot loop; a change in the kernels' loop structure must not make it count a
    fragment or the wrong copy (the ranges bracket the counted loops), and the
    counted loops of the default variants keep their state in registers."""
    r = isa_counts
    # the pair kernel's edge copy of its loop counts about 1 VALU per cell more
    # than the copy inside the matrix: the pair bounds exclude it
    bounds = {"i16_p8_lds_k1": (5.2, 6.2), "i16_p8_lds_kn": (5.2, 6.5), "i32_p8_lds_k1": (7.6, 8.8),
              "pair_r8_p8": (9.3, 10.3), "pair_r16_p8": (8.5, 9.4), "rescore_i32_r24_p8": (8.3, 9.5)}
    for key, (lo, hi) in bounds.items():
        assert lo <= r[key]["valu_per_cell"] <= hi, (key, r[key])
        assert r[key]["scratch"] == 0, (key, r[key])
