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
UNITS = ["sw_k_i32p8.hip", "sw_k_i32p16.hip", "sw_k_i16.hip", "sw_k_i16p8.hip", "sw_k_rescore.hip", "sw_pair.hip"]


def _asm(unit, tmp_path):
    out = tmp_path / (unit + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-S", os.path.join(CSRC, unit), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def dpp_under_partial_exec(asm: str):
    """(kernel, line) of each DPP move whose nearest preceding change of the
    execution mask narrows it (a saveexec) or is a branch target, before any
    restore of the full mask."""
    found = []
    for name in re.findall(r"^(_ZN4swdb\w*):", asm, re.M):
        m = re.search(r"^" + re.escape(name) + r":.*?s_endpgm", asm, re.S | re.M)
        body = m.group(0).split("\n")
        for i, line in enumerate(body):
            if "_dpp" not in line:
                continue
            for k in range(i - 1, max(0, i - 80), -1):
                u = body[k].strip()
                if u.startswith(("s_or_b64 exec", "s_mov_b64 exec")):
                    break
                if u.startswith(".LBB") or "saveexec" in u:
                    found.append((name, line.strip()))
                    break
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
