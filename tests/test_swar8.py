"""The 8-bit lane form (four subjects per 32-bit lane) on gfx950, closed on
its instruction count (no GPU needed).

The paper names lower-precision integers as future work; the library takes
the step to packed 16-bit lanes.  The next step, four 8-bit cells per 32-bit
lane, needs byte-wise saturating add, subtract and maximum, which gfx950's
vector ALU lacks (it has them for packed 16-bit halves only).  The probe
kernel ``isa_i8x4`` builds them from 32-bit operations (``csrc/sw_swar8.h``)
and runs the cell update of the packed kernels on them; its hot loop, counted
like the library's, issues several times the packed 16-bit kernel's VALU
instructions per cell, so the 8-bit form would be slower and is not built.

These tests check the byte-wise helpers against scalar arithmetic (every pair
of byte values in every byte position, with random neighbouring bytes) and
pin the count comparison."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2412_08308_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CHECK = r"""
#include <cstdio>
#include <cstdlib>
#include "sw_swar8.h"
using namespace swdb;
static unsigned byte(unsigned w, int k) { return (w >> (8 * k)) & 0xffu; }
int main() {
    unsigned long long bad = 0, n = 0;
    unsigned x = 0x2545F491u;
    for (int pos = 0; pos < 4; ++pos)
        for (unsigned a = 0; a < 256; ++a)
            for (unsigned b = 0; b < 256; ++b) {
                x ^= x << 13; x ^= x >> 17; x ^= x << 5;
                unsigned y = x * 2654435761u;
                unsigned A = (x & ~(0xffu << (8 * pos))) | (a << (8 * pos));
                unsigned B = (y & ~(0xffu << (8 * pos))) | (b << (8 * pos));
                unsigned s = swar8_adds(A, B), d = swar8_subs(A, B), m = swar8_max(A, B);
                for (int k = 0; k < 4; ++k) {
                    unsigned ak = byte(A, k), bk = byte(B, k);
                    unsigned es = ak + bk > 255 ? 255 : ak + bk;
                    unsigned ed = ak > bk ? ak - bk : 0;
                    unsigned em = ak > bk ? ak : bk;
                    bad += (byte(s, k) != es) + (byte(d, k) != ed) + (byte(m, k) != em);
                    n += 3;
                }
            }
    printf("%llu %llu\n", bad, n);
    return bad != 0;
}
"""


@pytest.mark.skipif(not shutil.which("g++"), reason="g++ not available")
def test_swar8_helpers_match_bytewise_arithmetic(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECK)
    exe = tmp_path / "check"
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__host__=", "-D__device__=", "-D__forceinline__=inline",
                    "-I", CSRC, str(src), "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    bad, n = map(int, r.stdout.split())
    assert n == 4 * 256 * 256 * 4 * 3 and bad == 0, r.stdout


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_eight_bit_lanes_issue_more_per_cell(isa_counts):
    """Four 8-bit cells per lane cost more VALU instructions per cell than
    two 16-bit cells per lane, by a wide margin."""
    r = isa_counts
    i8, i16 = r["i8x4_probe"]["valu_per_cell"], r["i16_p8_lds_k1"]["valu_per_cell"]
    assert r["i8x4_probe"]["scratch"] == 0
    assert i8 > 3 * i16, (i8, i16)
