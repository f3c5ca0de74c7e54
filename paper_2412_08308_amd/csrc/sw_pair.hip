// Intra-task alignment of one long pair: every lane of the device works on
// cells of a single matrix (paper Section 2.2 / Fig. 1, intra-task scheme; the
// paper's pairwise workload aligns DNA sequences of 162K to 7M residues,
// Section 4.1).
//
// The matrix is cut into tiles of K*R query rows (a band: K pipelined lanes of
// R rows each, as in the database search) by wc subject columns (a chunk).
// Tile (b, c) depends on (b-1, c), (b, c-1) and (b-1, c-1) only, so all tiles
// of one anti-diagonal b + c = d are independent; the host launches the
// diagonals in order on one stream.  No wave ever waits for another workgroup.
// Boundaries travel between launches through in-place buffers (PairArgs).
//
// Each lane group runs one tile.  Lanes start from their rows of the chunk's
// left boundary and keep H - Go and E in registers across the chunk; lane g
// works on column step - g only while that is a column of the chunk (the
// pipeline fill steps leave its state alone), the group head reads the band's
// top boundary from rowbuf, the tail writes the band's bottom row back into it,
// and after the sweep every lane writes its rows of the chunk's last column
// into colbuf.  These rectangular tiles serve the passes that write direction
// codes or checkpoints, whose layouts follow rows and columns; the plain score
// pass runs skewed tiles without the pipeline fill (pair_skew_tile).
#include <type_traits>

#include "sw_device.h"

namespace swdb {

// TRACE (8 rows per lane only): also write each cell's 4-bit direction code
// (PairArgs::dir) and find the first cell, in column-major order, whose H
// equals the score already computed by a plain pass (PairArgs::end_key).  The
// codes follow the traceback rules: the diagonal before E before F, a gap
// opened from H rather than extended when both give its value.
// CKPT (score pass of a checkpointed alignment): also store the checkpoint
// rows and columns and the chunk maxima (PairArgs).
template <int R, int ES, bool TRACE = false, bool CKPT = false>
__device__ __forceinline__ void pair_tile(const PairArgs& a, int lane)
{
    static_assert(!TRACE || R == 8, "direction words hold 8 rows");
    static_assert(!(TRACE && CKPT), "checkpoints come from the score pass");
    constexpr uint32_t CS = code_stride(R, ES);
    constexpr uint32_t BS = kCodes * CS;
    constexpr int NB = R * ES;
    constexpr int NV = (NB + 15) / 16;

    const int K = a.K;
    const int nsubw = kWave / K;
    const int sub = lane / K;
    const int g = lane - sub * K;
    const bool inb = sub < nsubw;
    const int tile = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * nsubw) + (inb ? sub : 0);
    const bool valid = inb && tile < a.ntiles;
    const int b = a.b_lo + (valid ? tile : 0);
    const int c = a.d - b;
    const bool head = g == 0;
    const bool tail = g == K - 1;
    const int wc = a.wc;
    const int64_t c0 = (int64_t)c * wc;
    const int rb = b * K + g;
    const int64_t row0 = (int64_t)rb * R;
    const uint32_t pbase = (uint32_t)min(rb, a.nbr) * BS;
    const int go = a.go, ge = a.ge;
    const bool has_top = valid && b > 0;
    const bool has_left = valid && c > 0;
    const bool put_bottom = valid && tail && b < a.nb - 1;
    const bool put_right = valid && c < a.nc - 1;
    int2* __restrict__ top = a.rowbuf + c0;
    int2* __restrict__ side = a.colbuf + row0;
    // checkpoint row below this band / column right of this chunk (CKPT)
    int2* __restrict__ ck_bottom = nullptr;
    int2* __restrict__ ck_right = nullptr;
    if constexpr (CKPT) {
        if (put_bottom && (b + 1) % a.ckpt_gb == 0)
            ck_bottom = a.ckpt_row + (int64_t)((b + 1) / a.ckpt_gb - 1) * a.ckpt_row_stride + c0;
        if (put_right && (c + 1) % a.ckpt_gc == 0)
            ck_right = a.ckpt_col + (int64_t)((c + 1) / a.ckpt_gc - 1) * a.ckpt_col_stride + row0;
    }
    const uint4* __restrict__ resp = reinterpret_cast<const uint4*>(a.subj + c0);

    int Y[R], E[R];
    if (has_left) {
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            const int4 v = *reinterpret_cast<const int4*>(side + r);
            Y[r] = v.x; E[r] = v.y; Y[r + 1] = v.z; E[r + 1] = v.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) { Y[r] = -go; E[r] = 0; }
    }
    // H - Go of the cell above-left of this lane's first row: the previous
    // lane's last row in the chunk to the left, or the corner for the head
    int ydiag = -go;
    if (has_left) {
        if (!head)
            ydiag = side[-1].x;
        else if (b > 0)
            ydiag = (TRACE && b == a.b_org && a.top_ckpt) ? a.top_ckpt[c0 - 1].x : a.corner[b * 3 + c % 3];
    }
    int ybot = -go, fbot = 0;
    int S = 0;
    const int s_target = TRACE ? *a.score : 0;
    unsigned long long key = ~0ull;          // first cell holding s_target (TRACE)
    // direction word of this lane's row block at column c0 + j: dir[doff + j * stride]
    const int64_t doff = (c0 - a.dir_col0) * a.dir_stride + (rb - a.dir_rb0);

    // Lane g works on column step - g.  Its code for the next step is the code
    // lane g - 1 holds now (the head reads it from the residue stream), so the
    // profile entries of the next column are loaded one step ahead, outside the
    // per-lane column predicate, and their latency overlaps this column's cells.
    const int nsteps = (wc + K - 1 + 3) & ~3;
    uint4 rv = head ? resp[0] : pad16();
    int code = head ? (int)(rv.x & 0xffu) : kPad;
    uint4 pv[NV];
    ldprof<NB, false>(pv, a.prof, pbase + (uint32_t)code * CS);
    for (int blk = 0; blk < nsteps; blk += 16) {
        const uint4 rvn = head ? resp[(blk + 16) >> 4] : pad16();
        const int n4 = min(4, (nsteps - blk) >> 2);
#pragma unroll 1
        for (int k4 = 0; k4 < n4; ++k4) {
            const int col0 = blk + 4 * k4;
            const uint32_t w = rv.x;                      // residues col0 .. col0 + 3
            const uint32_t wn = k4 == 3 ? rvn.x : rv.y;   // col0 + 4 .. col0 + 7
            rv = make_uint4(rv.y, rv.z, rv.w, 0u);
            int ringY[4], ringF[4];
            if (has_top && head && col0 < wc) {
                const int4* p4 = reinterpret_cast<const int4*>(top + col0);
                const int4 v0 = p4[0], v1 = p4[1];
                ringY[0] = v0.x; ringF[0] = v0.y; ringY[1] = v0.z; ringF[1] = v0.w;
                ringY[2] = v1.x; ringF[2] = v1.y; ringY[3] = v1.z; ringF[3] = v1.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) { ringY[k] = -go; ringF[k] = 0; }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                // shifts and loads run with every lane active (a shift reads
                // other lanes' registers); the column body only for this lane's
                // own columns 0..wc-1, so its state stays that of its last column
                // (pinned: a shift folded into the head/non-head select would be
                // executed by the non-head lanes alone and read stale values)
                int cd = shr1(code), yd = shr1(ybot), fd = shr1(fbot);
                pin(cd);
                pin(yd);
                pin(fd);
                const uint32_t wsrc = u < 3 ? w : wn;
                const int shift = u < 3 ? 8 * (u + 1) : 0;
                const int cnext = head ? (int)((wsrc >> shift) & 0xffu) : cd;
                uint4 pvn[NV];
                ldprof<NB, false>(pvn, a.prof, pbase + (uint32_t)cnext * CS);
                const int j = col0 + u - g;               // this lane's column
                if ((unsigned)j < (unsigned)wc) {
                    const int yt = head ? ringY[u] : yd;
                    const int ft = head ? ringF[u] : fd;
                    int dg = ydiag;
                    ydiag = yt;
                    int hup = yt, F = ft;
                    int hprev = 0;
                    uint32_t word = 0;
                    int hs[TRACE ? R : 1];                // the column's H (trace)
                    int cmax = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int t = dg + pent<ES>(pv, r);
                        const int eo = E[r] - ge;
                        const int e = imax3(eo, Y[r], 0);
                        const int fo = F - ge;
                        F = max(fo, hup);
                        const int h = imax3(t, e, F);
                        if constexpr (TRACE) {
                            uint32_t code = h == 0 ? 0u : (h == t ? 1u : (h == e ? 2u : 3u));
                            code |= (Y[r] >= eo ? 4u : 0u) | (hup >= fo ? 8u : 0u);
                            word |= code << (4 * r);
                            hs[r] = h;
                            if (r & 1)
                                cmax = imax3(cmax, hprev, h);
                            else
                                hprev = h;
                        } else if (r & 1) {
                            S = imax3(S, hprev, h);
                            pin(S);
                        } else {
                            hprev = h;
                        }
                        dg = Y[r];
                        hup = h - go;
                        Y[r] = hup;
                        E[r] = e;
                    }
                    ybot = hup;
                    fbot = F;
                    if (put_bottom)
                        top[j] = make_int2(ybot, fbot);
                    if constexpr (CKPT) {
                        if (ck_bottom)
                            ck_bottom[j] = make_int2(ybot, fbot);
                    }
                    if constexpr (TRACE) {
                        const int64_t col = c0 + j;
                        if (valid) {
                            if (a.dir)
                                a.dir[doff + (int64_t)j * a.dir_stride] = word;
                            // no H exceeds the pair's score: only a column whose
                            // maximum is the score holds the end cell
                            if (cmax == s_target) {
                                uint32_t hits = 0;
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    hits |= (hs[r] == s_target ? 1u : 0u) << r;
                                const int64_t row = row0 + __builtin_ctz(hits);
                                if (key == ~0ull && col < a.n && row < a.m)
                                    key = ((unsigned long long)col << 32) | (unsigned long long)row;
                            }
                        }
                    }
                }
                code = cnext;
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    pv[i] = pvn[i];
            }
        }
        rv = rvn;
    }
    // right boundary: every lane's rows at the chunk's last column; the tail's
    // bottom cell there is the corner of the tile down-right
    if (put_right) {
#pragma unroll
        for (int r = 0; r < R; r += 2)
            *reinterpret_cast<int4*>(side + r) = make_int4(Y[r], E[r], Y[r + 1], E[r + 1]);
        if (put_bottom)
            a.corner[(b + 1) * 3 + (c + 1) % 3] = ybot;
        if constexpr (CKPT) {
            if (ck_right) {
#pragma unroll
                for (int r = 0; r < R; r += 2)
                    *reinterpret_cast<int4*>(ck_right + r) = make_int4(Y[r], E[r], Y[r + 1], E[r + 1]);
            }
        }
    }
    if constexpr (TRACE) {
        // first hit of the wave (column, then row), into the pair's end key
        for (int k = 32; k >= 1; k >>= 1) {
            const unsigned long long o = __shfl_xor(key, k);
            key = o < key ? o : key;
        }
        if (lane == 0 && key != ~0ull)
            atomicMin(a.end_key, key);
        return;
    }
    // tile maximum into the pair's score (and its chunk's maximum)
    S = valid ? S : 0;
    for (int k = 32; k >= 1; k >>= 1)
        S = max(S, __shfl_xor(S, k));
    if (lane == 0 && S > 0) {
        atomicMax(a.score, S);
        if constexpr (CKPT)
            atomicMax(a.chunk_max + c, S);
    }
}

// Score pass over skewed tiles.  Lane g of band b covers, in chunk c, the
// columns [c*wc - b*kr - g, +wc) (kr = K rounded up to 16): a lane's row block
// starts one column after the row block above it, as the DPP pipeline needs,
// so every lane has a column on every step -- a tile has no pipeline fill or
// drain -- and the head's first column is a multiple of 16.  Only columns in
// [0, n) are computed.  Tile (b, c) reads the band above's bottom row from
// rowbuf (written by tiles (b-1, c' <= c)), and its own lanes' state at the
// end of tile (b, c-1): colbuf (H - Go and E per row) and carry (per row
// block: H - Go and F of the bottom row at the lane's last column, which the
// lane below takes on its first step, and the H - Go of the cell above the
// lane's last column, its diagonal for the next column).  With kr >= K no two
// tiles of one anti-diagonal touch the same rowbuf entry, and every entry a
// tile reads is written on an earlier anti-diagonal and overwritten only on a
// later one (tests/test_skew_schedule.py steps through this schedule on the
// CPU, checks each launch's reads against the same launch's writes, and
// compares the scores with the oracle).
//
// TRACE (8 rows per lane, whole-matrix direction codes): also write each
// cell's direction code into dir and find the first cell, in column-major
// order, holding the score of the plain pass, as the rectangular tiles do;
// lanes of no tile write their words into their wave's sink slot, so that the
// store needs no branch either.
template <int R, int ES, bool TRACE = false>
__device__ __forceinline__ void pair_skew_tile(const PairArgs& a, int lane)
{
    static_assert(!TRACE || R == 8, "direction words hold 8 rows");
    constexpr uint32_t CS = code_stride(R, ES);
    constexpr uint32_t BS = kCodes * CS;
    constexpr int NB = R * ES;
    constexpr int NV = (NB + 15) / 16;

    const int K = a.K;
    const int nsubw = kWave / K;
    const int sub = lane / K;
    const int g = lane - sub * K;
    const bool inb = sub < nsubw;
    const int tile = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * nsubw) + (inb ? sub : 0);
    const bool valid = inb && tile < a.ntiles;
    const int b = a.b_lo + (valid ? tile : 0);
    const int c = a.d - b;
    const bool head = g == 0;
    const int wc = a.wc;
    const int n = (int)a.n;                                    // lengths are below 2^24
    const int jh = c * wc - b * a.kr;                          // the head's first column
    const int j0 = jh - g;                                     // this lane's first column
    const int rb = b * K + g;
    const int64_t row0 = (int64_t)rb * R;
    const uint32_t pbase = (uint32_t)min(rb, a.nbr) * BS;
    const int go = a.go, ge = a.ge;
    const bool has_top = valid && b > 0;
    const bool put_bottom = valid && g == K - 1 && b < a.nb - 1;
    // this lane computed column j0 - 1 in tile (b, c - 1)
    const bool has_left = valid && j0 >= 1 && j0 <= n;
    int2* __restrict__ top = a.rowbuf;
    int2* __restrict__ side = a.colbuf + row0;
    const uint4* __restrict__ resp = reinterpret_cast<const uint4*>(a.subj);
    const int nblk = (int)(a.n_pad >> 4);

    int Y[R], E[R];
    int ybot = -go, fbot = 0, ydiag = -go;
    if (has_left) {
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            const int4 v = *reinterpret_cast<const int4*>(side + r);
            Y[r] = v.x; E[r] = v.y; Y[r + 1] = v.z; E[r + 1] = v.w;
        }
        const int4 cv = a.carry[rb];
        ybot = cv.x; fbot = cv.y; ydiag = cv.z;
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) { Y[r] = -go; E[r] = 0; }
    }
    int S = 0;
    const int s_target = TRACE ? *a.score : 0;
    unsigned long long key = ~0ull;          // first cell holding s_target (TRACE)
    uint32_t* const dsink =
        reinterpret_cast<uint32_t*>(a.sink + (int64_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64);
    // direction word of this lane's row block at column j: dir[doff + j * stride]
    const int64_t doff = (int64_t)(rb - a.dir_rb0) - a.dir_col0 * a.dir_stride;

    // every lane of the wave inside [0, n) on every step: no per-column predicate
    const bool inner = !valid || (j0 >= 0 && j0 + wc <= n);
    // 16 codes from column col (a multiple of 16), read by every lane of the
    // group at its head's column (one address per group), the index clamped
    // into the buffer; blocks outside it hold no column that is computed
    auto block_at = [&](int col) { return resp[min(max(col >> 4, 0), nblk - 1)]; };

    // The last lane's bottom row goes to rowbuf through a buffer store that
    // every lane issues: the others aim past the buffer's range (n entries),
    // where the hardware drops the store, at an offset that still lies in the
    // workspace's spare rowbuf columns.  Without a branch around the store the
    // compiler's count of outstanding memory operations is exact, so the wait
    // for a profile load no longer includes the store issued just before it.
    typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
    const __amdgpu_buffer_rsrc_t rows_out = __builtin_amdgcn_make_buffer_rsrc(top, (short)0, n * 8, 0x00020000);
    const int sink = (n + 64) * 8;
    // the band above's bottom row for the head, 4 columns per load pair, read
    // by every lane of the group at the head's (clamped) column one group of 4
    // steps ahead, so that no wait depends on a load just issued
    auto ring_load = [&](int col, int4& v0, int4& v1) {
        const int4* p4 = reinterpret_cast<const int4*>(top + max(col, 0));
        v0 = p4[0];
        v1 = p4[1];
    };

    const int tmask = has_top ? -1 : 0;

    auto sweep = [&](auto edge) {
        constexpr bool EDGE = decltype(edge)::value;
        int4 rn0, rn1;
        ring_load(jh, rn0, rn1);
        uint4 rv = block_at(jh);
        int code = head ? (int)(rv.x & 0xffu) : ((valid && j0 >= 0 && j0 < n) ? (int)a.subj[j0] : kPad);
        uint4 pv[NV];
        ldprof<NB, false>(pv, a.prof, pbase + (uint32_t)code * CS);
        for (int blk = 0; blk < wc; blk += 16) {
            const uint4 rvn = block_at(jh + blk + 16);
            // the 16 steps of a residue block unrolled, so that every wait
            // counts exactly the loads and stores issued after the one it needs
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const int col0 = blk + 4 * k4;
                const uint32_t w = rv.x;                      // codes of columns col0 .. col0 + 3
                const uint32_t wn = k4 == 3 ? rvn.x : rv.y;   // col0 + 4 .. col0 + 7
                rv = make_uint4(rv.y, rv.z, rv.w, 0u);
                // (H - Go, F) of the band above, or the matrix's top border
                int ringY[4], ringF[4];
                ringY[0] = (rn0.x & tmask) | (-go & ~tmask); ringF[0] = rn0.y & tmask;
                ringY[1] = (rn0.z & tmask) | (-go & ~tmask); ringF[1] = rn0.w & tmask;
                ringY[2] = (rn1.x & tmask) | (-go & ~tmask); ringF[2] = rn1.y & tmask;
                ringY[3] = (rn1.z & tmask) | (-go & ~tmask); ringF[3] = rn1.w & tmask;
                ring_load(jh + col0 + 4, rn0, rn1);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // shifts with the whole wave active; the values are pinned so
                    // that no shift is folded into a select under a partial mask
                    int cd = shr1(code), yd = shr1(ybot), fd = shr1(fbot);
                    pin(cd);
                    pin(yd);
                    pin(fd);
                    const uint32_t wsrc = u < 3 ? w : wn;
                    const int shift = u < 3 ? 8 * (u + 1) : 0;
                    const int cnext = head ? (int)((wsrc >> shift) & 0xffu) : cd;
                    uint4 pvn[NV];
                    ldprof<NB, false>(pvn, a.prof, pbase + (uint32_t)cnext * CS);
                    const int j = j0 + col0 + u;              // this lane's column
                    if (!EDGE || (j >= 0 && j < n)) {
                        const int yt = head ? ringY[u] : yd;
                        const int ft = head ? ringF[u] : fd;
                        int dg = ydiag;
                        ydiag = yt;
                        int hup = yt, F = ft;
                        int hprev = 0;
                        uint32_t word = 0;
                        int hs[TRACE ? R : 1];            // the column's H (trace)
                        int cmax = 0;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int t = dg + pent<ES>(pv, r);
                            const int eo = E[r] - ge;
                            const int e = imax3(eo, Y[r], 0);
                            const int fo = F - ge;
                            F = max(fo, hup);
                            const int h = imax3(t, e, F);
                            if constexpr (TRACE) {
                                uint32_t cc = h == 0 ? 0u : (h == t ? 1u : (h == e ? 2u : 3u));
                                cc |= (Y[r] >= eo ? 4u : 0u) | (hup >= fo ? 8u : 0u);
                                word |= cc << (4 * r);
                                hs[r] = h;
                                if (r & 1)
                                    cmax = imax3(cmax, hprev, h);
                                else
                                    hprev = h;
                            } else if (r & 1) {
                                S = imax3(S, hprev, h);
                                pin(S);
                            } else {
                                hprev = h;
                            }
                            dg = Y[r];
                            hup = h - go;
                            Y[r] = hup;
                            E[r] = e;
                        }
                        ybot = hup;
                        fbot = F;
                        const u32x2 v = {(unsigned)ybot, (unsigned)fbot};
                        __builtin_amdgcn_raw_buffer_store_b64(v, rows_out, put_bottom ? j * 8 : sink, 0, 0);
                        if constexpr (TRACE) {
                            *((valid && a.dir) ? a.dir + (doff + (int64_t)j * a.dir_stride) : dsink) = word;
                            // no H exceeds the pair's score: only a column whose
                            // maximum is the score holds the end cell
                            if (cmax == s_target) {
                                uint32_t hits = 0;
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    hits |= (hs[r] == s_target ? 1u : 0u) << r;
                                const int64_t row = row0 + __builtin_ctz(hits);
                                if (valid && key == ~0ull && row < a.m)
                                    key = ((unsigned long long)j << 32) | (unsigned long long)row;
                            }
                        }
                    }
                    code = cnext;
#pragma unroll
                    for (int i = 0; i < NV; ++i)
                        pv[i] = pvn[i];
                }
            }
            rv = rvn;
        }
    };
    if (__all(inner))
        sweep(std::integral_constant<bool, false>{});
    else
        sweep(std::integral_constant<bool, true>{});

    // state after this lane's last column, for tile (b, c + 1)
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; r += 2)
            *reinterpret_cast<int4*>(side + r) = make_int4(Y[r], E[r], Y[r + 1], E[r + 1]);
        a.carry[rb] = make_int4(ybot, fbot, ydiag, 0);
    }
    if constexpr (TRACE) {
        for (int k = 32; k >= 1; k >>= 1) {
            const unsigned long long o = __shfl_xor(key, k);
            key = o < key ? o : key;
        }
        if (lane == 0 && key != ~0ull)
            atomicMin(a.end_key, key);
        return;
    }
    S = valid ? S : 0;
    for (int k = 32; k >= 1; k >>= 1)
        S = max(S, __shfl_xor(S, k));
    if (lane == 0 && S > 0)
        atomicMax(a.score, S);
}

// 16-row lanes keep their state in up to 168 registers (three waves per SIMD,
// more than long pairs put on one); 8-row lanes fit four
template <int R, int ES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(R == 8 ? 4 : 3))) k_pair_skew(PairArgs a)
{
    pair_skew_tile<R, ES>(a, threadIdx.x & 63);
}

// the direction codes and the end-cell search take about 175 registers
template <int ES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_trace_skew(PairArgs a)
{
    pair_skew_tile<8, ES, true>(a, threadIdx.x & 63);
}

template <int ES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_pair_diag_ckpt(PairArgs a)
{
    pair_tile<8, ES, false, true>(a, threadIdx.x & 63);
}

template <int ES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_trace_diag(PairArgs a)
{
    pair_tile<8, ES, true>(a, threadIdx.x & 63);
}

__global__ void k_trace_reset(unsigned long long* end_key)
{
    if (threadIdx.x == 0)
        *end_key = ~0ull;
}

// Walk of the traceback: from the end cell in state H, follow the direction
// codes -- the diagonal emits a residue pair, E a subject residue against a
// gap, F a query residue against a gap, each gap returning to H where it was
// opened -- until a diagonal step reaches a cell holding H = 0 (the alignment
// began at the cell before it) or the border; then reverse the operations
// into begin-to-end order.  The codes may come one block of the matrix at a
// time: the walk stops when it leaves the block in hand, keeping its state in
// a WalkState, and the host supplies the block holding the next cell.
//
// One wavefront per walk call: the codes of a window of 64 columns x 128 rows
// around the walk sit in LDS (each lane loads one column), and the wave
// reloads the window when the walk leaves it.  The walk's state is uniform;
// each pass takes the run of steps that continue in one direction (lane l
// reads the l-th cell along it, a ballot finds where the run ends) and its
// lanes write the run's operations.
constexpr int kWinCols = 64, kWinWords = 16;   // 16 words of 8 rows = 128 rows

__global__ void k_walk_init(const unsigned long long* __restrict__ end_key, const int32_t* __restrict__ score,
                            WalkState* w)
{
    if (threadIdx.x != 0)
        return;
    const unsigned long long key = *end_key;
    WalkState s{};
    s.ok = 1;
    if (*score > 0 && key != ~0ull) {
        s.j = (int64_t)(key >> 32) + 1;            // 1-based
        s.i = (int64_t)(key & 0xffffffffull) + 1;
        s.q_end = (int32_t)s.i;
        s.s_end = (int32_t)s.j;
    } else {
        s.done = 1;                                // empty alignment
    }
    *w = s;
}

__device__ __forceinline__ int walk_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ void __launch_bounds__(64) k_walk(const uint32_t* __restrict__ dir, int64_t stride, int64_t r_lo,
                                             int64_t c_lo, int64_t r_hi, int64_t c_hi, WalkState* wst,
                                             char* __restrict__ ops, int64_t cap)
{
    __shared__ uint32_t win[kWinCols][kWinWords];
    const int lane = threadIdx.x;
    const WalkState s0 = *wst;
    if (s0.done)
        return;
    // The state is the same in every lane: held in 32-bit scalars (positions,
    // block bounds and operation counts are below 2^31), so that a step of the
    // walk is a few scalar instructions and one LDS read.
    int i = walk_uniform((int)s0.i), j = walk_uniform((int)s0.j), n_ops = walk_uniform((int)s0.n_ops);
    int st = walk_uniform(s0.st), prev_m = walk_uniform(s0.prev_m), ok = walk_uniform(s0.ok), done = 0;
    int bi = 0, bj = 0;
    const int rlo = (int)r_lo, clo = (int)c_lo;
    const int rhi = (int)(r_hi < INT32_MAX ? r_hi : INT32_MAX), chi = (int)(c_hi < INT32_MAX ? c_hi : INT32_MAX);
    const int lim = (int)(cap < INT32_MAX ? cap : INT32_MAX);
    const int w_lo = rlo >> 3;                 // r_lo is a multiple of 8
    // window: block columns c0 .. c0 + 63, block words w0 .. w0 + 15.  Every
    // step moves up, left or both, so a window placed with the walk's cell at
    // its lower right corner is left only through its top or left edge.
    int c0 = INT32_MAX, w0 = 0;
    for (;;) {
        if (i < 1 || j < 1 || n_ops >= lim) {                // off the matrix: inconsistent codes
            done = 1;
            ok = 0;
            break;
        }
        if (i - 1 < rlo || j - 1 < clo || i - 1 >= rhi || j - 1 >= chi)
            break;                                            // the next cell is in another block
        const int col = j - 1 - clo, row = i - 1, wd = (row >> 3) - w_lo;
        if (col < c0 || wd < w0) {
            __syncthreads();
            c0 = col - (kWinCols - 1) > 0 ? col - (kWinCols - 1) : 0;
            w0 = wd - (kWinWords - 1) > 0 ? wd - (kWinWords - 1) : 0;
            const int cc = c0 + lane;
            if (cc <= col) {
                // all loads in flight at once: clamped addresses, words past
                // the column's end read as zero afterwards
                uint32_t v[kWinWords];
#pragma unroll
                for (int k = 0; k < kWinWords; ++k)
                    v[k] = dir[(int64_t)cc * stride + min((int64_t)w0 + k, stride - 1)];
#pragma unroll
                for (int k = 0; k < kWinWords; ++k)
                    win[lane][k] = ((int64_t)w0 + k < stride) ? v[k] : 0u;
            }
            __syncthreads();
        }
        // Cells the walk may reach from here in one direction without leaving
        // the window (hence the block) or passing the operation cap: lane l
        // looks at the l-th of them, and a ballot takes the run of steps that
        // continue the same way, so a run costs one pass instead of one per
        // step.
        const int room_r = row - ((w0 + w_lo) << 3) + 1, room_c = col - c0 + 1;
        const int left = lim - n_ops;
        const int dr = st == 1 ? 0 : 1, dc = st == 2 ? 0 : 1;        // diagonal, left (E) or up (F)
        const int room = min(min(dr ? room_r : kWave, dc ? room_c : kWave), min(left, kWave));
        const int l = lane < room ? lane : 0;
        const int rr = row - dr * l, cl = col - dc * l;
        const uint32_t c = (win[cl - c0][(rr >> 3) - w_lo - w0] >> (4 * (rr & 7))) & 15u;
        if (st == 0) {
            const unsigned long long run = __ballot(lane < room && (c & 3u) == 1u);
            const int k = ~run ? __builtin_ctzll(~run) : kWave;       // diagonal steps in a row
            if (k > 0) {
                // the walk ends at the border after the first cell of the
                // run on row 1 or column 1
                const int nb = min(i, j) <= k ? min(i, j) : k;
                if (lane < nb)
                    ops[n_ops + lane] = 'M';
                n_ops += nb;
                prev_m = 1;
                if (nb < k || min(i, j) == k) {
                    done = 1;
                    bi = i - (nb - 1);
                    bj = j - (nb - 1);
                    break;
                }
                i -= k;
                j -= k;
                continue;
            }
            const uint32_t src = (uint32_t)walk_uniform((int)c) & 3u;
            if (src == 0u) {
                // H = 0: after a diagonal step the alignment began at the
                // previous cell; anywhere else the codes are inconsistent
                done = 1;
                ok = prev_m;
                bi = i + 1;
                bj = j + 1;
                break;
            }
            prev_m = 0;
            st = src == 2u ? 1 : 2;
            continue;
        }
        // in a gap: each cell emits its operation; the gap was opened at the
        // first cell whose flag says so, and the walk is back in H after it
        const unsigned long long opened = __ballot(lane < room && (c & (st == 1 ? 4u : 8u)) != 0u);
        const int k = opened ? __builtin_ctzll(opened) + 1 : room;
        if (lane < k)
            ops[n_ops + lane] = st == 1 ? 'D' : 'I';
        n_ops += k;
        prev_m = 0;
        if (st == 1)
            j -= k;
        else
            i -= k;
        if (opened)
            st = 0;
    }
    __syncthreads();
    if (lane == 0) {
        WalkState s = s0;
        s.i = i;
        s.j = j;
        s.n_ops = n_ops;
        s.st = st;
        s.prev_m = prev_m;
        s.ok = ok;
        s.done = done;
        if (done && bi) {
            s.bi = bi;
            s.bj = bj;
        }
        *wst = s;
    }
}

__global__ void __launch_bounds__(64) k_walk_finish(const WalkState* __restrict__ wst,
                                                    const int32_t* __restrict__ score, char* __restrict__ ops,
                                                    AlignOut* out)
{
    const int lane = threadIdx.x;
    const WalkState s = *wst;
    AlignOut r{};
    r.score = *score;
    if (s.n_ops > 0 || s.q_end > 0) {
        r.q_end = s.q_end;
        r.s_end = s.s_end;
        if (s.done && s.ok) {
            r.q_begin = (int32_t)s.bi;
            r.s_begin = (int32_t)s.bj;
            r.n_ops = (int32_t)s.n_ops;
            for (int64_t x = lane, y = s.n_ops - 1 - lane; x < y; x += 64, y -= 64) {
                const char t = ops[x];
                ops[x] = ops[y];
                ops[y] = t;
            }
        } else {
            r.n_ops = -1;                                  // reported as an error by the host
        }
    }
    if (lane == 0)
        *out = r;
}

hipError_t launch_trace_diag(const PairArgs& a, int elem, hipStream_t st)
{
    const int waves = a.ntiles;                   // K = 64: one tile per wave
    const int blocks = (waves + 3) / 4;
    if (elem == 1)
        hipLaunchKernelGGL((k_trace_diag<1>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_trace_diag<2>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_trace_reset(unsigned long long* end_key, hipStream_t st)
{
    hipLaunchKernelGGL(k_trace_reset, dim3(1), dim3(64), 0, st, end_key);
    return hipGetLastError();
}

hipError_t launch_walk_init(const unsigned long long* end_key, const int32_t* score, WalkState* w,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_init, dim3(1), dim3(64), 0, st, end_key, score, w);
    return hipGetLastError();
}

hipError_t launch_walk(const uint32_t* dir, int64_t dir_stride, int64_t r_lo, int64_t c_lo, int64_t r_hi,
                       int64_t c_hi, WalkState* w, char* ops, int64_t cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk, dim3(1), dim3(kWinCols), 0, st, dir, dir_stride, r_lo, c_lo, r_hi, c_hi, w, ops,
                       cap);
    return hipGetLastError();
}

hipError_t launch_walk_finish(const WalkState* w, const int32_t* score, char* ops, AlignOut* out,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_finish, dim3(1), dim3(64), 0, st, w, score, ops, out);
    return hipGetLastError();
}

// Boundary buffers of a block run (bands [b_org, b_hi], chunks [c_org, c_hi]
// of the tile grid, kb / kc its checkpoint row / column indices): colbuf over
// the block's rows from checkpoint column kc - 1, rowbuf over its columns from
// checkpoint row kb - 1, and the corners of the first chunk's bands below the
// first from checkpoint column kc - 1 (the first band's corners come from the
// checkpoint row through PairArgs::top_ckpt).
__global__ void __launch_bounds__(256) k_block_init(PairArgs a, int64_t kb, int64_t kc, int64_t b_hi, int64_t c_org,
                                                    int64_t c_hi)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int64_t band_rows = (int64_t)a.K * 8;
    const int64_t r0 = (int64_t)a.b_org * band_rows, r1 = (b_hi + 1) * band_rows;
    const int64_t col0 = c_org * a.wc, col1 = (c_hi + 1) * a.wc;
    if (kc > 0) {
        const int2* src = a.ckpt_col + (kc - 1) * a.ckpt_col_stride;
        for (int64_t r = r0 + t; r < r1; r += nt)
            a.colbuf[r] = src[r];
        for (int64_t b = a.b_org + 1 + t; b <= b_hi; b += nt)
            a.corner[b * 3 + c_org % 3] = src[b * band_rows - 1].x;
    }
    if (kb > 0) {
        const int2* src = a.ckpt_row + (kb - 1) * a.ckpt_row_stride;
        for (int64_t c = col0 + t; c < col1; c += nt)
            a.rowbuf[c] = src[c];
    }
}

hipError_t launch_block_init(const PairArgs& a, int64_t kb, int64_t kc, int64_t b_hi, int64_t c_org,
                             int64_t c_hi, hipStream_t st)
{
    hipLaunchKernelGGL(k_block_init, dim3(1024), dim3(256), 0, st, a, kb, kc, b_hi, c_org, c_hi);
    return hipGetLastError();
}

hipError_t launch_pair_diag_ckpt(const PairArgs& a, int elem, hipStream_t st)
{
    const int blocks = (a.ntiles + 3) / 4;        // K = 64: one tile per wave
    if (elem == 1)
        hipLaunchKernelGGL((k_pair_diag_ckpt<1>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_pair_diag_ckpt<2>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Padded subject copy (codes taken modulo 32, pad code past the end) and the
// score cleared; thread 0 also stores the query's profile descriptor and
// offset, which the profile kernel reads from device memory.
__global__ void __launch_bounds__(256) k_pair_prep(const uint8_t* __restrict__ src, int64_t n, int64_t n_pad,
                                                   uint8_t* __restrict__ dst, int32_t* score, QueryDesc qd,
                                                   QueryDesc* qd_out, int64_t* qoff_out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *score = 0;
        *qd_out = qd;
        *qoff_out = 0;
    }
    for (int64_t j = t; j < n_pad; j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = j < n ? (uint8_t)(src[j] & (kAlpha - 1)) : kPad;
}

hipError_t launch_pair_prep(const uint8_t* subj, int64_t n, int64_t n_pad, uint8_t* dst, int32_t* score,
                            const QueryDesc& qd, QueryDesc* qd_out, int64_t* qoff_out, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n_pad + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_pair_prep, dim3((unsigned)blocks), dim3(256), 0, st, subj, n, n_pad, dst, score, qd,
                       qd_out, qoff_out);
    return hipGetLastError();
}

template <int R>
void launch_skew_rows(const PairArgs& a, int elem, int blocks, hipStream_t st)
{
    if (elem == 1)
        hipLaunchKernelGGL((k_pair_skew<R, 1>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_pair_skew<R, 2>), dim3(blocks), dim3(256), 0, st, a);
}

hipError_t launch_trace_skew(const PairArgs& a, int elem, hipStream_t st)
{
    const int groups_per_wave = kWave / a.K;
    const int waves = (a.ntiles + groups_per_wave - 1) / groups_per_wave;
    const int blocks = (waves + 3) / 4;
    if (elem == 1)
        hipLaunchKernelGGL((k_trace_skew<1>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_trace_skew<2>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pair_skew(const PairArgs& a, int rows, int elem, hipStream_t st)
{
    const int groups_per_wave = kWave / a.K;
    const int waves = (a.ntiles + groups_per_wave - 1) / groups_per_wave;
    const int blocks = (waves + 3) / 4;
    switch (rows) {
    case 8: launch_skew_rows<8>(a, elem, blocks, st); break;
    case 16: launch_skew_rows<16>(a, elem, blocks, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swdb
