// Device code of the gfx950 Smith-Waterman / Gotoh database search: the cell
// update, the wavefront work item, and the persistent search kernels.  Each
// kernel variant is instantiated in its own translation unit.
//
// The recurrence (paper Section 2.2, equations for H, E and F; zero borders;
// score S = largest H) is evaluated per cell with integer add/sub/max only,
// so the work runs on the vector ALUs; there is no MFMA in this path.
//
// Value representation inside the kernels.  For every cell the lane keeps
//   Y = H - Go   (used by the E equation of the next column, the F equation of
//                 the next row and, with the profile entry s + Go, as the
//                 diagonal term: Y[i-1][j-1] + (s + Go) = H[i-1][j-1] + s)
//   E            clamped at 0 (int32 lanes)
// and carries F and Y down a column.  Clamping E at 0, or letting E and F
// saturate at the bottom of the 16-bit range, never changes H: with Go, Ge >= 0
// every E or F derived from the zero borders is <= 0 and H already has a zero
// floor.  Per cell this is the paper's Algorithm 1 (two subtractions and a
// maximum for E, the same for F, an addition and maxima for H, the running
// maximum S) with the H - Go subtraction shared between E and F and the
// three-input maximum instruction of gfx950 merging two maxima.
//
// Work decomposition (inter-task parallelism, paper Section 2.2 / Fig. 1):
//   * subjects are sorted by length and interleaved 64 to a chunk, 16
//     residues per lane per 16-column block, so one wavefront load of a block is
//     1 KiB of contiguous bytes;
//   * a lane keeps R query rows in registers and sweeps all columns of its
//     subject; K lanes may share one subject, each owning R rows of a K*R-row
//     pass, lane g running one column behind lane g-1 and receiving the bottom
//     row of lane g-1 through a DPP wave shift (the limited intra-task form of
//     Fig. 1, used for long subjects);
//   * consecutive passes exchange the bottom row (Y, F) of every column through
//     a per-wavefront slot in the workspace;
//   * the query profile (s + Go for each residue code and query row) is staged
//     in LDS when it fits, otherwise read through the cache hierarchy.
//
// Packed 16-bit variant: two subjects per lane (low and high halves), signed
// saturating add/sub and packed max.  A subject whose 16-bit score equals
// 32767 may have saturated and is listed for an exact int32 rescore; any score
// below 32767 is exact because no intermediate value can have saturated.
#pragma once
#include "sw_internal.h"

namespace swdb {

extern "C" __shared__ __align__(16) uint8_t sw_lds[];

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t comp(const uint4& v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

__device__ __forceinline__ int shr1(int v)
{
    // lane i receives lane i-1 (DPP wave_shr:1); lane 0 keeps v (it is a group head)
    return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ int ror1(int v)
{
    // lane i receives lane i-1, lane 0 receives lane 63 (DPP wave_ror:1)
    return __builtin_amdgcn_update_dpp(v, v, 0x13c, 0xf, 0xf, false);
}

template <bool LDSP>
__device__ __forceinline__ uint4 ld16(const uint8_t* __restrict__ g, uint32_t off)
{
    if constexpr (LDSP)
        return *reinterpret_cast<const uint4*>(sw_lds + off);
    else
        return *reinterpret_cast<const uint4*>(g + off);
}

template <bool LDSP>
__device__ __forceinline__ uint2 ld8(const uint8_t* __restrict__ g, uint32_t off)
{
    if constexpr (LDSP)
        return *reinterpret_cast<const uint2*>(sw_lds + off);
    else
        return *reinterpret_cast<const uint2*>(g + off);
}

// The NB profile bytes of one residue code in one row block (NB a multiple of
// 8), as 16-byte vectors; a trailing half vector is zero-filled.
template <int NB, bool LDSP>
__device__ __forceinline__ void ldprof(uint4 (&v)[(NB + 15) / 16], const uint8_t* __restrict__ g, uint32_t off)
{
    static_assert(NB % 8 == 0, "profile row blocks are whole 8-byte units");
#pragma unroll
    for (int i = 0; i < NB / 16; ++i)
        v[i] = ld16<LDSP>(g, off + 16 * i);
    if constexpr (NB % 16 == 8) {
        const uint2 t = ld8<LDSP>(g, off + NB - 8);
        v[NB / 16] = make_uint4(t.x, t.y, 0u, 0u);
    }
}

// profile entry r of a loaded row block (sign-extended)
template <int ES, int NV>
__device__ __forceinline__ int pent(const uint4 (&v)[NV], int r)
{
    if constexpr (ES == 1) {
        const uint32_t w = comp(v[r >> 4], (r >> 2) & 3);
        return (int)(int8_t)(w >> (8 * (r & 3)));
    } else {
        const uint32_t w = comp(v[r >> 3], (r >> 1) & 3);
        return (int)(int16_t)(w >> (16 * (r & 1)));
    }
}

__device__ __forceinline__ uint4 pad16()
{
    const uint32_t p = 0x20202020u;   // four pad codes
    return make_uint4(p, p, p, p);
}

__device__ __forceinline__ int imax3(int a, int b, int c)
{
    return max(max(a, b), c);
}

// Materialise the running maximum in a register at this point.  Without it the
// compiler reassociates S = max(S, h) over every row of the unrolled body into
// one tree at the end, which keeps all those h values live and spills.  The
// statement emits no instruction.
template <typename T>
__device__ __forceinline__ void pin(T& v)
{
    asm volatile("" : "+v"(v));
}

typedef short v2s __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v2s as2(uint32_t x) { return __builtin_bit_cast(v2s, x); }
__device__ __forceinline__ uint32_t asu(v2s x) { return __builtin_bit_cast(uint32_t, x); }

// Slot layout: for each group of 4 columns, each lane group's 4 (Y, F) pairs
// are contiguous, so a 4-column group is two 16-byte accesses.  Entry of
// column `col` for lane group `sub`: (col / 4 * nsubw + sub) * 4 + col % 4;
// slot_col is the part that does not depend on the lane group.
__device__ __forceinline__ int64_t slot_col(int col, int nsubw)
{
    return (int64_t)(col >> 2) * nsubw * 4 + (col & 3);
}

// ------------------------------------------------------------------ int32 item

// One wavefront sweeps one item and writes its scores.  ES = profile entry
// bytes (1 or 2).  MULTI: lane groups of K > 1 lanes per subject.
template <int R, int ES, bool LDSP, bool MULTI>
__device__ __forceinline__ void item_i32(const SearchArgs& a, const Item it, const QueryDesc& qd,
                                         int2* __restrict__ slot, int lane)
{
    constexpr uint32_t CS = code_stride(R, ES);   // code stride (bytes)
    constexpr uint32_t BS = kCodes * CS;          // row-block stride (bytes)
    constexpr int NB = R * ES;                    // profile bytes per code
    constexpr int NV = (NB + 15) / 16;

    const int nsub = it.meta & 0xffff;
    const int K = MULTI ? ((it.meta >> 16) & 0xff) : 1; // lanes per subject, 1..64
    const int nsubw = MULTI ? kWave / K : kWave;        // lane groups in the wavefront
    const int sub = MULTI ? lane / K : lane;
    const int g = lane - sub * K;
    const bool inb = sub < nsubw;                       // lane belongs to a group
    const bool valid = sub < nsub;                      // nsub <= nsubw
    const int s = it.s0 + (valid ? sub : 0);
    const bool head = g == 0;
    const bool tail = g == K - 1;

    const uint4* __restrict__ resp = reinterpret_cast<const uint4*>(a.res + a.chunk_off[s >> 6]) + (s & 63);
    const int own = (a.slen[s] + 15) & ~15;   // columns stored for this lane's subject
    const int ncols = it.ncols;
    const int nbr = qd.nbr;
    const int P = (nbr + K - 1) / K;
    const int nsteps = MULTI ? ((ncols + K - 1 + 3) & ~3) : ncols;   // multiple of 4
    const int go = a.go, ge = a.ge;
    const uint8_t* __restrict__ gprof = a.prof + qd.prof_off;
    // this lane's slot entries: column c is lslot[slot_col(c, nsubw)] (a
    // wavefront-uniform offset)
    int2* __restrict__ lslot = slot + (int64_t)(inb ? sub : 0) * 4;

    int S = 0;
    for (int pass = 0; pass < P; ++pass) {
        const int rb = min(pass * K + g, nbr);     // row block nbr is all padding
        const uint32_t pbase = (uint32_t)rb * BS;
        const bool rd = pass > 0;
        const bool wr = pass < P - 1;
        int Y[R], E[R];
#pragma unroll
        for (int r = 0; r < R; ++r) { Y[r] = -go; E[r] = 0; }
        int ydiag = -go, ybot = -go, fbot = 0, code_prev = kPad;

        uint4 rv = (head && 0 < own) ? resp[0] : pad16();
        for (int blk = 0; blk < nsteps; blk += 16) {
            const uint4 rvn = (head && blk + 16 < own) ? resp[(blk + 16) * 4] : pad16();
            const int n4 = min(4, (nsteps - blk) >> 2);   // 4-column groups in this block
#pragma unroll 1
            for (int k4 = 0; k4 < n4; ++k4) {
                const int col0 = blk + 4 * k4;
                const uint32_t w = rv.x;                      // columns col0..col0+3
                rv = make_uint4(rv.y, rv.z, rv.w, 0u);
                int ringY[4], ringF[4];
                if (rd && col0 < ncols && inb) {
                    const int4* p4 = reinterpret_cast<const int4*>(lslot + slot_col(col0, nsubw));
                    const int4 v0 = p4[0], v1 = p4[1];
                    ringY[0] = v0.x; ringF[0] = v0.y; ringY[1] = v0.z; ringF[1] = v0.w;
                    ringY[2] = v1.x; ringF[2] = v1.y; ringY[3] = v1.z; ringF[3] = v1.w;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) { ringY[k] = -go; ringF[k] = 0; }
                }
                int wY[4], wF[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int code = (int)((w >> (8 * u)) & 0xffu);
                    int yt = ringY[u], ft = ringF[u];
                    if constexpr (MULTI) {
                        const int cd = shr1(code_prev);
                        const int yd = shr1(ybot), fd = shr1(fbot);
                        code = head ? code : cd;
                        yt = head ? yt : yd;
                        ft = head ? ft : fd;
                    }
                    uint4 pv[NV];
                    ldprof<NB, LDSP>(pv, gprof, pbase + (uint32_t)code * CS);

                    int dg = ydiag;
                    ydiag = yt;
                    int hup = yt, F = ft;
                    int hprev = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int t = dg + pent<ES>(pv, r);          // H[i-1][j-1] + s
                        const int e = imax3(E[r] - ge, Y[r], 0);     // E (clamped at 0)
                        F = max(F - ge, hup);                        // F
                        const int h = imax3(t, e, F);                // H
                        if (r & 1) {
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
                    code_prev = code;
                    wY[u] = ybot;
                    wF[u] = fbot;
                    if constexpr (MULTI) {
                        const int j = col0 + u - (K - 1);
                        if (wr && tail && inb && j >= 0 && j < ncols)
                            lslot[slot_col(j, nsubw)] = make_int2(ybot, fbot);
                    }
                }
                if constexpr (!MULTI) {
                    if (wr && col0 < ncols) {
                        int4* p4 = reinterpret_cast<int4*>(lslot + slot_col(col0, nsubw));
                        p4[0] = make_int4(wY[0], wF[0], wY[1], wF[1]);
                        p4[1] = make_int4(wY[2], wF[2], wY[3], wF[3]);
                    }
                }
            }
            rv = rvn;
        }
        // this pass's bottom rows must be visible to the next pass's first rows
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    if constexpr (MULTI) {
        const int hl = min(sub * K, kWave - 1);
        for (int k = 1; k < K; ++k)
            S = max(S, __shfl(S, min(hl + k, kWave - 1)));
    }
    if (head && valid)
        a.scores[(int64_t)qd.out_row * a.out_stride + a.perm[s]] = S;
}

// ------------------------------------------------------------------ packed 16-bit item

// One column of R rows in both 16-bit halves of a lane (low half: profile
// vector pa, high half: pb).  yt / ft enter the top row (H - Go and F of the
// row above), ydiag is H - Go of the row above in the previous column; ybot /
// fbot leave the bottom row.  ES = profile entry bytes: 2 (signed 16-bit) or 1
// (8-bit entries in [0, 127], zero-extended while the halves are paired).
template <int R, int ES, int NV>
__device__ __forceinline__ void column_i16(const uint4 (&pa)[NV], const uint4 (&pb)[NV], uint32_t (&Y)[R],
                                           uint32_t (&E)[R], uint32_t& ydiag, uint32_t yt, uint32_t ft,
                                           uint32_t& ybot, uint32_t& fbot, v2s& S, v2s vge, v2s vgo)
{
    const v2s zero = {0, 0};
    v2s dg = as2(ydiag);
    ydiag = yt;
    v2s hup = as2(yt), F = as2(ft);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        // (low-half entry, high-half entry) of row r; selector bytes 0-3 pick
        // from xa, 4-7 from xb, 0x0c gives 0x00
        uint32_t pr;
        if constexpr (ES == 2) {
            const uint32_t xa = comp(pa[r >> 3], (r >> 1) & 3);
            const uint32_t xb = comp(pb[r >> 3], (r >> 1) & 3);
            pr = __builtin_amdgcn_perm(xb, xa, (r & 1) ? 0x07060302u : 0x05040100u);
        } else {
            const uint32_t xa = comp(pa[r >> 4], (r >> 2) & 3);
            const uint32_t xb = comp(pb[r >> 4], (r >> 2) & 3);
            pr = __builtin_amdgcn_perm(xb, xa, 0x0c000c00u | (uint32_t)(r & 3) | ((uint32_t)(4 + (r & 3)) << 16));
        }
        const v2s t = __builtin_elementwise_add_sat(dg, as2(pr));
        const v2s e = __builtin_elementwise_max(__builtin_elementwise_sub_sat(as2(E[r]), vge), as2(Y[r]));
        F = __builtin_elementwise_max(__builtin_elementwise_sub_sat(F, vge), hup);
        const v2s h = __builtin_elementwise_max(__builtin_elementwise_max(t, e), __builtin_elementwise_max(F, zero));
        S = __builtin_elementwise_max(S, h);
        if (r & 1)
            pin(S);
        dg = as2(Y[r]);
        hup = h - vgo;
        Y[r] = asu(hup);
        E[r] = asu(e);
    }
    ybot = asu(hup);
    fbot = asu(F);
}

// Two subjects per lane (low and high halves); ES as for column_i16.
template <int R, int ES, bool LDSP, bool MULTI>
__device__ __forceinline__ void item_i16(const SearchArgs& a, const Item it, const QueryDesc& qd,
                                         int2* __restrict__ slot, int lane)
{
    constexpr uint32_t CS = code_stride(R, ES);
    constexpr uint32_t BS = kCodes * CS;
    constexpr int NB = R * ES;
    constexpr int NV = (NB + 15) / 16;

    const int nsub = it.meta & 0xffff;
    const int K = MULTI ? ((it.meta >> 16) & 0xff) : 1;
    const int nsubw = MULTI ? kWave / K : kWave;
    const int sub = MULTI ? lane / K : lane;
    const int g = lane - sub * K;
    const bool inb = sub < nsubw;
    const bool validA = inb && sub < nsub;
    const bool validB = inb && sub + nsubw < nsub;
    const int sA = it.s0 + (validA ? sub : 0);
    const int sB = it.s0 + (validB ? sub + nsubw : 0);
    const bool head = g == 0;
    const bool tail = g == K - 1;

    const uint4* __restrict__ respA = reinterpret_cast<const uint4*>(a.res + a.chunk_off[sA >> 6]) + (sA & 63);
    const uint4* __restrict__ respB = reinterpret_cast<const uint4*>(a.res + a.chunk_off[sB >> 6]) + (sB & 63);
    const int ownA = validA ? (a.slen[sA] + 15) & ~15 : 0;
    const int ownB = validB ? (a.slen[sB] + 15) & ~15 : 0;
    const int ncols = it.ncols;
    const int nbr = qd.nbr;
    const int P = (nbr + K - 1) / K;
    const int nsteps = MULTI ? ((ncols + K - 1 + 3) & ~3) : ncols;   // multiple of 4
    const uint32_t go2 = (uint32_t)(a.go & 0xffff) * 0x10001u;
    const uint32_t ge2 = (uint32_t)(a.ge & 0xffff) * 0x10001u;
    const uint32_t ngo2 = (uint32_t)((-a.go) & 0xffff) * 0x10001u;
    const uint8_t* __restrict__ gprof = a.prof + qd.prof_off;
    const v2s zero = {0, 0};
    const v2s vge = as2(ge2), vgo = as2(go2);
    int2* __restrict__ lslot = slot + (int64_t)(inb ? sub : 0) * 4;

    v2s S = zero;
    for (int pass = 0; pass < P; ++pass) {
        const int rb = min(pass * K + g, nbr);
        const uint32_t pbase = (uint32_t)rb * BS;
        const bool rd = pass > 0;
        const bool wr = pass < P - 1;
        uint32_t Y[R], E[R];
#pragma unroll
        for (int r = 0; r < R; ++r) { Y[r] = ngo2; E[r] = 0; }
        uint32_t ydiag = ngo2, ybot = ngo2, fbot = 0;
        int code_prev = kPad | (kPad << 8);

        uint4 rvA = (head && 0 < ownA) ? respA[0] : pad16();
        uint4 rvB = (head && 0 < ownB) ? respB[0] : pad16();
        for (int blk = 0; blk < nsteps; blk += 16) {
            const uint4 rvnA = (head && blk + 16 < ownA) ? respA[(blk + 16) * 4] : pad16();
            const uint4 rvnB = (head && blk + 16 < ownB) ? respB[(blk + 16) * 4] : pad16();
            const int n4 = min(4, (nsteps - blk) >> 2);   // 4-column groups in this block
#pragma unroll 1
            for (int k4 = 0; k4 < n4; ++k4) {
                const int col0 = blk + 4 * k4;
                // columns col0..col0+3: the block's word picked rather than shifted
                // out (the shift made every 4-column trip wait for all memory
                // operations in flight, the next block's residues among them)
                const uint32_t wA = comp(rvA, k4), wB = comp(rvB, k4);
                uint32_t ringY[4], ringF[4];
                if (rd && col0 < ncols && inb) {
                    const uint4* p4 = reinterpret_cast<const uint4*>(lslot + slot_col(col0, nsubw));
                    const uint4 v0 = p4[0], v1 = p4[1];
                    ringY[0] = v0.x; ringF[0] = v0.y; ringY[1] = v0.z; ringF[1] = v0.w;
                    ringY[2] = v1.x; ringF[2] = v1.y; ringY[3] = v1.z; ringF[3] = v1.w;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) { ringY[k] = ngo2; ringF[k] = 0; }
                }
                uint32_t wY[4], wF[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int code = (int)(((wA >> (8 * u)) & 0xffu) | (((wB >> (8 * u)) & 0xffu) << 8));
                    uint32_t yt = ringY[u], ft = ringF[u];
                    if constexpr (MULTI) {
                        const int cd = shr1(code_prev);
                        const uint32_t yd = (uint32_t)shr1((int)ybot), fd = (uint32_t)shr1((int)fbot);
                        code = head ? code : cd;
                        yt = head ? yt : yd;
                        ft = head ? ft : fd;
                    }
                    uint4 pa[NV], pb[NV];
                    ldprof<NB, LDSP>(pa, gprof, pbase + (uint32_t)(code & 0xff) * CS);
                    ldprof<NB, LDSP>(pb, gprof, pbase + (uint32_t)(code >> 8) * CS);

                    column_i16<R, ES>(pa, pb, Y, E, ydiag, yt, ft, ybot, fbot, S, vge, vgo);
                    code_prev = code;
                    wY[u] = ybot;
                    wF[u] = fbot;
                    if constexpr (MULTI) {
                        const int j = col0 + u - (K - 1);
                        if (wr && tail && inb && j >= 0 && j < ncols)
                            lslot[slot_col(j, nsubw)] = make_int2((int)ybot, (int)fbot);
                    }
                }
                if constexpr (!MULTI) {
                    if (wr && col0 < ncols) {
                        uint4* p4 = reinterpret_cast<uint4*>(lslot + slot_col(col0, nsubw));
                        p4[0] = make_uint4(wY[0], wF[0], wY[1], wF[1]);
                        p4[1] = make_uint4(wY[2], wF[2], wY[3], wF[3]);
                    }
                }
            }
            rvA = rvnA;
            rvB = rvnB;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    uint32_t Su = asu(S);
    if constexpr (MULTI) {
        const int hl = min(sub * K, kWave - 1);
        uint32_t acc = Su;
        for (int k = 1; k < K; ++k)
            acc = asu(__builtin_elementwise_max(as2(acc), as2((uint32_t)__shfl((int)Su, min(hl + k, kWave - 1)))));
        Su = acc;
    }
    if (head) {
        const int lo = (int)(int16_t)(Su & 0xffff);
        const int hi = (int)(int16_t)(Su >> 16);
        const int64_t ob = (int64_t)qd.out_row * a.out_stride;
        if (validA) {
            if (lo == 32767) {
                const int k = atomicAdd(&a.counters[1], 1);
                if (k < a.flag_cap) a.flags[k] = make_int2(it.q, sA);
                else atomicAdd(&a.status[kStatusRescoreFailed], 1);
            } else {
                a.scores[ob + a.perm[sA]] = lo;
            }
        }
        if (validB) {
            if (hi == 32767) {
                const int k = atomicAdd(&a.counters[1], 1);
                if (k < a.flag_cap) a.flags[k] = make_int2(it.q, sB);
                else atomicAdd(&a.status[kStatusRescoreFailed], 1);
            } else {
                a.scores[ob + a.perm[sB]] = hi;
            }
        }
    }
}

// Self-paired item (packed variant, the longest subjects): one subject per
// wavefront, and the two halves of lane g hold two row blocks of it -- the
// low half row block pass*128 + g, the high half pass*128 + 64 + g -- so one
// pass covers 128 row blocks and the per-lane work of the subject (the
// critical path of its item) is half that of 64-lane groups carrying two
// subjects.  Low halves run as a 64-lane pipeline (lane g one column behind
// lane g-1); the high halves continue it 64 columns later: a DPP wave
// rotation hands lane 63's low-half bottom row (and residue code) to lane 0's
// high half, and lane 63's high half writes the pass's bottom row to the slot
// (linear, one (H - Go, F) entry per column, value in the low 16 bits).
template <int R, int ES, bool LDSP>
__device__ __forceinline__ void item_i16_self(const SearchArgs& a, const Item it, const QueryDesc& qd,
                                              int2* __restrict__ slot, int lane)
{
    constexpr uint32_t CS = code_stride(R, ES);
    constexpr uint32_t BS = kCodes * CS;
    constexpr int NB = R * ES;
    constexpr int NV = (NB + 15) / 16;
    constexpr int D = 2 * kWave;                  // row blocks per pass; pipeline depth

    const int s = it.s0;
    const bool head = lane == 0;
    const bool tail = lane == kWave - 1;
    const uint4* __restrict__ resp = reinterpret_cast<const uint4*>(a.res + a.chunk_off[s >> 6]) + (s & 63);
    const int own = (a.slen[s] + 15) & ~15;
    const int ncols = it.ncols;
    const int nbr = qd.nbr;
    const int P = (nbr + D - 1) / D;
    const int nsteps = (ncols + D - 1 + 3) & ~3;
    const uint32_t go2 = (uint32_t)(a.go & 0xffff) * 0x10001u;
    const uint32_t ge2 = (uint32_t)(a.ge & 0xffff) * 0x10001u;
    const uint32_t ngo2 = (uint32_t)((-a.go) & 0xffff) * 0x10001u;
    const uint8_t* __restrict__ gprof = a.prof + qd.prof_off;
    const v2s vge = as2(ge2), vgo = as2(go2);

    v2s S = {0, 0};
    for (int pass = 0; pass < P; ++pass) {
        const uint32_t pbA = (uint32_t)min(pass * D + lane, nbr) * BS;          // row block nbr is padding
        const uint32_t pbB = (uint32_t)min(pass * D + kWave + lane, nbr) * BS;
        const bool rd = pass > 0;
        const bool wr = pass < P - 1;
        uint32_t Y[R], E[R];
#pragma unroll
        for (int r = 0; r < R; ++r) { Y[r] = ngo2; E[r] = 0; }
        uint32_t ydiag = ngo2, ybot = ngo2, fbot = 0;
        int code_prev = kPad | (kPad << 8);

        uint4 rv = (head && 0 < own) ? resp[0] : pad16();
        for (int blk = 0; blk < nsteps; blk += 16) {
            const uint4 rvn = (head && blk + 16 < own) ? resp[(blk + 16) * 4] : pad16();
            const int n4 = min(4, (nsteps - blk) >> 2);
#pragma unroll 1
            for (int k4 = 0; k4 < n4; ++k4) {
                const int col0 = blk + 4 * k4;
                const uint32_t w = rv.x;
                rv = make_uint4(rv.y, rv.z, rv.w, 0u);
                uint32_t ringY[4], ringF[4];
                if (rd && col0 < ncols && head) {
                    const uint4* p4 = reinterpret_cast<const uint4*>(slot + col0);
                    const uint4 v0 = p4[0], v1 = p4[1];
                    ringY[0] = v0.x; ringF[0] = v0.y; ringY[1] = v0.z; ringF[1] = v0.w;
                    ringY[2] = v1.x; ringF[2] = v1.y; ringY[3] = v1.z; ringF[3] = v1.w;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) { ringY[k] = ngo2; ringF[k] = 0; }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // lane g-1's values of the previous column (lane 0: lane 63's)
                    int rc = ror1(code_prev);
                    int ry = ror1((int)ybot), rf = ror1((int)fbot);
                    pin(rc);
                    pin(ry);
                    pin(rf);
                    const int fresh = (int)((w >> (8 * u)) & 0xffu);
                    const int code = head ? (fresh | ((rc & 0xff) << 8)) : rc;
                    const uint32_t yt = head ? ((ringY[u] & 0xffffu) | ((uint32_t)ry << 16)) : (uint32_t)ry;
                    const uint32_t ft = head ? ((ringF[u] & 0xffffu) | ((uint32_t)rf << 16)) : (uint32_t)rf;
                    uint4 pa[NV], pb[NV];
                    ldprof<NB, LDSP>(pa, gprof, pbA + (uint32_t)(code & 0xff) * CS);
                    ldprof<NB, LDSP>(pb, gprof, pbB + (uint32_t)(code >> 8) * CS);
                    column_i16<R, ES>(pa, pb, Y, E, ydiag, yt, ft, ybot, fbot, S, vge, vgo);
                    code_prev = code;
                    const int j = col0 + u - (D - 1);
                    if (wr && tail && j >= 0 && j < ncols)
                        slot[j] = make_int2((int)(ybot >> 16), (int)(fbot >> 16));
                }
            }
            rv = rvn;
        }
        // this pass's bottom row must be visible to the next pass's first rows
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    const uint32_t Su = asu(S);
    int best = max((int)(int16_t)(Su & 0xffff), (int)(int16_t)(Su >> 16));
    for (int off = 32; off > 0; off >>= 1)
        best = max(best, __shfl_xor(best, off));
    if (head) {
        if (best == 32767) {
            const int k = atomicAdd(&a.counters[1], 1);
            if (k < a.flag_cap) a.flags[k] = make_int2(it.q, s);
            else atomicAdd(&a.status[kStatusRescoreFailed], 1);
        } else {
            a.scores[(int64_t)qd.out_row * a.out_stride + a.perm[s]] = best;
        }
    }
}

// ------------------------------------------------------------------ persistent kernels

// Defence against a work item inconsistent with the launch: every index the
// item functions derive (subjects, slot entries) stays inside its buffer.
template <bool I16>
__device__ __forceinline__ bool item_fits(const SearchArgs& a, const Item& it, const QueryDesc& qd)
{
    const int nsub = it.meta & 0xffff;
    const int K = (it.meta >> 16) & 0xff;
    if (nsub <= 0 || K < 1 || K > kWave || it.s0 < 0 || it.ncols < 0)
        return false;
    if ((it.meta >> 25) & 1)   // self-paired: packed lanes, one subject, 64 lanes, linear slot
        return I16 && nsub == 1 && K == kWave && it.s0 < a.nseq &&
               (qd.nbr <= 2 * kWave || (int64_t)it.ncols <= a.slot_elems);
    if (nsub > (kWave / K) * (I16 ? 2 : 1) || (int64_t)it.s0 + nsub > a.nseq)
        return false;
    return qd.nbr <= K || (int64_t)it.ncols * (kWave / K) <= a.slot_elems;
}

// Copy one query's profile into LDS (all threads of the workgroup).
__device__ __forceinline__ void stage_profile(const SearchArgs& a, const QueryDesc& qd)
{
    const uint4* __restrict__ src = reinterpret_cast<const uint4*>(a.prof + qd.prof_off);
    uint4* dst = reinterpret_cast<uint4*>(sw_lds);
    const int n = qd.prof_bytes >> 4;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        dst[i] = src[i];
}

// One work item with the variant its lane groups and profile location need.
// Items on the critical path (far more per-lane work than the planner's
// target: the longest subjects) raise their wavefront's issue priority so the
// waves sharing the SIMD do not stretch them.
template <int R, int ES, bool I16>
__device__ __forceinline__ void run_item(const SearchArgs& a, const Item& it, const QueryDesc& qd,
                                         int2* __restrict__ slot, int lane)
{
    const bool multi = ((it.meta >> 16) & 0xff) > 1;
    const bool crit = (it.meta >> 24) & 1;
    const bool self = (it.meta >> 25) & 1;
    if (crit)
        __builtin_amdgcn_s_setprio(2);
    if constexpr (I16) {
        if (self) {
            if (qd.lds) item_i16_self<R, ES, true>(a, it, qd, slot, lane);
            else item_i16_self<R, ES, false>(a, it, qd, slot, lane);
        } else if (qd.lds) {
            if (multi) item_i16<R, ES, true, true>(a, it, qd, slot, lane);
            else item_i16<R, ES, true, false>(a, it, qd, slot, lane);
        } else {
            if (multi) item_i16<R, ES, false, true>(a, it, qd, slot, lane);
            else item_i16<R, ES, false, false>(a, it, qd, slot, lane);
        }
    } else {
        if (qd.lds) {
            if (multi) item_i32<R, ES, true, true>(a, it, qd, slot, lane);
            else item_i32<R, ES, true, false>(a, it, qd, slot, lane);
        } else {
            if (multi) item_i32<R, ES, false, true>(a, it, qd, slot, lane);
            else item_i32<R, ES, false, false>(a, it, qd, slot, lane);
        }
    }
    if (crit)
        __builtin_amdgcn_s_setprio(0);
}

// Persistent search over per-query work queues.  Every workgroup walks the
// queries in queue order (largest first); within a query each wavefront takes
// items on its own with one atomic on that query's head -- no barriers, so the
// waves of a workgroup never wait for each other inside a query.  A query whose
// profile fits in LDS is staged there between two barriers: the first waits
// until every wave of the workgroup has left the previous query's queue, the
// second until the copy is complete (skipped when the queue is already empty:
// a wave that saw it empty knows every later take fails too).  The barrier
// sequence depends only on the descriptors, so every wave meets the same
// barriers.
template <int R, int ES, bool I16>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_search(SearchArgs a)
{
    const int W = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    int2* __restrict__ slot = a.bnd + (int64_t)(blockIdx.x * W + wave) * a.slot_elems;
    for (int p = 0; p < a.nq; ++p) {
        const QueryDesc qd = a.qd[p];
        if (qd.lds) {
            __syncthreads();
            if (__hip_atomic_load(&a.heads[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < qd.item_count)
                stage_profile(a, qd);
            __syncthreads();
        }
        for (;;) {
            int wi = 0;
            if (lane == 0)
                wi = atomicAdd(&a.heads[p], 1);
            wi = __builtin_amdgcn_readfirstlane(wi);
            const int64_t ix = (int64_t)qd.item_begin + wi;
            if (wi >= qd.item_count || ix >= a.n_items)
                break;
            const Item it = a.items[ix];
            if (it.q == p && item_fits<I16>(a, it, qd))
                run_item<R, ES, I16>(a, it, qd, slot, lane);
            else if (lane == 0)
                atomicAdd(&a.status[kStatusBadItems], 1);
        }
    }
}

template <typename F>
inline hipError_t launch_kernel(F kern, int grid, int waves, int lds, hipStream_t st, const SearchArgs& a)
{
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * waves), lds, st, a);
    return hipGetLastError();
}

template <typename F>
inline int occupancy_of(F kern, int waves, int lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 64 * waves, lds) != hipSuccess || n < 1)
        n = 1;
    return n;
}

}  // namespace swdb
