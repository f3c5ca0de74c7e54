// Pipelined pass over one long pair ("flow"): the score of one matrix with
// one launch in place of one launch per anti-diagonal of tiles.
//
// Every wavefront takes one band of 64 lanes x R query rows at a time (bands
// w, w + waves, w + 2 waves, ... in order) and sweeps all subject columns:
// lane g computes column t - g at step t, receiving the bottom row of lane
// g - 1 (and its residue code) through a DPP wave shift, as in the tile
// kernels.  The band's state never leaves registers.  Its last lane hands the
// band's bottom row to the band below through one 64-bit word per column of
// a buffer updated in place: bits 0-23 hold H - Go + Go, bits 24-47 F + Go,
// bits 48-63 a tag, band + 1.  The head lane of the band below reads the word
// of its column 16 steps ahead and, before using it, checks that the tag names
// the band just above (each step its own word, or from 8 rows per lane on,
// the 16 words of a block at once); tags are unique per band within a call
// (the buffer is cleared first), so a word not yet written is never mistaken
// for one that is.  The words are read and written with agent-scope coherent accesses
// (relaxed atomics: no cache writeback or invalidate is needed, since every
// word carries its own validity), so bands on different XCDs meet in memory.
//
// A band waits only for the band above it, which a lower-numbered wavefront
// or this wavefront's previous round runs; every wavefront of the launch is
// resident at once (the host checks the occupancy first), so the pipeline
// needs no other ordering.  Wavefronts are numbered XCD by XCD, so that most
// handoffs stay within one L2.  The bands advance at the pace of the
// slowest one, so the launch places them evenly: workgroups of W waves (W / 4
// per SIMD), one workgroup per CU (its LDS request keeps a second one off the
// CU), each wave with a band profile of its own in LDS.  Every wait is
// bounded in time: a wave that gives up sets the status word, the waves
// waiting behind it see it and stop, and the score is then reported as -1
// (k_pair_flow_finish).
//
// The packing holds values in [0, 2^24): the host takes this pass only when
// the largest possible score, max(SM) x min(m, n), is below 2^24 and the
// bands number at most 2^16 - 1.
#include <algorithm>
#include <type_traits>

#include "sw_device.h"

namespace swdb {

// raw buffer store cache policy: sc1 (agent-scope coherent, as a relaxed
// agent-scope atomic store)
constexpr int kStoreSc1 = 16;

__device__ __forceinline__ unsigned long long flow_word(const unsigned long long* rows, int j)
{
    return __hip_atomic_load(rows + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The NW 32-bit words of a profile row block's entries (16-byte aligned).
template <int NW>
__device__ __forceinline__ void flow_ldprof(uint32_t (&v)[NW], const uint8_t* __restrict__ p)
{
    constexpr int N4 = NW / 4 * 4;
#pragma unroll
    for (int i = 0; i < N4; i += 4) {
        const uint4 x = *reinterpret_cast<const uint4*>(p + 4 * i);
        v[i] = x.x; v[i + 1] = x.y; v[i + 2] = x.z; v[i + 3] = x.w;
    }
    if constexpr (NW - N4 >= 2) {
        const uint2 x = *reinterpret_cast<const uint2*>(p + 4 * N4);
        v[N4] = x.x; v[N4 + 1] = x.y;
    }
    if constexpr ((NW - N4) % 2 == 1)
        v[NW - 1] = *reinterpret_cast<const uint32_t*>(p + 4 * (NW - 1));
}

// The NW words of a lane's entries for one code from the band's LDS profile.
template <int NW, int PS>
__device__ __forceinline__ void flow_ldlds(uint32_t (&v)[NW], uint32_t off)
{
    static_assert(NW * 4 <= PS, "entries fit the stride");
    if constexpr (PS == 4) {
        v[0] = *reinterpret_cast<const uint32_t*>(sw_lds + off);
    } else if constexpr (PS == 8) {
        const uint2 x = *reinterpret_cast<const uint2*>(sw_lds + off);
        v[0] = x.x;
        if constexpr (NW > 1) v[1] = x.y;
    } else {
#pragma unroll
        for (int i = 0; i < NW; i += 4) {
            const uint4 x = *reinterpret_cast<const uint4*>(sw_lds + off + 4 * i);
            v[i] = x.x;
            if (i + 1 < NW) v[i + 1] = x.y;
            if (i + 2 < NW) v[i + 2] = x.z;
            if (i + 3 < NW) v[i + 3] = x.w;
        }
    }
}

template <int ES, int NW>
__device__ __forceinline__ int flow_entry(const uint32_t (&v)[NW], int r)
{
    if constexpr (ES == 1)
        return (int)(int8_t)(v[r >> 2] >> (8 * (r & 3)));
    else
        return (int)(int16_t)(v[r >> 1] >> (16 * (r & 1)));
}

// Slow path of a read: poll the word of column j until its tag is `want`,
// another wave has failed, or the time limit (or a poll count of the same
// order) passes; then *failed is set.
constexpr uint32_t kFlowMaxPolls = 1u << 25;
// Columns a band that had to wait lets the band above get ahead of its
// read-ahead: a handoff word can take a few microseconds to reach the band
// below, and a band that falls back by less keeps waiting again (measured on
// MI355X at 10 and 16 rows per lane: 32 columns beat 16).
constexpr int kFlowSlack = 32;

__device__ __forceinline__ unsigned long long flow_wait(const FlowArgs& a, int j, uint32_t want,
                                                           int* failed)
{
    const uint64_t begin = __builtin_amdgcn_s_memrealtime();
    for (uint32_t polls = 0;; ++polls) {
        const unsigned long long w = flow_word(a.rows, j);
        if (__builtin_amdgcn_readfirstlane((uint32_t)(w >> 48)) == want)
            return w;
        const int stop = __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(stop) != 0 || polls >= kFlowMaxPolls ||
            __builtin_amdgcn_s_memrealtime() - begin > a.timeout) {
            *failed = 1;
            __hip_atomic_fetch_or(a.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return w;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// max(a, b, c) as one v_max3_i32: written out because the compiler, knowing
// the cell values are non-negative, splits it into a signed and an unsigned
// two-input maximum
__device__ __forceinline__ int max3_i32(int a, int b, int c)
{
    int r;
    asm volatile("v_max3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t min3_u32(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_elementwise_min(__builtin_elementwise_min(a, b), c);
}

// TRACE: the direction-code pass of an alignment with whole-matrix codes:
// every cell's 4-bit code into the 32-bit word dir[column * dir_stride + row
// block] of its 8-row block (with 4 rows per lane, a lane writes the low or
// the high half of its block's word) and the first cell holding the score,
// column-major, into end_key, exactly as the code tiles do; no score.
template <int R, int ES, bool TRACE = false>
__device__ __forceinline__ void pair_flow(const FlowArgs& a, int wave_id, int lane, uint32_t lds0)
{
    static_assert(!TRACE || R == 8 || R == 4, "direction words hold 8 rows");
    constexpr uint32_t CS = code_stride(R, ES);
    constexpr uint32_t BS = kCodes * CS;
    constexpr int NW = (R * ES + 3) / 4;
    constexpr uint32_t PS = flow_lds_stride(R, ES);
    constexpr bool BLOCKWISE = R >= kFlowBlockwiseRows;     // the handoff words' tags checked per 16-step block

    const int n = a.n;
    const int go = a.go, ge = a.ge;
    const bool head = lane == 0, tail = lane == kWave - 1;
    const uint4* __restrict__ resp = reinterpret_cast<const uint4*>(a.subj);
    const int nblk = a.n_pad >> 4;
    const int T = n + kWave - 1;               // steps of a band
    const int nsteps16 = (T + 15) & ~15;
    typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
    // the tail lane's handoff store; the other lanes aim at entry n, past the
    // descriptor's range (dropped), still inside the buffer's n + 16 entries
    const __amdgpu_buffer_rsrc_t rows_out = __builtin_amdgcn_make_buffer_rsrc(a.rows, (short)0, n * 8, 0x00020000);
    // the same words read ahead through a range-checked descriptor: a word
    // past column n - 1 reads as 0 (its tag never matches), so the offset
    // needs no clamp
    const __amdgpu_buffer_rsrc_t rows_in = rows_out;
    int S = 0;
    int failed = 0;
    const int s_target = TRACE ? *a.score : 0;
    unsigned long long key = ~0ull;          // first cell holding s_target (TRACE)
    for (int b = wave_id; b < a.nb && !failed; b += a.waves) {
        const int rb = b * kWave + lane;
        // the band's profile in this wave's LDS region: entry group (code c,
        // lane g) at lds0 + (c * 64 + g) * PS, so lanes reading the same code
        // read consecutive addresses; the profile reads of the sweep then wait
        // on the LDS counter, never behind the coherent loads and stores of
        // the handoff words.  A lane reads only the entries it wrote itself,
        // and a wave's LDS accesses complete in order, so no barrier is needed
        // (the waves of a workgroup run different numbers of bands).
        {
            const uint8_t* __restrict__ src = a.prof + (size_t)min(rb, a.nbr) * BS;
            for (int c = 0; c < kCodes; ++c) {
                uint32_t v[NW];
                flow_ldprof<NW>(v, src + (uint32_t)c * CS);
                uint32_t* d = reinterpret_cast<uint32_t*>(sw_lds + lds0 + ((uint32_t)c * kWave + lane) * PS);
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    d[i] = v[i];
            }
        }
        // the rest of the band, compiled twice: the first band (no band
        // above) and every other one, whose steps then carry no per-step test
        // of that and no selects between the border and the band above
        auto run_band = [&](auto top) {
            constexpr bool has_top = decltype(top)::value;
            const bool put = b < a.nb - 1;
            // inside the matrix every lane's column is in [0, n): the band's last
            // lane stores column t - 63 at byte t * 8 + sbase, the other lanes past
            // the descriptor's range (dropped)
            const int sbase = (tail && put) ? -(kWave - 1) * 8 : (1 << 30);
            const uint32_t want = (uint32_t)b;                 // the band above wrote tag (b - 1) + 1
            const uint32_t wtag = (uint32_t)(b + 1) << 16;     // this band's tag, in the word's high half
            int Y[R], E[R];
#pragma unroll
            for (int r = 0; r < R; ++r) { Y[r] = -go; E[r] = 0; }
            int ydiag = -go, ybot = -go, fbot = 0;
            // the head's words of the first 16 columns; then each word is loaded 16
            // steps before its use, into the ring slot the step just consumed
            unsigned long long ring[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                ring[u] = flow_word(a.rows, min(u, n - 1));
            // subject codes of the current and the next 16-column block; the block
            // after is loaded a block ahead, so its wait never falls behind the
            // handoff words' loads and stores just issued
            uint4 rv = resp[0];
            uint4 rvn = resp[min(1, nblk - 1)];
            int code = head ? (int)(rv.x & 0xffu) : kPad;
            uint32_t pv[NW];
            flow_ldlds<NW, PS>(pv, lds0 + ((uint32_t)code * kWave + lane) * PS);

            auto sweep = [&](auto edge, int t0) {
                constexpr bool EDGE = decltype(edge)::value;
                // From kFlowBlockwiseRows rows per lane on, while every column of the block is
                // inside the matrix, the tags of its 16 words (slot u holds
                // column t0 + u) are checked at once: the band above writes
                // tag b, older words carry smaller tags, so the block is ready
                // when the least tag is b.  A stale word was read ahead before
                // the band above wrote it, and so were the words after it: the
                // band then waits until the band above is kFlowSlack columns
                // past the block's last word and reads all 16 again, falling
                // behind the band above in one wait rather than one poll per
                // step.  The check waits for the block's last read-ahead loads,
                // which shorter steps (fewer rows) do not hide: there each
                // step checks its own word.
                const bool whole = BLOCKWISE && (!EDGE || t0 + 15 < n);
                auto ready = [&]() {
                    uint32_t least = (uint32_t)(ring[0] >> 32);
#pragma unroll
                    for (int u = 1; u < 16; u += 2)
                        least = min3_u32(least, (uint32_t)(ring[u] >> 32),
                                         (uint32_t)(ring[u + 1 < 16 ? u + 1 : u] >> 32));
                    return __builtin_amdgcn_readfirstlane(least) >= (want << 16);
                };
                if (has_top && whole && __builtin_expect(!ready(), 0)) {
                    do {
                        flow_wait(a, min(t0 + 15 + kFlowSlack, n - 1), want, &failed);
#pragma unroll
                        for (int u = 0; u < 16; ++u) {
                            const u32x2 rw = __builtin_amdgcn_raw_buffer_load_b64(rows_in, (t0 + u) * 8, 0, kStoreSc1);
                            ring[u] = ((unsigned long long)rw[1] << 32) | rw[0];
                        }
                    } while (!failed && !ready());
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int t = t0 + u;
                    unsigned long long word = ring[u];
                    if (has_top && !whole && (!EDGE || t < n) &&
                        __builtin_amdgcn_readfirstlane((uint32_t)(word >> 48)) != want)
                        word = flow_wait(a, t, want, &failed);
                    const int yh = (int)(word & 0xffffffu) - go;
                    const int fh = (int)((word >> 24) & 0xffffffu) - go;
                    // the word of column t + 16, into the slot just consumed (an
                    // agent-scope coherent read, as flow_word)
                    const u32x2 nw = __builtin_amdgcn_raw_buffer_load_b64(rows_in, (t + 16) * 8, 0, kStoreSc1);
                    ring[u] = ((unsigned long long)nw[1] << 32) | nw[0];
                    // shifts with the whole wave active, pinned so that none is
                    // folded into a select under a partial execution mask
                    int cd = shr1(code), yd = shr1(ybot), fd = shr1(fbot);
                    pin(cd);
                    pin(yd);
                    pin(fd);
                    const uint32_t nxt = u < 15 ? comp(rv, (u + 1) >> 2) >> (8 * ((u + 1) & 3)) : rvn.x;
                    const int cnext = head ? (int)(nxt & 0xffu) : cd;
                    uint32_t pvn[NW];
                    flow_ldlds<NW, PS>(pvn, lds0 + ((uint32_t)cnext * kWave + lane) * PS);
                    const int j = t - lane;                    // this lane's column
                    if (!EDGE || (j >= 0 && j < n)) {
                        const int yt = head ? (has_top ? yh : -go) : yd;
                        const int ft = head ? (has_top ? fh : 0) : fd;
                        int dg = ydiag;
                        ydiag = yt;
                        int hup = yt, F = ft;
                        int hprev = 0;
                        uint32_t word = 0;
                        int hs[TRACE ? R : 1];            // the column's H (trace)
                        int cmax = 0;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int tt = dg + flow_entry<ES>(pv, r);      // H[i-1][j-1] + s
                            const int eo = E[r] - ge;
                            const int e = imax3(eo, Y[r], 0);               // E (clamped at 0)
                            const int fo = F - ge;
                            F = max(fo, hup);                               // F
                            const int h = imax3(tt, e, F);                  // H
                            if constexpr (TRACE) {
                                uint32_t cc = h == 0 ? 0u : (h == tt ? 1u : (h == e ? 2u : 3u));
                                cc |= (Y[r] >= eo ? 4u : 0u) | (hup >= fo ? 8u : 0u);
                                word |= cc << (4 * r);
                                hs[r] = h;
                                if (r & 1)
                                    cmax = max3_i32(cmax, hprev, h);
                                else
                                    hprev = h;
                            } else if (r & 1) {
                                S = max3_i32(S, hprev, h);
                            } else {
                                hprev = h;
                            }
                            if (!TRACE && (R & 1) && r == R - 1)
                                S = max(S, h);
                            dg = Y[r];
                            hup = h - go;
                            Y[r] = hup;
                            E[r] = e;
                        }
                        ybot = hup;
                        fbot = F;
                        if constexpr (TRACE) {
                            if constexpr (R == 8)
                                a.dir[(int64_t)j * a.dir_stride + rb] = word;
                            else                     // rows 4 (rb & 1) .. 4 (rb & 1) + 3 of block rb / 2
                                reinterpret_cast<uint16_t*>(a.dir)[(int64_t)j * 2 * a.dir_stride + rb] =
                                    (uint16_t)word;
                            // no H exceeds the pair's score: only a column whose
                            // maximum is the score holds the end cell
                            if (cmax == s_target) {
                                uint32_t hits = 0;
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    hits |= (hs[r] == s_target ? 1u : 0u) << r;
                                const int64_t row = (int64_t)rb * R + __builtin_ctz(hits);
                                const unsigned long long k2 = ((unsigned long long)j << 32) | (unsigned long long)row;
                                if (row < a.m && k2 < key)
                                    key = k2;
                            }
                        }
                    }
                    const uint32_t yv = (uint32_t)(ybot + go), fv = (uint32_t)(fbot + go);
                    const u32x2 v = {(yv & 0xffffffu) | (fv << 24), ((fv >> 8) & 0xffffu) | wtag};
                    if constexpr (EDGE) {
                        const bool st = tail && put && !failed && j >= 0 && j < n;
                        __builtin_amdgcn_raw_buffer_store_b64(v, rows_out, st ? j * 8 : n * 8, 0, kStoreSc1);
                    } else {
                        __builtin_amdgcn_raw_buffer_store_b64(v, rows_out, t * 8 + sbase, 0, kStoreSc1);
                    }
                    code = cnext;
#pragma unroll
                    for (int i = 0; i < NW; ++i)
                        pv[i] = pvn[i];
                }
            };
            // blocks where some lane is outside [0, n) (the pipeline's fill and
            // drain) run a copy of the sweep with a per-lane predicate; the blocks
            // between run without, in a loop of their own
            const int fast_lo = kWave, fast_hi = max(kWave, n & ~15);     // [fast_lo, fast_hi): every lane inside
            auto block = [&](auto edge, int t0) {
                const uint4 ahead = resp[min((t0 >> 4) + 2, nblk - 1)];
                sweep(edge, t0);
                rv = rvn;
                rvn = ahead;
            };
            for (int t0 = 0; t0 < min(fast_lo, nsteps16) && !failed; t0 += 16)
                block(std::integral_constant<bool, true>{}, t0);
            for (int t0 = fast_lo; t0 < fast_hi && !failed; t0 += 16)
                block(std::integral_constant<bool, false>{}, t0);
            for (int t0 = max(fast_lo, fast_hi); t0 < nsteps16 && !failed; t0 += 16)
                block(std::integral_constant<bool, true>{}, t0);
        };
        if (b > 0)
            run_band(std::integral_constant<bool, true>{});
        else
            run_band(std::integral_constant<bool, false>{});
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
    for (int k = 32; k >= 1; k >>= 1)
        S = max(S, __shfl_xor(S, k));
    if (lane == 0 && S > 0)
        atomicMax(a.score, S);
}

// Up to 6 rows per lane the state fits 128 registers (workgroups of up to 16
// waves, four per SIMD); more rows take up to 256 (up to 8 waves, two per
// SIMD).  Wave w of workgroup g is wave group * W + w of the launch, group the
// number of g counted XCD by XCD (below).  TRACE: the direction-code pass.
template <int R, int ES, bool TRACE = false>
__global__ void __launch_bounds__(R <= 6 ? 1024 : 512) __attribute__((amdgpu_waves_per_eu(R <= 6 ? 4 : 2)))
k_pair_flow(FlowArgs a)
{
    const int wpg = (int)(blockDim.x >> 6);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // Workgroups go to the device's 8 XCDs in turn (workgroup g to XCD g mod
    // 8), each XCD with an L2 of its own.  Number them XCD by XCD, so that a
    // band and the one below it share an L2 except where one XCD's share of
    // the workgroups ends; the numbering is a permutation of the grid.
    const int G = (int)gridDim.x, g = (int)blockIdx.x;
    const int x = g & (kXcds - 1), per = G / kXcds, extra = G % kXcds;
    const int group = x * per + min(x, extra) + g / kXcds;
    pair_flow<R, ES, TRACE>(a, group * wpg + w, (int)(threadIdx.x & 63), (uint32_t)(w * flow_lds_bytes(R, ES)));
}

// Clear the handoff words and the status word before a flow pass.
__global__ void __launch_bounds__(256) k_flow_clear(unsigned long long* rows, int64_t count, int32_t* status)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0)
        *status = 0;
    for (int64_t i = t; i < count; i += (int64_t)gridDim.x * blockDim.x)
        rows[i] = 0ull;
}

// A timed-out wait makes the score meaningless: report -1.
__global__ void k_pair_flow_finish(const int32_t* status, int32_t* score)
{
    if (*status)
        *score = -1;
}

// The kernel of (rows, elem), or of the direction-code pass (4 or 8 rows per
// lane); null for a shape it is not built for.
static const void* flow_kernel(int rows, int elem, bool trace = false)
{
    if (trace) {
        switch (rows * 4 + elem) {
        case 4 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<4, 1, true>);
        case 4 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<4, 2, true>);
        case 8 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<8, 1, true>);
        case 8 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<8, 2, true>);
        default: return nullptr;
        }
    }
    switch (rows * 4 + elem) {
    case 4 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<4, 1>);
    case 4 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<4, 2>);
    case 6 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<6, 1>);
    case 6 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<6, 2>);
    case 8 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<8, 1>);
    case 8 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<8, 2>);
    case 10 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<10, 1>);
    case 10 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<10, 2>);
    case 12 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<12, 1>);
    case 12 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<12, 2>);
    case 16 * 4 + 1: return reinterpret_cast<const void*>(&k_pair_flow<16, 1>);
    case 16 * 4 + 2: return reinterpret_cast<const void*>(&k_pair_flow<16, 2>);
    default: return nullptr;
    }
}

hipError_t launch_pair_flow(const FlowArgs& a, int rows, int elem, int wpg, int grid, int lds, hipStream_t st)
{
    const void* k = flow_kernel(rows, elem, a.dir != nullptr);
    if (!k || wpg < 1 || wpg > (rows <= 6 ? 16 : 8) || grid < 1 || (int64_t)grid * wpg != a.waves ||
        lds < flow_group_lds(rows, elem, wpg))
        return hipErrorInvalidValue;
    const int64_t clear = (int64_t)a.n + 16;
    hipLaunchKernelGGL(k_flow_clear, dim3((unsigned)std::min<int64_t>((clear + 255) / 256, 1024)), dim3(256), 0,
                       st, a.rows, clear, a.status);
    FlowArgs arg = a;
    void* args[] = {&arg};
    const hipError_t e = hipLaunchKernel(k, dim3((unsigned)grid), dim3((unsigned)(64 * wpg)), args, (size_t)lds, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_pair_flow_finish, dim3(1), dim3(1), 0, st, a.status, a.score);
    return hipGetLastError();
}

int flow_occupancy(int rows, int elem, int wpg, int lds, bool trace)
{
    const void* k = flow_kernel(rows, elem, trace);
    int n = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * wpg, (size_t)lds) != hipSuccess)
        return 0;
    return n;
}

}  // namespace swdb
