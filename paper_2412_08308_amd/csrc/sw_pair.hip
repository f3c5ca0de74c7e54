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
// into colbuf.
#include "sw_device.h"

namespace swdb {

// TRACE (8 rows per lane only): also write each cell's 4-bit direction code
// (PairArgs::dir) and find the first cell, in column-major order, whose H
// equals the score already computed by a plain pass (PairArgs::end_key).  The
// codes follow the traceback rules: the diagonal before E before F, a gap
// opened from H rather than extended when both give its value.
template <int R, int ES, bool TRACE = false>
__device__ __forceinline__ void pair_tile(const PairArgs& a, int lane)
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
    if (has_left)
        ydiag = head ? (b > 0 ? a.corner[b * 3 + c % 3] : -go) : side[-1].x;
    int ybot = -go, fbot = 0;
    int S = 0;
    const int s_target = TRACE ? *a.score : 0;
    unsigned long long key = ~0ull;          // first cell holding s_target (TRACE)

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
                    uint32_t word = 0, hits = 0;
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
                            hits |= (h == s_target ? 1u : 0u) << r;
                        }
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
                    if (put_bottom)
                        top[j] = make_int2(ybot, fbot);
                    if constexpr (TRACE) {
                        const int64_t col = c0 + j;
                        if (valid) {
                            a.dir[col * a.dir_stride + rb] = word;
                            const int64_t row = row0 + (hits ? __builtin_ctz(hits) : 0);
                            if (hits && key == ~0ull && col < a.n && row < a.m)
                                key = ((unsigned long long)col << 32) | (unsigned long long)row;
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
    // tile maximum into the pair's score
    S = valid ? S : 0;
    for (int k = 32; k >= 1; k >>= 1)
        S = max(S, __shfl_xor(S, k));
    if (lane == 0 && S > 0)
        atomicMax(a.score, S);
}

template <int R, int ES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_pair_diag(PairArgs a)
{
    pair_tile<R, ES>(a, threadIdx.x & 63);
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
// codes -- the diagonal emits a residue pair and stops when its predecessor
// holds H = 0 or lies on the border, E emits a subject residue against a gap,
// F a query residue against a gap, each returning to H where the gap was
// opened -- then reverse the operations into begin-to-end order.  One
// wavefront: the codes of a window of 64 columns x 128 rows around the walk
// sit in LDS (each lane loads one column), every lane runs the same walk on
// them (uniform control flow; lane 0 writes the operations), and the wave
// reloads the window when the walk leaves it.
constexpr int kWinCols = 64, kWinWords = 16;   // 16 words of 8 rows = 128 rows

__global__ void __launch_bounds__(64) k_traceback(const uint32_t* __restrict__ dir, int64_t stride,
                                                  const unsigned long long* __restrict__ end_key,
                                                  const int32_t* __restrict__ score, char* __restrict__ ops,
                                                  int64_t cap, AlignOut* out)
{
    __shared__ uint32_t win[kWinCols][kWinWords];
    const int lane = threadIdx.x;
    AlignOut r{};
    r.score = *score;
    const unsigned long long key = *end_key;
    int64_t n_ops = 0;
    if (r.score > 0 && key != ~0ull) {
        int64_t j = (int64_t)(key >> 32) + 1, i = (int64_t)(key & 0xffffffffull) + 1;   // 1-based
        r.q_end = (int32_t)i;
        r.s_end = (int32_t)j;
        int64_t c0 = -1, w0 = 0;     // window: columns c0..c0+63, words w0..w0+15 (0-based)
        // code of 1-based cell (ii, jj), reloading the window around it if needed
        auto code = [&](int64_t ii, int64_t jj) -> uint32_t {
            const int64_t col = jj - 1, row = ii - 1;
            if (c0 < 0 || col < c0 || col >= c0 + kWinCols || (row >> 3) < w0 || (row >> 3) >= w0 + kWinWords) {
                __syncthreads();
                c0 = col - (kWinCols - 1) > 0 ? col - (kWinCols - 1) : 0;
                w0 = (row >> 3) - (kWinWords - 4) > 0 ? (row >> 3) - (kWinWords - 4) : 0;
                const int64_t cc = c0 + lane;
                if (cc <= col) {
#pragma unroll
                    for (int k = 0; k < kWinWords; ++k)
                        win[lane][k] = (w0 + k < stride) ? dir[cc * stride + w0 + k] : 0u;
                }
                __syncthreads();
            }
            const uint32_t w = win[col - c0][(row >> 3) - w0];
            return (w >> (4 * (row & 7))) & 15u;
        };
        int state = 0;
        bool ok = false;
        while (n_ops < cap && i >= 1 && j >= 1) {
            const uint32_t c = code(i, j);
            char op = 0;
            if (state == 0) {
                const uint32_t src = c & 3u;
                if (src == 1u) {
                    op = 'M';
                    const bool stop = i == 1 || j == 1 || (code(i - 1, j - 1) & 3u) == 0u;
                    if (lane == 0)
                        ops[n_ops] = op;
                    ++n_ops;
                    if (stop) {
                        ok = true;
                        break;
                    }
                    --i;
                    --j;
                    continue;
                } else if (src == 2u) {
                    state = 1;
                } else if (src == 3u) {
                    state = 2;
                } else {
                    break;                        // H = 0 on the path: inconsistent codes
                }
                continue;
            }
            if (state == 1) {
                op = 'D';
                if (c & 4u)
                    state = 0;
                --j;
            } else {
                op = 'I';
                if (c & 8u)
                    state = 0;
                --i;
            }
            if (lane == 0)
                ops[n_ops] = op;
            ++n_ops;
        }
        if (ok) {
            r.q_begin = (int32_t)i;
            r.s_begin = (int32_t)j;
            __syncthreads();                      // the walk's writes before the reversal
            for (int64_t x = lane, y = n_ops - 1 - lane; x < y; x += 64, y -= 64) {
                const char t = ops[x];
                ops[x] = ops[y];
                ops[y] = t;
            }
        } else {
            n_ops = -1;                           // reported as an error by the host
        }
    }
    r.n_ops = (int32_t)n_ops;
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

hipError_t launch_traceback(const uint32_t* dir, int64_t dir_stride, const unsigned long long* end_key,
                            const int32_t* score, char* ops, int64_t cap, AlignOut* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_traceback, dim3(1), dim3(kWinCols), 0, st, dir, dir_stride, end_key, score, ops, cap, out);
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
void launch_pair_rows(const PairArgs& a, int elem, int blocks, hipStream_t st)
{
    if (elem == 1)
        hipLaunchKernelGGL((k_pair_diag<R, 1>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_pair_diag<R, 2>), dim3(blocks), dim3(256), 0, st, a);
}

hipError_t launch_pair_diag(const PairArgs& a, int rows, int elem, hipStream_t st)
{
    const int groups_per_wave = kWave / a.K;
    const int waves = (a.ntiles + groups_per_wave - 1) / groups_per_wave;
    const int blocks = (waves + 3) / 4;
    switch (rows) {
    case 8: launch_pair_rows<8>(a, elem, blocks, st); break;
    case 16: launch_pair_rows<16>(a, elem, blocks, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swdb
