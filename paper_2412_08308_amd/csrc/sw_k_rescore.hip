// Exact int32 rescore of the subjects the packed 16-bit search lists: the
// list sort by cost and the pass-pipelined rescore kernel, for both profile
// entry widths of the packed variants (kI16Rows rows; 8-bit entries are
// non-negative, so the int32 reader's sign extension reads them unchanged).
#include "sw_device.h"

namespace swdb {

// ------------------------------------------------------------------ int32 rescore

// Exact int32 rescore of the subjects listed by the 16-bit pass (one list
// entry = query, subject).  A workgroup of W wavefronts takes one entry at a
// time from the list (a queue head in the counters); a subject's query rows
// are split into passes of 64 lanes x R rows, wavefront w sweeps passes w,
// w + W, ..., and the passes run as a pipeline: pass p reads the bottom row
// (Y, F) that pass p - 1 writes to a per-workgroup buffer in the workspace as
// soon as pass p - 1 has published, through a counter in LDS, that the columns
// it needs are written.  The critical path of a long subject is then one pass
// instead of all of them.  Every wait is bounded: after kSpinLimit polls the
// workgroup gives up on the subject, stores -1 (no Smith-Waterman score is
// negative) and counts the subject in the status words, so the kernel always
// drains and the call's status reports the failure.

constexpr uint32_t kSpinLimit = 1u << 24;

// Published progress of a pass: (pass << 32) | columns whose bottom row is
// written.  Monotonic per buffer, so a counter never needs a reset inside a
// subject even when W < passes and buffers are reused.
__device__ __forceinline__ uint64_t progress(int pass, int cols)
{
    return ((uint64_t)(uint32_t)pass << 32) | (uint32_t)cols;
}

// Wait until *p >= need or the workgroup has failed; false on time-out (the
// failure is then recorded for the workgroup).
__device__ __forceinline__ bool wait_progress(uint64_t* p, uint64_t need, int* failed)
{
    for (uint32_t it = 0; it < kSpinLimit; ++it) {
        const uint64_t v = __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (v >= need)
            return true;
        if (__hip_atomic_load(failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return false;
}

// One pass of one subject on one wavefront: lane g owns query row block
// pass*64 + g and runs g columns behind lane 0 (the same cell update and DPP
// hand-down as the int32 search item with 64 lanes per subject).  Reads the
// previous pass's bottom row from `bin`, writes its own to `bout`.  Returns
// the wavefront's largest H, or -1 if a wait timed out.
template <int R, int ES>
__device__ __forceinline__ int rescore_pass(const SearchArgs& a, const QueryDesc& qd, int s, int ncols, int pass,
                                            int P, const int2* __restrict__ bin, int2* __restrict__ bout,
                                            uint64_t* prog_in, uint64_t* prog_out, int* failed, int lane)
{
    constexpr uint32_t CS = code_stride(R, ES);
    constexpr uint32_t BS = kCodes * CS;
    constexpr int NB = R * ES;
    constexpr int NV = (NB + 15) / 16;
    constexpr int K = kWave;

    const bool head = lane == 0;
    const bool tail = lane == K - 1;
    const uint4* __restrict__ resp = reinterpret_cast<const uint4*>(a.res + a.chunk_off[s >> 6]) + (s & 63);
    const int nsteps = (ncols + K - 1 + 3) & ~3;
    const int rb = min(pass * K + lane, qd.nbr);    // row block nbr is all padding
    const uint32_t pbase = (uint32_t)rb * BS;
    const bool rd = pass > 0;
    const bool wr = pass < P - 1;
    const int go = a.go, ge = a.ge;
    const uint8_t* __restrict__ gprof = a.prof + qd.prof_off;

    int Y[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { Y[r] = -go; E[r] = 0; }
    int ydiag = -go, ybot = -go, fbot = 0;
    int S = 0;
    bool ok = true;

    // The profile vector of the next column is loaded one column ahead: lane
    // g's next code is lane g-1's current one (a DPP shift of the current
    // code), the head's is the next residue.
    uint4 rv = (head && 0 < ncols) ? resp[0] : pad16();
    int code = head ? (int)(rv.x & 0xffu) : kPad;
    uint4 pv[NV];
    ldprof<NB, false>(pv, gprof, pbase + (uint32_t)code * CS);
    for (int blk = 0; blk < nsteps; blk += 16) {
        const uint4 rvn = (head && blk + 16 < ncols) ? resp[(blk + 16) * 4] : pad16();
        const int n4 = min(4, (nsteps - blk) >> 2);
#pragma unroll 1
        for (int k4 = 0; k4 < n4; ++k4) {
            const int col0 = blk + 4 * k4;
            if (rd && ok && (col0 & 63) == 0 && col0 < ncols)
                ok = wait_progress(prog_in, progress(pass - 1, min(ncols, col0 + 64)), failed);
            const uint32_t w = rv.x;
            rv = make_uint4(rv.y, rv.z, rv.w, 0u);
            // first residue of the next 4-column group
            const uint32_t wn = k4 < 3 ? rv.x : rvn.x;
            int ringY[4], ringF[4];
            if (rd && col0 < ncols && head) {
                const int4* p4 = reinterpret_cast<const int4*>(bin + col0);
                const int4 v0 = p4[0], v1 = p4[1];
                ringY[0] = v0.x; ringF[0] = v0.y; ringY[1] = v0.z; ringF[1] = v0.w;
                ringY[2] = v1.x; ringF[2] = v1.y; ringY[3] = v1.z; ringF[3] = v1.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) { ringY[k] = -go; ringF[k] = 0; }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int yd = shr1(ybot), fd = shr1(fbot), cd = shr1(code);
                pin(yd);
                pin(fd);
                pin(cd);
                const int yt = head ? ringY[u] : yd;
                const int ft = head ? ringF[u] : fd;
                const int hn = (int)(((u < 3 ? w : wn) >> (8 * ((u + 1) & 3))) & 0xffu);
                const int cn = head ? hn : cd;
                uint4 pn[NV];
                ldprof<NB, false>(pn, gprof, pbase + (uint32_t)cn * CS);

                int dg = ydiag;
                ydiag = yt;
                int hup = yt, F = ft;
                int hprev = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int t = dg + pent<ES>(pv, r);
                    const int e = imax3(E[r] - ge, Y[r], 0);
                    F = max(F - ge, hup);
                    const int h = imax3(t, e, F);
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
                code = cn;
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    pv[i] = pn[i];
                const int j = col0 + u - (K - 1);
                if (wr && tail && j >= 0 && j < ncols)
                    bout[j] = make_int2(ybot, fbot);
            }
            if (wr && ((col0 + 4) & 63) == 0) {
                // columns < col0 + 4 - (K - 1) of this pass's bottom row are written
                const int done = min(ncols, max(0, col0 + 4 - (K - 1)));
                if (tail)
                    __hip_atomic_store(prog_out, progress(pass, done), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        rv = rvn;
    }
    if (wr && tail)
        __hip_atomic_store(prog_out, progress(pass, ncols), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (int off = 32; off > 0; off >>= 1)
        S = max(S, __shfl_xor(S, off));
    return ok ? S : -1;
}

template <int R, int ES>
__global__ void __launch_bounds__(64 * kRescoreMaxWaves) __attribute__((amdgpu_waves_per_eu(ES == 1 ? 4 : 3)))
k_rescore(SearchArgs a)
{
    __shared__ uint64_t prog[kRescoreMaxWaves];
    __shared__ int2 cur;
    __shared__ int smax;
    __shared__ int failed;
    const int W = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    int2* __restrict__ bufs = a.bnd + (int64_t)blockIdx.x * W * a.slot_elems;
    const int cnt = min(a.counters[1], a.flag_cap);
    if ((int)blockIdx.x >= cnt)
        return;                                // the first cnt workgroups take every entry
    for (;;) {
        __syncthreads();                       // the previous subject is finished by every wavefront
        if (threadIdx.x == 0) {
            const int f = atomicAdd(&a.counters[2], 1);
            cur = f < cnt ? a.flags[f] : make_int2(-1, -1);
            smax = 0;
            failed = 0;
        }
        if (threadIdx.x < W)
            prog[threadIdx.x] = 0;
        __syncthreads();
        const int2 e = cur;
        if (e.x < 0)
            break;
        if (e.x >= a.nq || e.y < 0 || e.y >= a.nseq) {
            if (threadIdx.x == 0)              // not an entry of this launch
                atomicAdd(&a.status[kStatusBadItems], 1);
            continue;
        }
        const QueryDesc qd = a.qd[e.x];
        const int ncols = (a.slen[e.y] + 15) & ~15;
        if ((int64_t)ncols > a.slot_elems) {   // buffers sized below the subject: no score
            if (threadIdx.x == 0) {
                a.scores[(int64_t)qd.out_row * a.out_stride + a.perm[e.y]] = -1;
                atomicAdd(&a.status[kStatusRescoreFailed], 1);
            }
            continue;
        }
        const int P = (qd.nbr + kWave - 1) / kWave;
        int S = 0;
        for (int p = wave; p < P; p += W) {
            const int b = p % W, bp = (p + W - 1) % W;
            const int Sp = rescore_pass<R, ES>(a, qd, e.y, ncols, p, P, bufs + (int64_t)bp * a.slot_elems,
                                               bufs + (int64_t)b * a.slot_elems, &prog[bp], &prog[b], &failed, lane);
            S = (S < 0 || Sp < 0) ? -1 : max(S, Sp);
        }
        if (lane == 0)
            atomicMax(&smax, S < 0 ? INT_MAX : S);
        __syncthreads();
        if (threadIdx.x == 0) {
            a.scores[(int64_t)qd.out_row * a.out_stride + a.perm[e.y]] = smax == INT_MAX ? -1 : smax;
            if (smax == INT_MAX)
                atomicAdd(&a.status[kStatusRescoreFailed], 1);
        }
    }
}

// Order the overflow list (query, subject) by rescore cost, largest first, so
// that the rescore workgroups, which take entries in list order, start the
// longest subjects first and the shortest fill the tail.  One workgroup; a
// bitonic sort in LDS of (cost, position) keys, then an in-place permutation
// of the list.  Lists longer than kFlagSortCap are left in append order (only
// the balance of the rescore depends on the order).
__global__ void __launch_bounds__(1024) k_flag_sort(SearchArgs a)
{
    __shared__ uint64_t key[kFlagSortCap];
    const int cnt = min(a.counters[1], a.flag_cap);
    if (threadIdx.x == 0 && cnt > 0)
        atomicAdd(&a.status[kStatusFlagged], cnt);
    if (cnt <= 1 || cnt > kFlagSortCap)
        return;
    int n = 1;
    while (n < cnt)
        n <<= 1;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        float cost = 0.f;
        if (i < cnt) {
            const int2 e = a.flags[i];
            if (e.x >= 0 && e.x < a.nq && e.y >= 0 && e.y < a.nseq)
                cost = (float)a.qd[e.x].nbr * (float)a.slen[e.y] + 1.f;
        }
        // a non-negative float orders like its bit pattern
        key[i] = ((uint64_t)__float_as_uint(cost) << 32) | (uint32_t)i;
    }
    __syncthreads();
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t x = key[i], y = key[l];
                    // descending runs where (i & k) == 0, so the final order is descending
                    if (((i & k) == 0) ? x < y : x > y) {
                        key[i] = y;
                        key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    // gather every thread's new entries before any is overwritten
    constexpr int kPer = kFlagSortCap / 1024;
    int2 v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int i = threadIdx.x + t * blockDim.x;
        if (i < cnt)
            v[t] = a.flags[(uint32_t)key[i]];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int i = threadIdx.x + t * blockDim.x;
        if (i < cnt)
            a.flags[i] = v[t];
    }
}

hipError_t launch_flag_sort(const SearchArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_flag_sort, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_rescore(Variant v, const SearchArgs& a, int grid, int waves, hipStream_t st)
{
    if (v == kI16)
        return launch_kernel(k_rescore<kI16Rows, 2>, grid, waves, 0, st, a);
    if (v == kI16_P8)
        return launch_kernel(k_rescore<kI16Rows, 1>, grid, waves, 0, st, a);
    return hipErrorInvalidValue;   // int32 variants never flag subjects
}

}  // namespace swdb
