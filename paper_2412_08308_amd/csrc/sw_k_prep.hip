// Per-search and per-database preparation kernels, and launch dispatch.
#include "sw_internal.h"

namespace swdb {

hipError_t launch_search_i32p8(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st);
hipError_t launch_search_i32p16(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st);
hipError_t launch_search_i16(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st);
hipError_t launch_search_i16p8(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st);
int occupancy_i32p8(int waves, int lds);
int occupancy_i32p16(int waves, int lds);
int occupancy_i16(int waves, int lds);
int occupancy_i16p8(int waves, int lds);

LaunchInfo variant_info(Variant v)
{
    switch (v) {
    case kI32_R32_P8: return {32, 1, 1};
    case kI32_R32_P16: return {32, 2, 1};
    case kI16: return {kI16Rows, 2, 2};
    case kI16_P8: return {kI16Rows, 1, 2};
    }
    return {0, 0, 0};
}

// Query profiles (the substitution term of the H equation, looked up per query
// row and subject residue code): entry (row block rb, code c, row r) =
// SM[Q[rb*R + r]][c] + Go for rows inside the query and codes < 32, the pad
// value elsewhere (the most negative entry, or 0 for the zero-extended 8-bit
// profile of the packed lanes: a pad cell then adds -Go to its diagonal, so it
// never exceeds the real cells it derives from); row block nbr is entirely
// padding.
// A query residue code >= 32 sets *a.bad (when given) and is read modulo 32,
// so that every profile read stays inside the matrix.
template <typename PE>
__global__ void __launch_bounds__(256) k_profile(ProfileArgs a, int R)
{
    const int q = blockIdx.y;
    const QueryDesc qd = a.qd[q];
    const int entries = (qd.nbr + 1) * kCodes * R;
    const int cse = code_stride(R, (int)sizeof(PE)) / (int)sizeof(PE);   // code stride in entries
    PE* __restrict__ out = reinterpret_cast<PE*>(a.prof + qd.prof_off);
    const uint8_t* __restrict__ qs = a.queries + a.q_off[q];
    const PE padv = (PE)a.pad;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < entries; e += gridDim.x * blockDim.x) {
        const int r = e % R;
        const int c = (e / R) % kCodes;
        const int rb = e / (R * kCodes);
        const int row = rb * R + r;
        PE v = padv;
        if (row < qd.m && c < kAlpha) {
            const int raw = qs[row];
            if (c == 0 && raw >= kAlpha && a.bad)
                atomicOr(a.bad, 1);
            const int qc = raw & (kAlpha - 1);
            v = (PE)(a.sm.v[qc * kAlpha + c] + a.go);
        }
        out[((int64_t)rb * kCodes + c) * cse + r] = v;
    }
}

// Lane interleaving of a length-sorted database.  Thread t writes the 16 bytes
// of (chunk c, column block b, lane l): columns 16b..16b+15 of sorted subject
// 64c + l, pad code past its end.  A code >= 32 sets *bad.
__global__ void __launch_bounds__(256) k_interleave(const uint8_t* __restrict__ src, const int64_t* __restrict__ src_off,
                                                    const int32_t* __restrict__ perm, const int32_t* __restrict__ slen,
                                                    const int64_t* __restrict__ chunk_off, int32_t nseq,
                                                    int64_t total, const int64_t* __restrict__ block_prefix,
                                                    int32_t nchunks, uint8_t* __restrict__ dst, int32_t* bad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total)
        return;
    const int64_t gb = t >> 6;
    const int l = (int)(t & 63);
    int lo = 0, hi = nchunks - 1;               // last chunk whose first block <= gb
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block_prefix[mid] <= gb) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const int64_t b = gb - block_prefix[c];
    const int64_t s = (int64_t)c * 64 + l;
    uint32_t o[4] = {0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u};
    if (s < nseq) {
        const int len = slen[s];
        const uint8_t* p = src + src_off[perm[s]];
        int badv = 0;
        for (int k = 0; k < 16; ++k) {
            const int64_t col = b * 16 + k;
            if (col < len) {
                const uint32_t x = p[col];
                badv |= x >= (uint32_t)kAlpha;
                o[k >> 2] = (o[k >> 2] & ~(0xffu << (8 * (k & 3)))) | (x << (8 * (k & 3)));
            }
        }
        if (badv)
            atomicOr(bad, 1);
    }
    *reinterpret_cast<uint4*>(dst + chunk_off[c] + (b * 64 + l) * 16) = make_uint4(o[0], o[1], o[2], o[3]);
}

hipError_t launch_profile(const ProfileArgs& a, int rows, int elem, int max_entries, hipStream_t st)
{
    if (a.nq <= 0)
        return hipSuccess;
    int bx = (max_entries + 255) / 256;
    if (bx < 1) bx = 1;
    if (bx > 2048) bx = 2048;
    dim3 grid(bx, a.nq);
    if (elem == 1)
        hipLaunchKernelGGL(k_profile<int8_t>, grid, dim3(256), 0, st, a, rows);
    else
        hipLaunchKernelGGL(k_profile<int16_t>, grid, dim3(256), 0, st, a, rows);
    return hipGetLastError();
}

hipError_t launch_search(Variant v, const SearchArgs& a, int grid, int waves, int lds_bytes, hipStream_t st)
{
    switch (v) {
    case kI32_R32_P8: return launch_search_i32p8(a, grid, waves, lds_bytes, st);
    case kI32_R32_P16: return launch_search_i32p16(a, grid, waves, lds_bytes, st);
    case kI16: return launch_search_i16(a, grid, waves, lds_bytes, st);
    case kI16_P8: return launch_search_i16p8(a, grid, waves, lds_bytes, st);
    }
    return hipErrorInvalidValue;
}

int search_occupancy(Variant v, int waves, int lds_bytes)
{
    switch (v) {
    case kI32_R32_P8: return occupancy_i32p8(waves, lds_bytes);
    case kI32_R32_P16: return occupancy_i32p16(waves, lds_bytes);
    case kI16: return occupancy_i16(waves, lds_bytes);
    case kI16_P8: return occupancy_i16p8(waves, lds_bytes);
    }
    return 1;
}

hipError_t launch_interleave(const uint8_t* src, const int64_t* src_off, const int32_t* perm,
                             const int32_t* slen, const int64_t* chunk_off, int32_t nseq,
                             int64_t total, const int64_t* block_prefix, int32_t nchunks,
                             uint8_t* dst, int32_t* bad, hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_interleave, dim3((unsigned)blocks), dim3(256), 0, st, src, src_off, perm, slen,
                       chunk_off, nseq, total, block_prefix, nchunks, dst, bad);
    return hipGetLastError();
}

}  // namespace swdb
