// Not part of the library.  Compiled only to AMD assembly by isa_count.py:
// every hot-loop variant of the search, instantiated alone in a kernel with
// the same attributes as the persistent search kernels, so that its innermost
// loop (four subject columns x R query rows) can be counted instruction by
// instruction; and the hot loop of an 8-bit lane form that the library does
// not build (isa_i8x4), counted to compare it with the packed 16-bit lanes.
#include "sw_device.h"
#include "sw_swar8.h"

namespace swdb {

// Four subjects per lane in unsigned 8-bit lanes (the step below the packed
// 16-bit lanes), one pass of R query rows, 8-bit profile entries s + bias
// staged in LDS (bias = -(smallest score), passed in nq): the hot loop an
// 8-bit inter-task kernel would run, built only for its instruction count.
// Each subject column reads four profile rows (one per subject's residue
// code) and transposes their bytes (two byte permutes per row); per cell,
// with byte-wise saturation at 0 and 255:
//   t = (Hdiag + (s + bias)) - bias,  E = max(E - Ge, Y),  F = max(F - Ge, Yup),
//   H = max(t, E, F),  Y = H - Go (shared by the next column's E and the next
//   row's F),  S = max(S, H).
// Subject codes: one 32-bit word per column per lane (four subjects' codes),
// four columns per 16-byte load.
template <int R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) isa_i8x4(SearchArgs a)
{
    static_assert(R % 4 == 0, "rows in groups of four (byte transposes)");
    constexpr uint32_t CS = code_stride(R, 1);
    const int lane = threadIdx.x & 63;
    const Item it = a.items[blockIdx.x];
    const uint4* __restrict__ cw4 = reinterpret_cast<const uint4*>(a.res + a.chunk_off[blockIdx.x]) + lane;
    const uint32_t go = (uint32_t)a.go * 0x01010101u, ge = (uint32_t)a.ge * 0x01010101u;
    const uint32_t bias = (uint32_t)a.nq * 0x01010101u;
    uint32_t H[R], Y[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = 0; Y[r] = 0; E[r] = 0; }
    uint32_t S = 0;
    for (int j = 0; j < it.ncols; j += 4) {
        const uint4 cw = cw4[(int64_t)(j >> 2) * kWave];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t cc = comp(cw, c);
            uint4 pr[4][(R + 15) / 16];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                ldprof<R, true>(pr[k], nullptr, ((cc >> (8 * k)) & 0xffu) * CS);
            uint32_t hdiag = 0, yup = 0, f = 0;     // top border (one pass)
#pragma unroll
            for (int r4 = 0; r4 < R; r4 += 4) {
                // rows r4..r4+3 of the four profile rows: a 4x4 byte transpose
                const uint32_t w0 = comp(pr[0][r4 >> 4], (r4 >> 2) & 3), w1 = comp(pr[1][r4 >> 4], (r4 >> 2) & 3);
                const uint32_t w2 = comp(pr[2][r4 >> 4], (r4 >> 2) & 3), w3 = comp(pr[3][r4 >> 4], (r4 >> 2) & 3);
                const uint32_t a0 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);
                const uint32_t a1 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);
                const uint32_t b0 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
                const uint32_t b1 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
                const uint32_t prof[4] = {__builtin_amdgcn_perm(b0, a0, 0x05040100u),
                                          __builtin_amdgcn_perm(b0, a0, 0x07060302u),
                                          __builtin_amdgcn_perm(b1, a1, 0x05040100u),
                                          __builtin_amdgcn_perm(b1, a1, 0x07060302u)};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r4 + q;
                    const uint32_t t = swar8_subs(swar8_adds(hdiag, prof[q]), bias);
                    const uint32_t e = swar8_max(swar8_subs(E[r], ge), Y[r]);
                    f = swar8_max(swar8_subs(f, ge), yup);
                    const uint32_t h = swar8_max(swar8_max(t, e), f);
                    hdiag = H[r];
                    H[r] = h;
                    yup = swar8_subs(h, go);
                    Y[r] = yup;
                    E[r] = e;
                    S = swar8_max(S, h);
                    pin(S);
                }
            }
        }
    }
    a.scores[(int64_t)blockIdx.x * kWave + lane] = (int)S;
}

template __global__ void isa_i8x4<16>(SearchArgs);

template <int R, int ES, bool L, bool M>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) isa_i32(SearchArgs a)
{
    const Item it = a.items[blockIdx.x];
    const QueryDesc qd = a.qd[0];
    item_i32<R, ES, L, M>(a, it, qd, a.bnd + (int64_t)blockIdx.x * a.slot_elems, threadIdx.x & 63);
}

template <int R, int ES, bool L, bool M>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) isa_i16(SearchArgs a)
{
    const Item it = a.items[blockIdx.x];
    const QueryDesc qd = a.qd[0];
    item_i16<R, ES, L, M>(a, it, qd, a.bnd + (int64_t)blockIdx.x * a.slot_elems, threadIdx.x & 63);
}

template <int R, int ES, bool L>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) isa_i16_self(SearchArgs a)
{
    const Item it = a.items[blockIdx.x];
    const QueryDesc qd = a.qd[0];
    item_i16_self<R, ES, L>(a, it, qd, a.bnd + (int64_t)blockIdx.x * a.slot_elems, threadIdx.x & 63);
}

template __global__ void isa_i32<32, 1, true, false>(SearchArgs);
template __global__ void isa_i32<32, 1, true, true>(SearchArgs);
template __global__ void isa_i32<32, 1, false, false>(SearchArgs);
template __global__ void isa_i32<32, 1, false, true>(SearchArgs);
template __global__ void isa_i32<32, 2, true, false>(SearchArgs);
template __global__ void isa_i32<32, 2, false, false>(SearchArgs);
template __global__ void isa_i16<24, 2, true, false>(SearchArgs);
template __global__ void isa_i16<24, 2, true, true>(SearchArgs);
template __global__ void isa_i16<24, 2, false, false>(SearchArgs);
template __global__ void isa_i16<24, 2, false, true>(SearchArgs);
template __global__ void isa_i16<24, 1, true, false>(SearchArgs);
template __global__ void isa_i16<24, 1, true, true>(SearchArgs);
template __global__ void isa_i16<24, 1, false, false>(SearchArgs);
template __global__ void isa_i16<24, 1, false, true>(SearchArgs);
template __global__ void isa_i16_self<24, 1, true>(SearchArgs);
template __global__ void isa_i16_self<24, 1, false>(SearchArgs);
template __global__ void isa_i16_self<24, 2, true>(SearchArgs);
template __global__ void isa_i16_self<24, 2, false>(SearchArgs);

}  // namespace swdb
