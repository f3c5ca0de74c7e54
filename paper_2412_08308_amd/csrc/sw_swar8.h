// Four unsigned 8-bit lanes in one 32-bit word ("SIMD within a register"),
// saturating at 0 and 255: the arithmetic an 8-bit inter-task lane form of
// the search would need (the lower-precision integers the paper names as
// future work, one step below the packed 16-bit lanes).  gfx950's vector ALU
// has packed 16-bit saturating add/sub and packed 16-bit max, but no packed
// 8-bit forms, so each operation is built from 32-bit logic and add/sub.
//
// Used only by the instruction-count probe (sw_isa_probe.hip) and by a CPU
// test that checks every function against byte-wise scalar arithmetic.
#pragma once
#include <cstdint>

namespace swdb {

constexpr uint32_t kTop8 = 0x80808080u;   // bit 7 of every byte

// 0xff in every byte whose bit 7 is set in t (t holds only bits 7):
// per byte 0x80 -> 2 * 0x80 - 1 = 0xff; the carry into the next byte cancels
// its -1, and the top byte wraps modulo 2^32.
__host__ __device__ __forceinline__ uint32_t swar8_fill(uint32_t t)
{
    return (t << 1) - (t >> 7);
}

// Byte-wise min(a + b, 255).  The low 7 bits of each byte are added without
// a carry into the next byte; bit 7 of the sum is the xor of the two bit 7s
// and the carry into it; a byte overflows when the majority of those three
// is set.
__host__ __device__ __forceinline__ uint32_t swar8_adds(uint32_t a, uint32_t b)
{
    const uint32_t lo = (a & ~kTop8) + (b & ~kTop8);
    const uint32_t hx = (a ^ b) & kTop8;
    const uint32_t sum = lo ^ hx;
    const uint32_t carry = ((a & b) | (lo & hx)) & kTop8;
    return sum | swar8_fill(carry);
}

// Byte-wise max(a - b, 0).  (a | 0x80) - (b & 0x7f) per byte lies in
// [1, 255], so no borrow crosses a byte; its bit 7 differs from that of
// a - b exactly when a and b have the same bit 7.  A byte borrows (a < b)
// when a's bit 7 is clear and b's set, or they are equal and the difference's
// bit 7 is set.
__host__ __device__ __forceinline__ uint32_t swar8_subs(uint32_t a, uint32_t b)
{
    const uint32_t same = ~(a ^ b) & kTop8;
    const uint32_t r = ((a | kTop8) - (b & ~kTop8)) ^ same;
    const uint32_t borrow = ((~a & b & kTop8) | (same & r)) & kTop8;
    return r & ~swar8_fill(borrow);
}

// Byte-wise max(a, b) = b + max(a - b, 0): every byte sum stays below 256.
__host__ __device__ __forceinline__ uint32_t swar8_max(uint32_t a, uint32_t b)
{
    return swar8_subs(a, b) + b;
}

}  // namespace swdb
