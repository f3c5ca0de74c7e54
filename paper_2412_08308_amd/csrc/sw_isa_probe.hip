// Not part of the library.  Compiled only to AMD assembly by isa_count.py:
// every hot-loop variant of the search, instantiated alone in a kernel with
// the same attributes as the persistent search kernels, so that its innermost
// loop (four subject columns x R query rows) can be counted instruction by
// instruction.
#include "sw_device.h"

namespace swdb {

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
