// Packed 2x16-bit saturating lanes with an 8-bit query profile (entries
// s + Go in [0, 127], zero-extended when the two subjects' entries are paired),
// 24 query rows per lane (the subjects it flags are rescored in sw_k_rescore.hip).
#include "sw_device.h"

namespace swdb {

hipError_t launch_search_i16p8(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st)
{
    return launch_kernel(k_search<kI16Rows, 1, true>, grid, waves, lds, st, a);
}


int occupancy_i16p8(int waves, int lds) { return occupancy_of(k_search<kI16Rows, 1, true>, waves, lds); }

}  // namespace swdb
