// Packed 2x16-bit saturating lanes (two subjects per lane), 24 query rows per
// lane, and the exact int32 rescore of the subjects it flags.
#include "sw_device.h"

namespace swdb {

hipError_t launch_search_i16(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st)
{
    return launch_kernel(k_search<kI16Rows, 2, true>, grid, waves, lds, st, a);
}

hipError_t launch_rescore_i16(const SearchArgs& a, int grid, int waves, hipStream_t st)
{
    // same profile layout as the 16-bit pass: kI16Rows rows of 16-bit entries
    return launch_kernel(k_rescore<kI16Rows, 2>, grid, waves, 0, st, a);
}

int occupancy_i16(int waves, int lds) { return occupancy_of(k_search<kI16Rows, 2, true>, waves, lds); }

}  // namespace swdb
