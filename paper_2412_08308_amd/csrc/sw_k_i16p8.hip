// Packed 2x16-bit saturating lanes with an 8-bit query profile (entries
// s + Go in [0, 127], zero-extended when the two subjects' entries are paired),
// 24 query rows per lane, and the exact int32 rescore of the subjects it flags.
#include "sw_device.h"

namespace swdb {

hipError_t launch_search_i16p8(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st)
{
    return launch_kernel(k_search<kI16Rows, 1, true>, grid, waves, lds, st, a);
}

hipError_t launch_rescore_i16p8(const SearchArgs& a, int grid, int waves, hipStream_t st)
{
    // same profile as the packed pass: kI16Rows rows of 8-bit entries (the
    // entries are non-negative, so the int32 item's sign extension reads them
    // unchanged)
    return launch_kernel(k_rescore<kI16Rows, 1>, grid, waves, 0, st, a);
}

int occupancy_i16p8(int waves, int lds) { return occupancy_of(k_search<kI16Rows, 1, true>, waves, lds); }

}  // namespace swdb
