// int32 lanes, 32 query rows per lane, 16-bit query profile entries (used when
// a substitution score plus the gap-open penalty does not fit 8 bits).
#include "sw_device.h"

namespace swdb {

hipError_t launch_search_i32p16(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st)
{
    return launch_kernel(k_search<32, 2, false>, grid, waves, lds, st, a);
}

int occupancy_i32p16(int waves, int lds) { return occupancy_of(k_search<32, 2, false>, waves, lds); }

}  // namespace swdb
