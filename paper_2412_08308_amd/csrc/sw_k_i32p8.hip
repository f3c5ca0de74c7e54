// int32 lanes, 32 query rows per lane, 8-bit query profile entries.
#include "sw_device.h"

namespace swdb {

hipError_t launch_search_i32p8(const SearchArgs& a, int grid, int waves, int lds, hipStream_t st)
{
    return launch_kernel(k_search<32, 1, false>, grid, waves, lds, st, a);
}

int occupancy_i32p8(int waves, int lds) { return occupancy_of(k_search<32, 1, false>, waves, lds); }

}  // namespace swdb
