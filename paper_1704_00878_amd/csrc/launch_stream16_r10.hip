// sw_stream16_kernel (packed 16-bit) instances with R = 10..16 rows per lane.
#include "launch_stream_impl.hpp"

namespace hk {

void launch_stream16_r10(int R, int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st) {
    launch_stream16_range<10, 16>(R, LS, a, grid, lds, st);
}

}  // namespace hk
