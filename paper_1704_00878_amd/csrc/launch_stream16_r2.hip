// sw_stream16_kernel (packed 16-bit) instances with R = 2..9 rows per lane.
#include "launch_stream_impl.hpp"

namespace hk {

void launch_stream16_r2(int R, int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st) {
    launch_stream16_range<2, 9>(R, LS, a, grid, lds, st);
}

}  // namespace hk
