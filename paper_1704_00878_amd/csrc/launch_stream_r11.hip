// sw_stream_kernel instances with R = 11..16 rows per lane.
#include "launch_stream_impl.hpp"

namespace hk {

void launch_stream_r11(int R, int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                      hipStream_t st) {
    launch_stream_range<11, 16>(R, LS, a, tb, endc, p16, grid, lds, st);
}

}  // namespace hk
