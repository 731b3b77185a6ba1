// Launchers of the wavefront forward kernels.  Each geometry (rows per lane
// R, lanes per stream LS, traceback / end-cell variant, profile width) is a
// separate template instance; the instances are spread over several
// translation units (launch_stream_*.hip) so that they compile in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "sw_kernels.hpp"

namespace hk {

// 64-lane streams with R = 1..8 (int16 or int32 profile); 32- and 16-lane
// streams with R = 2..16 (int16 profile)
inline bool stream_supported(int R, int LS, bool p16) {
    if (LS == 64) return R >= 1 && R <= 8;
    return (LS == 32 || LS == 16) && p16 && R >= 2 && R <= 16;
}

// packed 16-bit kernel (traceback with end cells): 32- and 16-lane streams, R = 2..16
inline bool stream16_supported(int R, int LS) { return (LS == 32 || LS == 16) && R >= 2 && R <= 16; }

// sw_stream_kernel for R in [1, 5], [6, 10] and [11, 16] (one translation unit each)
void launch_stream_r1(int R, int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                      hipStream_t st);
void launch_stream_r6(int R, int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                      hipStream_t st);
void launch_stream_r11(int R, int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                       hipStream_t st);
// sw_stream16_kernel for R in [2, 9] and [10, 16]
void launch_stream16_r2(int R, int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st);
void launch_stream16_r10(int R, int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st);

inline void launch_stream(int R, int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                          hipStream_t st) {
    if (R <= 5) launch_stream_r1(R, LS, a, tb, endc, p16, grid, lds, st);
    else if (R <= 10) launch_stream_r6(R, LS, a, tb, endc, p16, grid, lds, st);
    else launch_stream_r11(R, LS, a, tb, endc, p16, grid, lds, st);
}

inline void launch_stream16(int R, int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st) {
    if (R <= 9) launch_stream16_r2(R, LS, a, grid, lds, st);
    else launch_stream16_r10(R, LS, a, grid, lds, st);
}

}  // namespace hk
