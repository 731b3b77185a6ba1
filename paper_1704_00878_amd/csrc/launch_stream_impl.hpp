// Template dispatch behind launch.hpp: included by the launch_stream_*.hip
// translation units only.
#pragma once
#include "launch.hpp"
#include "stream16_kernels.hpp"

namespace hk {

template <int R, int LS, bool P16>
void launch_stream_RLP(const StreamArgs &a, bool tb, bool endc, int grid, size_t lds, hipStream_t st) {
    if (tb)
        hipLaunchKernelGGL((sw_stream_kernel<R, LS, true, true, P16>), dim3(grid), dim3(512), lds, st, a);
    else if (endc)
        hipLaunchKernelGGL((sw_stream_kernel<R, LS, false, true, P16>), dim3(grid), dim3(512), lds, st, a);
    else
        hipLaunchKernelGGL((sw_stream_kernel<R, LS, false, false, P16>), dim3(grid), dim3(512), lds, st, a);
}

template <int R>
void launch_stream_R(int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                     hipStream_t st) {
    if constexpr (R <= 8) {
        if (LS == 64) {
            if (p16) launch_stream_RLP<R, 64, true>(a, tb, endc, grid, lds, st);
            else launch_stream_RLP<R, 64, false>(a, tb, endc, grid, lds, st);
            return;
        }
    }
    if constexpr (R >= 2) {
        if (LS == 32) launch_stream_RLP<R, 32, true>(a, tb, endc, grid, lds, st);
        else launch_stream_RLP<R, 16, true>(a, tb, endc, grid, lds, st);
    }
}

// R in [LO, HI]: one case per instantiated R
template <int LO, int HI>
void launch_stream_range(int R, int LS, const StreamArgs &a, bool tb, bool endc, bool p16, int grid, size_t lds,
                         hipStream_t st) {
    if constexpr (LO <= HI) {
        if (R == LO) launch_stream_R<LO>(LS, a, tb, endc, p16, grid, lds, st);
        else launch_stream_range<LO + 1, HI>(R, LS, a, tb, endc, p16, grid, lds, st);
    }
}

template <int R>
void launch_stream16_R(int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st) {
    if (LS == 32) hipLaunchKernelGGL((sw_stream16_kernel<R, 32>), dim3(grid), dim3(512), lds, st, a);
    else hipLaunchKernelGGL((sw_stream16_kernel<R, 16>), dim3(grid), dim3(512), lds, st, a);
}

template <int LO, int HI>
void launch_stream16_range(int R, int LS, const StreamArgs &a, int grid, size_t lds, hipStream_t st) {
    if constexpr (LO <= HI) {
        if (R == LO) launch_stream16_R<LO>(LS, a, grid, lds, st);
        else launch_stream16_range<LO + 1, HI>(R, LS, a, grid, lds, st);
    }
}

}  // namespace hk
