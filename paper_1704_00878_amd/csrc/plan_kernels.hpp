// Small kernels around the wavefront forward pass: staging of stream
// residues and decoding of the end-cell keys.
#pragma once
#include "sw_kernels.hpp"

namespace hk {

// keys -> score and end cell (i1, j1), 1-based; slot q belongs to pair pid[q].
__global__ void decode_keys_kernel(const unsigned long long *keys, const int32_t *slot_pid, int nslots,
                                   int32_t *score, int32_t *endcell) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nslots) return;
    const unsigned long long k = keys[q];
    const int pid = slot_pid[q];
    const int h = (int)(k >> 32);
    score[pid] = h;
    if (endcell) {
        endcell[2 * pid] = h > 0 ? (0xffff - (int)(k & 0xffff)) + 1 : 0;
        endcell[2 * pid + 1] = h > 0 ? 0xffff - (int)((k >> 16) & 0xffff) : 0;
    }
}

// Stage the residues of every stream: sres[sbase + c0(q) + x] = s_q[x], with
// kFirstCol on x = 0, and clear the slot's end-cell key.  One workgroup per
// pair slot.
__global__ void stage_stream_kernel(const uint8_t *res, const int64_t *off, const int32_t *slot_pid,
                                    const int64_t *slot_col, int nslots, int clamp, uint8_t *sres,
                                    unsigned long long *keys) {
    const int q = blockIdx.x;
    if (q >= nslots) return;
    if (threadIdx.x == 0) keys[q] = 0ull;
    const int pid = slot_pid[q];
    const int64_t so = off[pid];
    const int n = (int)(off[pid + 1] - so);
    uint8_t *dst = sres + slot_col[q];
    for (int x = threadIdx.x; x < n; x += blockDim.x)
        dst[x] = (uint8_t)(min((int)(res[so + x] & 31), clamp) | (x == 0 ? kFirstCol : 0));
}

}  // namespace hk
