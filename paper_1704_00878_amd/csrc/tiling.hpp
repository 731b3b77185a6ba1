// Group enumeration of the exhaustive center (the sequence most similar to
// all others needs the score of every pair): all pairs (a, b), a < b, of
// positions in length order, tiled into groups of one center position a and
// `step` consecutive partner positions [q*step, (q+1)*step), block q.  Block q
// holds the groups a = 0 .. c_q - 1 with c_q = min((q+1)*step, n) - 1 (each
// center stays below some partner of its block), and groups are numbered
// block by block, so group g lies in the block q with P(q) <= g < P(q+1),
// P(q) = step*q*(q+1)/2 - q.  Lanes of a group whose partner position is not
// above the center's are idle.  The numbering is closed form: nothing of size
// O(n^2) is ever built.  Compiled for host and device.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace hk {

__host__ __device__ inline int64_t tri_prefix(int64_t q, int step) { return (int64_t)step * q * (q + 1) / 2 - q; }

// number of groups for n positions
__host__ __device__ inline int64_t tri_groups(int64_t n, int step) {
    if (n < 2) return 0;
    const int64_t nb = (n + step - 1) / step;
    return tri_prefix(nb - 1, step) + (n - 1);
}

// group g (0 <= g < tri_groups(n, step)) -> center position, first partner position
__host__ __device__ inline void tri_group(int64_t g, int64_t n, int step, int64_t *apos, int64_t *b0) {
    const int64_t nb = (n + step - 1) / step;
    int64_t q = (int64_t)sqrt(2.0 * (double)g / (double)step);
    if (q > nb - 1) q = nb - 1;
    while (q > 0 && tri_prefix(q, step) > g) --q;
    while (q + 1 <= nb - 1 && tri_prefix(q + 1, step) <= g) ++q;
    *apos = g - tri_prefix(q, step);
    *b0 = q * step;
}

}  // namespace hk
