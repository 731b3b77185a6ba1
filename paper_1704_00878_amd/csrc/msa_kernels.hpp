// Center-star merge and row emission (Fig. 3: the first reduction builds the
// longest center-star sequence from all inserted-space vectors; the second map
// builds each row from its inserted-space vector and its own sequence), plus
// encoding, small fills and the avg SP evaluation of the Results section.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int kGap = 255;

// Fill with a kernel (graph-capturable, no memset nodes).
__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        p[x] = v;
}

__global__ void fill_u16_kernel(uint16_t *p, uint16_t v, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        p[x] = v;
}

// Score-only calls that ask for cells report (0, 0, i1, j1).
__global__ void endcell_to_cells_kernel(const int32_t *endcell, int n, int32_t *cells) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    reinterpret_cast<int4 *>(cells)[k] = make_int4(0, 0, endcell[2 * k], endcell[2 * k + 1]);
}

// Largest residue code in [p, p + n) -> *out (atomicMax; *out zeroed before).
__global__ void maxcode_kernel(const uint8_t *p, int64_t n, int *out) {
    int mx = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        mx = max(mx, (int)p[x]);
    for (int sh = 32; sh > 0; sh >>= 1) mx = max(mx, __shfl_xor(mx, sh));
    if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(out, mx);
}

// ASCII -> residue code through a 256-entry table.
__global__ void encode_kernel(const uint8_t *ascii, int64_t len, uint8_t *codes, const uint8_t *table) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < len;
         x += (int64_t)gridDim.x * blockDim.x)
        codes[x] = table[ascii[x]];
}

// The center's own row: no insertions, every center position aligned.
__global__ void center_row_kernel(uint16_t *ins, uint32_t *aligned, int center, int m, int aw) {
    uint16_t *ir = ins + (int64_t)center * (m + 1);
    uint32_t *ar = aligned + (int64_t)center * aw;
    for (int p = threadIdx.x; p <= m; p += blockDim.x) ir[p] = 0;
    for (int w = threadIdx.x; w < aw; w += blockDim.x) {
        const int lo = w * 32;
        const int nb = min(32, m - lo);
        ar[w] = nb >= 32 ? 0xffffffffu : ((1u << nb) - 1u);
    }
}

// G[p] = max_k ins[k][p].  Block (256 threads) covers 256 slots x kRows rows,
// reduces in registers and publishes with one integer atomicMax per slot
// (max is order-independent, so the result is deterministic).
constexpr int kMergeRows = 64;
__global__ void merge_max_kernel(const uint16_t *ins, int n, int m1, int32_t *G) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m1) return;
    const int k0 = blockIdx.y * kMergeRows;
    const int k1 = min(n, k0 + kMergeRows);
    int g = 0;
    for (int k = k0; k < k1; ++k) g = max(g, (int)ins[(int64_t)k * m1 + p]);
    if (g > 0) atomicMax(G + p, g);
}

// col[p] = sum_{q<p} (G[q] + 1); width = m + sum G.  One workgroup of 1024.
__global__ void __launch_bounds__(1024) merge_scan_kernel(const int32_t *G, int m1, int64_t *col, int64_t *width) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int per = (m1 + 1023) / 1024;
    const int lo = min(m1, tid * per), hi = min(m1, lo + per);
    int64_t sum = 0;
    for (int p = lo; p < hi; ++p) sum += G[p] + 1;
    part[tid] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t acc = tid > 0 ? part[tid - 1] : 0;
    for (int p = lo; p < hi; ++p) { col[p] = acc; acc += G[p] + 1; }
    if (tid == 1023) *width = part[1023] - 1;
}

// Column map: for every MSA column x, (p << 1) | 1 for the column of center
// position p, (p << 1) for a column of gap block p; off[x] = offset in block.
__global__ void colmap_kernel(const int32_t *G, const int64_t *col, int m, int32_t *cmap, int32_t *coff) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > m) return;
    const int64_t c0 = col[p];
    const int g = G[p];
    for (int t = 0; t < g; ++t) { cmap[c0 + t] = p << 1; coff[c0 + t] = t; }
    if (p < m) { cmap[c0 + g] = (p << 1) | 1; coff[c0 + g] = 0; }
}

// One workgroup per row: scan the row's (ins + aligned) to get the sequence
// position where each block starts, then write the row column by column.
__global__ void __launch_bounds__(256)
rows_kernel(const uint8_t *res, const int64_t *off, const int32_t *rowids, int nrows, int m,
            const uint16_t *ins, const uint32_t *aligned, int aw,
            const int32_t *cmap, const int32_t *coff, int64_t width, uint8_t *msa) {
    extern __shared__ int spos[];    // [m+1] start of block p in s, then ins copy
    int *sins = spos + (m + 1);
    __shared__ int partial[256];
    const int r = blockIdx.x;
    if (r >= nrows) return;
    const int k = rowids ? rowids[r] : r;
    const uint8_t *s = res + off[k];
    const int n = (int)(off[k + 1] - off[k]);
    const uint16_t *ir = ins + (int64_t)k * (m + 1);
    const uint32_t *ar = aligned + (int64_t)k * aw;
    const int tid = threadIdx.x;
    const int m1 = m + 1;
    const int per = (m1 + 255) / 256;
    const int lo = min(m1, tid * per), hi = min(m1, lo + per);
    int sum = 0;
    for (int p = lo; p < hi; ++p) {
        const int v = ir[p];
        sins[p] = v;
        sum += v + ((p < m) ? (int)((ar[p >> 5] >> (p & 31)) & 1u) : 0);
    }
    partial[tid] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int v = tid >= d ? partial[tid - d] : 0;
        __syncthreads();
        partial[tid] += v;
        __syncthreads();
    }
    int acc = tid > 0 ? partial[tid - 1] : 0;
    for (int p = lo; p < hi; ++p) {
        spos[p] = acc;
        acc += sins[p] + ((p < m) ? (int)((ar[p >> 5] >> (p & 31)) & 1u) : 0);
    }
    __syncthreads();
    uint8_t *row = msa + (int64_t)k * width;
    for (int64_t x = tid; x < width; x += 256) {
        const int cm = cmap[x];
        const int p = cm >> 1;
        uint8_t b = kGap;
        if (cm & 1) {
            const int q = spos[p] + sins[p];
            if (((ar[p >> 5] >> (p & 31)) & 1u) && q < n) b = s[q];
        } else {
            const int t = coff[x];
            const int q = spos[p] + t;
            if (t < sins[p] && q < n) b = s[q];
        }
        row[x] = b;
    }
}

// avg SP numerator and BLOSUM column SP over an N x W MSA, one thread per
// column; counts per residue code kept in LDS.  out[0] += sum over columns of
// (pairs of different residues) + 2*(residue-gap pairs); out[1] += BLOSUM SP.
__global__ void __launch_bounds__(128)
sp_kernel(const uint8_t *msa, int n, int64_t width, const int8_t *mat, int alpha, int ge,
          unsigned long long *out) {
    __shared__ int cnt[128][33];
    __shared__ int smat[32][32];
    const int tid = threadIdx.x;
    for (int x = tid; x < 1024; x += 128) {
        const int a = x >> 5, b = x & 31;
        smat[a][b] = (a < alpha && b < alpha) ? mat[a * alpha + b] : 0;
    }
    const int64_t x = (int64_t)blockIdx.x * 128 + tid;
    for (int c = 0; c < 33; ++c) cnt[tid][c] = 0;
    __syncthreads();
    if (x < width) {
        for (int k = 0; k < n; ++k) {
            const int b = msa[(int64_t)k * width + x];
            cnt[tid][b == kGap ? 32 : (b & 31)]++;
        }
        const int64_t g = cnt[tid][32], r = n - g;
        int64_t same = 0, bl = 0;
        for (int a = 0; a < 32; ++a) {
            const int64_t ca = cnt[tid][a];
            if (!ca) continue;
            same += ca * (ca - 1) / 2;
            bl += ca * (ca - 1) / 2 * smat[a][a];
            for (int b = a + 1; b < 32; ++b) bl += ca * (int64_t)cnt[tid][b] * smat[a][b];
        }
        const int64_t sp = (r * (r - 1) / 2 - same) + 2 * g * r;
        bl -= (int64_t)ge * g * r;
        atomicAdd(out, (unsigned long long)sp);
        atomicAdd(out + 1, (unsigned long long)bl);
    }
}

}  // namespace hk
