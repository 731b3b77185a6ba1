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
// 16-byte loads where aligned, one atomic per workgroup.
__global__ void __launch_bounds__(256) maxcode_kernel(const uint8_t *p, int64_t n, int *out) {
    __shared__ int red[4];
    int mx = 0;
    const int64_t head = min<int64_t>(n, (int64_t)((16 - ((uintptr_t)p & 15)) & 15));
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = tid; x < head; x += stride) mx = max(mx, (int)p[x]);
    const int64_t nv = (n - head) >> 4;
    const uint4 *pv = reinterpret_cast<const uint4 *>(p + head);
    for (int64_t x = tid; x < nv; x += stride) {
        const uint4 q = pv[x];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int y = 0; y < 4; ++y)
            mx = max(mx, max(max((int)(w[y] & 255), (int)((w[y] >> 8) & 255)),
                             max((int)((w[y] >> 16) & 255), (int)(w[y] >> 24))));
    }
    for (int64_t x = head + (nv << 4) + tid; x < n; x += stride) mx = max(mx, (int)p[x]);
    for (int sh = 32; sh > 0; sh >>= 1) mx = max(mx, __shfl_xor(mx, sh));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int b = max(max(red[0], red[1]), max(red[2], red[3]));
        if (b > 0) atomicMax(out, b);
    }
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

// Column map: for every MSA column x, cmap[x] = (p << 16) | t for offset t of
// gap block p, or (p << 16) | 0xffff for the column of center position p.
// (A gap block holds at most max_k ins_k[p] < 65535 columns.)
__global__ void colmap_kernel(const int32_t *G, const int64_t *col, int m, uint32_t *cmap) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > m) return;
    const int64_t c0 = col[p];
    const int g = G[p];
    for (int t = 0; t < g; ++t) cmap[c0 + t] = ((uint32_t)p << 16) | (uint32_t)t;
    if (p < m) cmap[c0 + g] = ((uint32_t)p << 16) | 0xffffu;
}

// Rows: a workgroup keeps the column map in LDS (when it fits) and emits many
// rows; per row it scans (ins + aligned) to find where each block starts in
// the sequence, then writes the row four columns per store where aligned.
__device__ __forceinline__ uint8_t row_byte(uint32_t cm, const int *spos, const int *sins, const uint32_t *ar,
                                            const uint8_t *s, int n) {
    const int p = (int)(cm >> 16), t = (int)(cm & 0xffffu);
    uint8_t b = kGap;
    if (t == 0xffff) {
        const int q = spos[p] + sins[p];
        if (((ar[p >> 5] >> (p & 31)) & 1u) && q < n) b = s[q];
    } else {
        const int q = spos[p] + t;
        if (t < sins[p] && q < n) b = s[q];
    }
    return b;
}

__global__ void __launch_bounds__(256)
rows_kernel(const uint8_t *res, const int64_t *off, int nrows, int m,
            const uint16_t *ins, const uint32_t *aligned, int aw,
            const uint32_t *cmap_g, int64_t width, int cmap_in_lds, uint8_t *msa) {
    extern __shared__ int sh[];
    int *spos = sh;                 // [m+1] start of block p in s
    int *sins = spos + (m + 1);     // [m+1] ins copy
    uint32_t *cml = reinterpret_cast<uint32_t *>(sins + (m + 1));   // [width] when in LDS
    __shared__ int partial[256];
    const int tid = threadIdx.x;
    if (cmap_in_lds) {
        for (int64_t x = tid; x < width; x += 256) cml[x] = cmap_g[x];
    }
    const uint32_t *cm = cmap_in_lds ? cml : cmap_g;
    const int m1 = m + 1;
    const int per = (m1 + 255) / 256;
    const int lo = min(m1, tid * per), hi = min(m1, lo + per);
    for (int k = blockIdx.x; k < nrows; k += gridDim.x) {
        const uint8_t *s = res + off[k];
        const int n = (int)(off[k + 1] - off[k]);
        const uint16_t *ir = ins + (int64_t)k * m1;
        const uint32_t *ar = aligned + (int64_t)k * aw;
        __syncthreads();   // previous row done with spos / sins
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
        const int64_t head = min<int64_t>(width, (int64_t)((4 - ((uintptr_t)row & 3)) & 3));
        if (tid < head) row[tid] = row_byte(cm[tid], spos, sins, ar, s, n);
        const int64_t nq = (width - head) >> 2;
        uint32_t *rq = reinterpret_cast<uint32_t *>(row + head);
        for (int64_t q = tid; q < nq; q += 256) {
            const int64_t x = head + 4 * q;
            const uint32_t v = (uint32_t)row_byte(cm[x], spos, sins, ar, s, n) |
                               ((uint32_t)row_byte(cm[x + 1], spos, sins, ar, s, n) << 8) |
                               ((uint32_t)row_byte(cm[x + 2], spos, sins, ar, s, n) << 16) |
                               ((uint32_t)row_byte(cm[x + 3], spos, sins, ar, s, n) << 24);
            rq[q] = v;
        }
        for (int64_t x = head + 4 * nq + tid; x < width; x += 256) row[x] = row_byte(cm[x], spos, sins, ar, s, n);
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
