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

// A substitution matrix passed by value (kernel argument), copied into device
// memory by one workgroup: no host staging buffer is involved.
struct MatrixArg {
    int8_t v[32 * 32];
};

__global__ void matrix_copy_kernel(MatrixArg mat, int n, int8_t *dst) {
    for (int x = threadIdx.x; x < n; x += blockDim.x) dst[x] = mat.v[x];
}

// Score-only calls that ask for cells report (0, 0, i1, j1).
__global__ void endcell_to_cells_kernel(const int32_t *endcell, int n, int32_t *cells) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    reinterpret_cast<int4 *>(cells)[k] = make_int4(0, 0, endcell[2 * k], endcell[2 * k + 1]);
}

// Largest code in [p, p + n) and [q, q + nq), raised into *out as
// (tag | code) with atomicMax (one atomic per workgroup).  16-byte loads where
// aligned.
__device__ __forceinline__ int maxcode_range(const uint8_t *p, int64_t n, int64_t tid, int64_t stride) {
    int mx = 0;
    const int64_t head = min<int64_t>(n, (int64_t)((16 - ((uintptr_t)p & 15)) & 15));
    for (int64_t x = tid; x < head; x += stride) mx = max(mx, (int)p[x]);
    const int64_t nv = (n - head) >> 4;
    const uint4 *pv = reinterpret_cast<const uint4 *>(p + head);
    for (int64_t x = tid; x < nv; x += stride) {
        const uint4 v = pv[x];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int y = 0; y < 4; ++y)
            mx = max(mx, max(max((int)(w[y] & 255), (int)((w[y] >> 8) & 255)),
                             max((int)((w[y] >> 16) & 255), (int)(w[y] >> 24))));
    }
    for (int64_t x = head + (nv << 4) + tid; x < n; x += stride) mx = max(mx, (int)p[x]);
    return mx;
}

__global__ void __launch_bounds__(256) maxcode_kernel(const uint8_t *p, int64_t n, const uint8_t *q, int64_t nq,
                                                      uint32_t tag, uint32_t *out) {
    __shared__ int red[4];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int mx = n > 0 ? maxcode_range(p, n, tid, stride) : 0;
    if (nq > 0) mx = max(mx, maxcode_range(q, nq, tid, stride));
    for (int sh = 32; sh > 0; sh >>= 1) mx = max(mx, __shfl_xor(mx, sh));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int b = max(max(red[0], red[1]), max(red[2], red[3]));
        atomicMax(out, tag | (uint32_t)b);
    }
}

// Zero up to four word ranges (and one trailing uint16) in one launch.
struct ZeroArgs {
    uint32_t *p[4];
    int64_t n[4];
    uint16_t *tail16;
};

__global__ void zero_kernel(ZeroArgs z) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        for (int64_t x = tid; x < z.n[r]; x += stride) z.p[r][x] = 0u;
    if (tid == 0 && z.tail16) *z.tail16 = 0;
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
// mail (optional, host memory mapped for the device): mail[0] = width, then
// mail[1] = seq with a system-scope release, so a host spinning on mail[1]
// reads the width without a stream synchronisation
__global__ void __launch_bounds__(1024) merge_scan_kernel(const int32_t *G, int m1, int64_t *col, int64_t *width,
                                                          int64_t *mail, int64_t seq) {
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
    if (tid == 1023) {
        *width = part[1023] - 1;
        if (mail) {
            __hip_atomic_store(mail, part[1023] - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(mail + 1, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Rows: one wavefront per row, up to four wavefronts per workgroup, each
// with its own LDS region.  Per row the wavefront stages the row's insertion
// counts and aligned bits, finds where each block starts in the sequence
// with a wave-wide prefix sum, and builds the row in LDS a chunk of columns
// at a time: fill with gaps, place every residue at its column (block p by
// binary search over the block starts; offset t < ins[p] goes to col[p] + t,
// the aligned residue to the center column col[p] + G[p]), then copy the
// chunk out with 16-byte stores.  The chunk sits in LDS at the row's
// misalignment, so aligned LDS words map onto aligned global words.
constexpr int kWaveRows = 4;

struct RowsArgs {
    const uint8_t *res;
    const int64_t *off;
    int nrows, m;
    const uint16_t *ins;
    const uint32_t *aligned;
    int aw;
    const int32_t *G;         // [m+1]
    const int64_t *col;       // [m+1]
    int64_t width;
    int ch;                   // columns per chunk (multiple of 16)
    int wave_bytes;           // LDS bytes per wavefront region
    int gc_lds;               // col staged in LDS for the workgroup (after the wave regions)
    uint8_t *msa;             // [nrows][width]
};

__global__ void __launch_bounds__(64 * kWaveRows) rows_kernel(RowsArgs a) {
    extern __shared__ uint4 lds_rows[];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int wpb = blockDim.x >> 6;
    const int m = a.m, m1 = m + 1;
    const int64_t width = a.width;
    // per wavefront: block starts in the sequence (uint16: lengths < 65536),
    // insertion counts, aligned bits, then the row chunk
    const size_t h2 = ((size_t)m1 * 2 + 3) & ~(size_t)3;
    char *wsh = reinterpret_cast<char *>(lds_rows) + (size_t)wid * a.wave_bytes;
    uint16_t *spos = reinterpret_cast<uint16_t *>(wsh);                         // [m1]
    uint16_t *sins = reinterpret_cast<uint16_t *>(wsh + h2);                   // [m1]
    uint32_t *abit = reinterpret_cast<uint32_t *>(wsh + 2 * h2);
    const size_t bo = (2 * h2 + 4 * (size_t)a.aw + 15) & ~(size_t)15;
    uint8_t *buf = reinterpret_cast<uint8_t *>(wsh + bo);                     // [ch + 16], 16-byte aligned
    uint4 *buf16 = reinterpret_cast<uint4 *>(buf);
    // the workgroup's column table: col[p] for p <= m and width + 1 after
    // it, so block p's gap count is col[p + 1] - col[p] - 1
    int *gcl = reinterpret_cast<int *>(reinterpret_cast<char *>(lds_rows) + (size_t)wpb * a.wave_bytes);
    if (a.gc_lds) {
        for (int p = tid; p <= m1; p += blockDim.x) gcl[p] = p < m1 ? (int)a.col[p] : (int)(width + 1);
        __syncthreads();
    }
    auto colg = [&](int p) __attribute__((always_inline)) -> int2 {
        return a.gc_lds ? make_int2(gcl[p], gcl[p + 1] - gcl[p] - 1) : make_int2((int)a.col[p], a.G[p]);
    };
    auto colv = [&](int p) __attribute__((always_inline)) -> int64_t {   // col[p], p <= m
        return a.gc_lds ? (int64_t)gcl[p] : a.col[p];
    };
    const int per = (m1 + 63) / 64;
    const int lo = min(m1, lane * per), hi = min(m1, lo + per);
    for (int k = blockIdx.x * wpb + wid; k < a.nrows; k += gridDim.x * wpb) {
        const int64_t so = a.off[k];
        const int n = (int)(a.off[k + 1] - so);
        const uint8_t *s = a.res + so;
        const uint16_t *ir = a.ins + (int64_t)k * m1;
        const uint32_t *ar = a.aligned + (int64_t)k * a.aw;
        __builtin_amdgcn_wave_barrier();   // the previous row is done with this region
        // staged with 8 loads in flight per lane (a long center's counts are
        // hundreds of loads per lane)
        for (int q0 = 0; q0 < a.aw; q0 += 512) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + 64 * u + lane;
                v[u] = q < a.aw ? ar[q] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + 64 * u + lane;
                if (q < a.aw) abit[q] = v[u];
            }
        }
        for (int p0 = 0; p0 < m1; p0 += 512) {
            uint16_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + 64 * u + lane;
                v[u] = p < m1 ? ir[p] : (uint16_t)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + 64 * u + lane;
                if (p < m1) sins[p] = v[u];
            }
        }
        __builtin_amdgcn_wave_barrier();
        int sum = 0;
        for (int p = lo; p < hi; ++p)
            sum += (int)sins[p] + ((p < m) ? (int)((abit[p >> 5] >> (p & 31)) & 1u) : 0);
        int inc = sum;   // inclusive prefix over the 64 lanes
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(inc, d, 64);
            if (lane >= d) inc += v;
        }
        int acc = inc - sum;
        for (int p = lo; p < hi; ++p) {
            spos[p] = (uint16_t)acc;
            acc += (int)sins[p] + ((p < m) ? (int)((abit[p >> 5] >> (p & 31)) & 1u) : 0);
        }
        __builtin_amdgcn_wave_barrier();
        uint8_t *row = a.msa + (int64_t)k * width;
        const int a0 = (int)((uintptr_t)row & 15);
        // Residues are split over the lanes chunk by chunk.  Columns grow with
        // the residue index, so a chunk of columns [x0, x1) holds the residues
        // first_at(x0) .. first_at(x1) - 1; first_at(x) is found from block p,
        // the last with col[p] <= x: block p's residues before column x are its
        // first min(x - col[p], ins[p]) (its insertions sit at col[p] + t, its
        // aligned residue at col[p + 1] - 1).  Each lane then places a
        // contiguous run of that range: one binary search for the block of its
        // first residue (within the chunk's blocks), then a short forward walk.
        auto first_at = [&](int64_t x, int &pblk) __attribute__((always_inline)) -> int {
            int l0 = pblk, h0 = m;   // col[pblk] <= x
            while (l0 < h0) {
                const int mid = (l0 + h0 + 1) >> 1;
                if (colv(mid) <= x) l0 = mid;
                else h0 = mid - 1;
            }
            pblk = l0;
            return (int)spos[l0] + (int)min<int64_t>(x - colv(l0), (int64_t)sins[l0]);
        };
        auto search = [&](int q, int l, int h) __attribute__((always_inline)) {   // last block in [l, h] with start <= q
            while (l < h) {
                const int mid = (l + h + 1) >> 1;
                if (spos[mid] <= q) l = mid;
                else h = mid - 1;
            }
            return l;
        };
        int qa = 0, pa = 0;   // the chunk's first residue and its block
        for (int64_t x0 = 0; x0 < width; x0 += a.ch) {
            const int len = (int)min<int64_t>(a.ch, width - x0);
            int pb = pa;
            const int qb = x0 + len >= width ? n : first_at(x0 + len, pb);
            const int nw = (a0 + len + 15) >> 4;
            for (int q = lane; q < nw; q += 64) buf16[q] = make_uint4(~0u, ~0u, ~0u, ~0u);
            __builtin_amdgcn_wave_barrier();
            const int pc = (qb - qa + 63) >> 6;
            const int r0 = min(qb, qa + lane * pc), r1 = min(qb, r0 + pc);
            int l = r0 < r1 ? search(r0, pa, x0 + len >= width ? m : pb) : 0;
            for (int q = r0; q < r1; ++q) {
                for (int st = 0; st < 4 && l < m && spos[l + 1] <= q; ++st) ++l;
                if (l < m && spos[l + 1] <= q) l = search(q, l, m);
                const int tq = q - spos[l];
                const int2 cg = colg(l);
                const int64_t dest = cg.x + (tq < (int)sins[l] ? tq : cg.y);
                if (dest >= x0 && dest < x0 + len) buf[a0 + (int)(dest - x0)] = s[q];
            }
            __builtin_amdgcn_wave_barrier();
            // copy out: LDS byte a0 + c holds column x0 + c
            uint8_t *dst = row + x0 - a0;   // 16-byte aligned (x0 is a multiple of 16)
            for (int q = lane; q < nw; q += 64) {
                const int b0 = 16 * q;
                if (b0 >= a0 && b0 + 16 <= a0 + len) {
                    *reinterpret_cast<uint4 *>(dst + b0) = buf16[q];
                } else {
                    for (int c = max(b0, a0); c < min(b0 + 16, a0 + len); ++c) dst[c] = buf[c];
                }
            }
            __builtin_amdgcn_wave_barrier();
            qa = qb;
            pa = pb;
        }
    }
}

constexpr int kRowsChunkMinBlocks = 4096;   // centers with more blocks take the chunked row kernels
constexpr int kRowChunk = 256;              // blocks per task, four per lane
constexpr int kRowWin = 2048;               // LDS bytes of a task's column window
constexpr int kRowRes = 2048;               // LDS bytes of a task's residues (more: read from global memory)
constexpr int kRowWave = kRowWin + 16 + kRowRes;   // LDS bytes per wavefront

// Chunked rows, first pass, one wavefront per row: ck[k][c] = residues of row
// k before block c * kRowChunk (insertions plus aligned bits), lane L counting
// blocks 4L .. 4L + 3 of each chunk (coalesced loads).
__global__ void __launch_bounds__(256) rows_count_kernel(RowsArgs a, int32_t *ck, int nck) {
    const int lane = threadIdx.x & 63;
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int nwave = (int)((gridDim.x * blockDim.x) >> 6);
    const int m = a.m, m1 = m + 1;
    for (int k = wave; k < a.nrows; k += nwave) {
        const uint16_t *ir = a.ins + (int64_t)k * m1;
        const uint32_t *ar = a.aligned + (int64_t)k * a.aw;
        int run = 0;
        for (int c = 0; c < nck; ++c) {
            const int b = c * kRowChunk + 4 * lane;
            int v = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (b + u < m1) v += (int)ir[b + u];
            if (b < m) {   // blocks b .. b + 3 share an aligned word (b is a multiple of 4)
                const uint32_t nb = (uint32_t)min(4, m - b);
                v += __popc((ar[b >> 5] >> (b & 31)) & ((1u << nb) - 1u));
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) ck[(int64_t)k * nck + c] = run;
            run += v;
        }
    }
}

// Chunked rows, second pass: one wavefront per (row k, chunk c) task, lane L
// owning blocks p = c * kRowChunk + 4L + u (u < 4).  Wave prefix sums over the
// lanes give each lane its first residue (from ck) and first column (from
// col[c * kRowChunk]); the chunk's residues are staged in LDS (coalesced), and
// its columns are built in an LDS window of kRowWin bytes at a time (filled
// with gaps, then each residue placed: block p's insertion t at its column +
// t, its aligned residue at its column + G[p]) and copied out with 16-byte
// stores, byte stores where a 16-byte word is shared with a neighbouring
// chunk.  The window sits in LDS at the
// output's misalignment, so aligned LDS words map onto aligned global words.
__global__ void __launch_bounds__(256) rows_chunk_kernel(RowsArgs a, const int32_t *ck, int nck) {
    extern __shared__ uint4 lds_rows[];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint8_t *buf = reinterpret_cast<uint8_t *>(lds_rows) + wid * kRowWave;
    uint4 *buf16 = reinterpret_cast<uint4 *>(buf);
    uint8_t *rbuf = buf + kRowWin + 16;   // the task's residues
    const int m = a.m, m1 = m + 1;
    const int64_t width = a.width;
    const int64_t ntask = (int64_t)a.nrows * nck;
    for (int64_t task = (int64_t)blockIdx.x * 4 + wid; task < ntask; task += (int64_t)gridDim.x * 4) {
        const int k = (int)(task / nck), c = (int)(task - (int64_t)k * nck);
        const int b = c * kRowChunk, bend = min(b + kRowChunk, m1);
        const int64_t so = a.off[k];
        const int n = (int)(a.off[k + 1] - so);
        const uint8_t *s = a.res + so;
        const uint16_t *ir = a.ins + (int64_t)k * m1;
        const uint32_t *ar = a.aligned + (int64_t)k * a.aw;
        const int p0 = b + 4 * lane;
        int ni[4], gg[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ni[u] = p0 + u < bend ? (int)ir[p0 + u] : 0;
            gg[u] = p0 + u < bend ? a.G[p0 + u] : 0;
        }
        const uint32_t al4 = p0 < m ? (ar[p0 >> 5] >> (p0 & 31)) & ((1u << min(4, m - p0)) - 1u) : 0u;
        int nres = 0, ncol = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            nres += ni[u] + (int)((al4 >> u) & 1u);
            ncol += p0 + u < bend ? gg[u] + (p0 + u < m ? 1 : 0) : 0;
        }
        int ir_ = nres, ic_ = ncol;   // inclusive prefix sums over the lanes
        for (int d = 1; d < 64; d <<= 1) {
            const int t1 = __shfl_up(ir_, d, 64), t2 = __shfl_up(ic_, d, 64);
            if (lane >= d) {
                ir_ += t1;
                ic_ += t2;
            }
        }
        const int qt = ck[task];                // the chunk's first residue
        const int q0 = qt + ir_ - nres;         // the lane's first residue
        // the chunk's residues qt .. qt + ntot - 1 into LDS (eight loads in
        // flight per lane), when they fit
        const int ntot = __shfl(ir_, 63, 64);
        const bool rl = ntot <= kRowRes;
        if (rl) {
            for (int i0 = 0; i0 < ntot; i0 += 512) {
                uint8_t v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + 64 * u + lane;
                    v[u] = i < ntot && qt + i < n ? s[qt + i] : (uint8_t)255;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + 64 * u + lane;
                    if (i < ntot) rbuf[i] = v[u];
                }
            }
        }
        auto resid = [&](int r) __attribute__((always_inline)) -> uint8_t {
            return rl ? rbuf[r - qt] : (r < n ? s[r] : (uint8_t)255);
        };
        const int64_t colb = a.col[b];
        const int64_t span = (bend < m1 ? a.col[bend] : width) - colb;
        const int cl = ic_ - ncol;              // the lane's first column, relative to colb
        uint8_t *row = a.msa + (int64_t)k * width;
        const int a0 = (int)((uintptr_t)(row + colb) & 15);
        for (int64_t x0 = 0; x0 < span; x0 += kRowWin) {
            const int wl = (int)min<int64_t>(kRowWin, span - x0);
            const int nw = (a0 + wl + 15) >> 4;
            for (int q = lane; q < nw; q += 64) buf16[q] = make_uint4(~0u, ~0u, ~0u, ~0u);
            __builtin_amdgcn_wave_barrier();
            int cu = cl, qu = q0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (p0 + u < bend) {
                    // insertions t at cu + t, for the t inside the window
                    const int64_t t0 = max<int64_t>(0, x0 - cu), t1 = min<int64_t>(ni[u], x0 + wl - cu);
                    for (int64_t t = t0; t < t1; ++t) buf[a0 + (int)(cu + t - x0)] = resid(qu + (int)t);
                    qu += ni[u];
                    if (p0 + u < m) {
                        if ((al4 >> u) & 1u) {
                            const int64_t pos = (int64_t)cu + gg[u] - x0;
                            if (pos >= 0 && pos < wl) buf[a0 + (int)pos] = resid(qu);
                            ++qu;
                        }
                        cu += gg[u] + 1;
                    } else {
                        cu += gg[u];
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            uint8_t *dst = row + colb + x0 - a0;   // 16-byte aligned
            for (int q = lane; q < nw; q += 64) {
                const int b0 = 16 * q;
                if (b0 >= a0 && b0 + 16 <= a0 + wl) {
                    *reinterpret_cast<uint4 *>(dst + b0) = buf16[q];
                } else {
                    for (int e = max(b0, a0); e < min(b0 + 16, a0 + wl); ++e) dst[e] = buf[e];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

constexpr int kProfCols = 256;      // columns per workgroup (one per lane)
constexpr int kProfMaxSlab = 65535; // rows per workgroup (16-bit partial counts)
constexpr int kProfRows = 32;       // rows loaded per pass

// rows of one column into the lane's LDS counters (stride 256 words): bin 0
// gaps, 1 + a for residue code a, top = alpha + 1 anything else; EDGE: a lane
// past the last column (in == false) reads the last column and counts into
// bin top + 1, which is discarded, so the row loop has no branch
template <bool EDGE>
__device__ __forceinline__ void colprof_rows(const uint8_t *p, int64_t width, int rows, uint32_t *lc, uint32_t top,
                                             bool in) {
    auto count = [&](uint32_t b) __attribute__((always_inline)) {
        uint32_t bin = min((b + 1u) & 255u, top);
        if (EDGE) bin = in ? bin : top + 1u;
        atomicAdd(lc + bin * 256, 1u);
    };
    int r = 0;
    for (; r + kProfRows <= rows; r += kProfRows, p += kProfRows * width) {
        uint32_t v[kProfRows];
#pragma unroll
        for (int u = 0; u < kProfRows; ++u) v[u] = p[u * width];
#pragma unroll
        for (int u = 0; u < kProfRows; ++u) count(v[u]);
    }
    for (; r < rows; ++r, p += width) count(*p);
}

// Column profile of an N x W MSA, first pass: workgroup (x, y) counts the
// bytes of columns 256 x .. 256 x + 255 over the rows of slab y.  Lane t owns
// column 256 x + t, so each byte load of a wavefront covers 64 consecutive
// bytes of a row; 32 rows are loaded before they are counted.  The lane's
// counters sit in LDS (word bin * 256 + t, no barrier needed): bin 0 counts
// gaps, bin 1 + a residue code a, bin alpha + 1 any other byte (which raises
// *bad).  The slab's counts go, without atomics, to part[y][column][slot]
// (uint16; slot a < alpha a residue code, slot alpha the gaps), written in
// contiguous runs.  A lane past the last column reads the last column and
// counts into a discarded bin, so the row loop has no branch.
__global__ void __launch_bounds__(256)
colprof_kernel(const uint8_t *msa, int n, int64_t width, int alpha, int slab, uint16_t *part, int *bad) {
    extern __shared__ uint32_t pcnt[];
    const int nbin = alpha + 3;
    const int t = threadIdx.x;
    uint32_t *lc = pcnt + t;
    for (int x = 0; x < nbin; ++x) lc[x * 256] = 0;
    const int64_t cb = (int64_t)blockIdx.x * kProfCols;
    const bool in = cb + t < width;
    const int r0 = blockIdx.y * slab;
    const int r1 = min(n, r0 + slab);
    const uint8_t *p = msa + (int64_t)r0 * width + (in ? cb + t : width - 1);
    if (cb + kProfCols <= width) colprof_rows<false>(p, width, r1 - r0, lc, (uint32_t)alpha + 1u, true);
    else colprof_rows<true>(p, width, r1 - r0, lc, (uint32_t)alpha + 1u, in);
    if (in && lc[(alpha + 1) * 256] != 0) atomicOr(bad, 1);
    __syncthreads();
    // slab counts out: element e of the workgroup's run is (column e / nsym, slot e % nsym)
    const int nsym = alpha + 1;
    const int64_t ncols = min((int64_t)kProfCols, width - cb);
    uint16_t *dst = part + ((int64_t)blockIdx.y * width + cb) * nsym;
    for (int e = t; e < ncols * nsym; e += 256) {
        const int c = e / nsym, slot = e - c * nsym;
        dst[e] = (uint16_t)pcnt[(slot == alpha ? 0 : slot + 1) * 256 + c];
    }
}

// Second pass: profile[e] = sum over slabs of part[slab][e], e < width * nsym.
__global__ void __launch_bounds__(256)
colprof_sum_kernel(const uint16_t *part, int nslab, int64_t nelem, int32_t *prof) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nelem) return;
    int32_t s = 0;
    for (int y = 0; y < nslab; ++y) s += part[(int64_t)y * nelem + e];
    prof[e] = s;
}

// avg SP numerator and BLOSUM column SP from a column profile, one thread
// per column: out[0] += (pairs of different residues) + 2 * (residue-gap
// pairs); out[1] += sum of S over residue pairs - ge * (residue-gap pairs).
__global__ void __launch_bounds__(256)
sp_profile_kernel(const int32_t *prof, int64_t width, int alpha, const int8_t *mat, int ge,
                  unsigned long long *out) {
    __shared__ int smat[32][32];
    const int tid = threadIdx.x;
    for (int x = tid; x < 1024; x += 256) {
        const int a = x >> 5, b = x & 31;
        smat[a][b] = (a < alpha && b < alpha) ? mat[a * alpha + b] : 0;
    }
    __syncthreads();
    const int64_t x = (int64_t)blockIdx.x * 256 + tid;
    if (x >= width) return;
    const int32_t *c = prof + x * (alpha + 1);
    const int64_t g = c[alpha];
    int64_t r = 0, same = 0, bl = 0;
    for (int a = 0; a < alpha; ++a) {
        const int64_t ca = c[a];
        if (!ca) continue;
        r += ca;
        same += ca * (ca - 1) / 2;
        bl += ca * (ca - 1) / 2 * smat[a][a];
        for (int b = a + 1; b < alpha; ++b) bl += ca * (int64_t)c[b] * smat[a][b];
    }
    const int64_t sp = (r * (r - 1) / 2 - same) + 2 * g * r;
    bl -= (int64_t)ge * g * r;
    atomicAdd(out, (unsigned long long)sp);
    atomicAdd(out + 1, (unsigned long long)bl);
}

}  // namespace hk
