// Phylogeny from the MSA for gfx950 (Methods, "NJ method for constructing
// phylogenetic trees with Spark", Fig. 4): pairwise p-distances between MSA
// rows, the nearest-seed labels of the sampled clustering, and neighbour
// joining (Saitou and Nei) over distance matrices.
//
// Distances are integer counts (columns where both rows hold a residue, and
// those of them that differ) turned into a double by one IEEE division, so
// they are exact.  Neighbour joining does every double operation on its own
// (the kernels turn floating-point contraction off, so no multiply and add
// fuse) and in a fixed order (row sums in slot order), so the joins and
// branch lengths are the same bits on any schedule of the lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int kPdTile = 64;    // pairs per workgroup: 64 rows of A x 64 rows of B
constexpr int kPdChunk = 64;   // columns staged per pass (16 words per row)
constexpr int kPdStride = 17;  // LDS 64-bit words per staged row (16 + 1: no bank conflicts between rows)

// One group of pairs: rows rows[a0 + i] (i < na) against rows[b0 + j] (j <
// nb); D[i * ld + j] (and the counts, when given) at out offset o.  diag0:
// the group is square over the same rows and its diagonal is written as 0.
struct PdGroup {
    int64_t a0, b0;
    int na, nb;
    int64_t o, ld;
    int diag0;
    int tiles_b;      // ceil(nb / 64)
    int64_t tile0;    // first tile of this group (prefix over groups)
};

struct PdArgs {
    const uint8_t *msa;
    int64_t width;
    const int32_t *rows;
    const PdGroup *groups;
    int ngroups;
    double *D;
    int32_t *mism, *comp;   // optional
    // column slices: nslice > 1 splits the width into slices of cslice
    // columns (a multiple of kPdChunk), each slice's counts added atomically
    // into acc (2 int32 per output, zeroed) and D formed by a finalize pass
    int nslice;
    int64_t cslice;
    int32_t *acc;
    int mode;   // 0: whole width, D out; 1: one slice into acc; 2: D (and counts) from acc
};

// bit 7 of each byte set when that byte of v is nonzero (no carries between bytes)
__device__ __forceinline__ uint32_t nz_bytes(uint32_t v) {
    return ((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v;
}

// Bytes c .. c + 15 of a row (the gap byte where the row is absent or past the
// width), as four little-endian words: five aligned words realigned by the
// row's byte offset where all of them lie inside the row, else byte by byte.
__device__ __forceinline__ void pd_load16(const uint8_t *p, int64_t c, int64_t width, uint32_t w[4]) {
    if (p && c + 20 <= width) {
        const uint8_t *q = p + c;
        const uint32_t *al = reinterpret_cast<const uint32_t *>(reinterpret_cast<uintptr_t>(q) & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(q) & 3u);
        uint32_t d[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) d[i] = al[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
        return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t v = 0;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int64_t cc = c + 4 * q + y;
            v |= ((p && cc < width) ? (uint32_t)p[cc] : 255u) << (8 * y);
        }
        w[q] = v;
    }
}

// A workgroup of 256 threads takes one 64 x 64 tile of a group's pairs (and
// one column slice when the tiles are too few to fill the chip); thread
// (ty, tx) counts pairs (4 ty + i, 4 tx + j), i, j < 4.  Each pass stages 64
// columns of the tile's 128 rows in LDS (gap bytes past the width or past the
// group's rows, which count nowhere): per word of four columns, the bytes with
// bit 7 cleared and a mask with bit 7 set in each byte that is not the gap
// (255), read together as one 64-bit word; per row, the 64 columns' non-gap
// bits packed into two words.  Residue codes are below 128, so two residues
// differ exactly where their low seven bits do, and bit 7 of
// ((x ^ y) + 0x7F7F7F7F) marks those bytes without carries between bytes: a
// pair-word costs one xor-add, one three-input and with both masks and one
// popcount-add.  The residue pairs (both bytes not the gap) are counted on the
// packed bits, 32 columns per and and popcount.
template <bool PIPE>
__global__ void __launch_bounds__(256) pdist_kernel(PdArgs a) {
#pragma clang fp contract(off)
    __shared__ uint2 sa[kPdTile * kPdStride], sb[kPdTile * kPdStride];
    __shared__ uint32_t ga[kPdTile * 2], gb[kPdTile * 2];
    // the group and tile of this workgroup (and its column slice)
    int lo = 0, hi = a.ngroups - 1;
    const int64_t t = a.mode == 1 ? blockIdx.x / a.nslice : blockIdx.x;
    const int64_t slice = a.mode == 1 ? blockIdx.x - t * a.nslice : 0;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.groups[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    const PdGroup g = a.groups[lo];
    const int64_t tl = t - g.tile0;
    const int ta = (int)(tl / g.tiles_b), tb = (int)(tl - (int64_t)ta * g.tiles_b);
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    // staging: thread tid loads 16 bytes of row (tid >> 2) of each operand
    const int lr = tid >> 2, part = tid & 3, lb = 16 * part;
    const int ia = ta * kPdTile + lr, ib = tb * kPdTile + lr;
    const uint8_t *pa = ia < g.na ? a.msa + (int64_t)a.rows[g.a0 + ia] * a.width : nullptr;
    const uint8_t *pb = ib < g.nb ? a.msa + (int64_t)a.rows[g.b0 + ib] * a.width : nullptr;
    uint32_t mm[4][4], cc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mm[i][j] = cc[i][j] = 0u;
    const int64_t cbeg = a.mode == 1 ? slice * a.cslice : 0;
    const int64_t cend = a.mode == 1 ? min(a.width, cbeg + a.cslice) : (a.mode == 2 ? 0 : a.width);
    // PIPE (sliced launches, about one workgroup per CU): the next pass's
    // bytes are loaded while this pass compares; otherwise after it, which
    // keeps registers for more resident workgroups (the other workgroups on
    // the CU hide the load latency)
    uint32_t wa[4], wb[4];
    if (PIPE && cbeg < cend) {
        pd_load16(pa, cbeg + lb, a.width, wa);
        pd_load16(pb, cbeg + lb, a.width, wb);
    }
    for (int64_t c0 = cbeg; c0 < cend; c0 += kPdChunk) {
        if (!PIPE) {
            pd_load16(pa, c0 + lb, a.width, wa);
            pd_load16(pb, c0 + lb, a.width, wb);
        }
        __syncthreads();   // the previous pass is done with the staged words
        uint32_t bits_a = 0, bits_b = 0;   // 16 non-gap bits, at 0-3, 8-11, 16-19, 24-27
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t fa = nz_bytes(~wa[q]) & 0x80808080u, fb = nz_bytes(~wb[q]) & 0x80808080u;
            sa[lr * kPdStride + 4 * part + q] = make_uint2(wa[q] & 0x7F7F7F7Fu, fa);
            sb[lr * kPdStride + 4 * part + q] = make_uint2(wb[q] & 0x7F7F7F7Fu, fb);
            bits_a |= fa >> (7 - q);
            bits_b |= fb >> (7 - q);
        }
        // the odd part's bits fill the even part's gaps (any order of the
        // columns' bits serves, the same for both operands)
        const uint32_t na = __shfl_xor(bits_a, 1), nb = __shfl_xor(bits_b, 1);
        if (!(part & 1)) {
            ga[2 * lr + (part >> 1)] = bits_a | (na << 4);
            gb[2 * lr + (part >> 1)] = bits_b | (nb << 4);
        }
        __syncthreads();
        if (PIPE && c0 + kPdChunk < cend) {
            pd_load16(pa, c0 + kPdChunk + lb, a.width, wa);
            pd_load16(pb, c0 + kPdChunk + lb, a.width, wb);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    cc[i][j] += __popc(ga[2 * (4 * ty + i) + h] & gb[2 * (4 * tx + j) + h]);
#pragma unroll 4
        for (int k = 0; k < kPdChunk / 4; ++k) {
            uint2 x[4], y[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                x[i] = sa[(4 * ty + i) * kPdStride + k];
                y[i] = sb[(4 * tx + i) * kPdStride + k];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    mm[i][j] += __popc(((x[i].x ^ y[j].x) + 0x7F7F7F7Fu) & x[i].y & y[j].y);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = ta * kPdTile + 4 * ty + i;
        if (r >= g.na) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int s = tb * kPdTile + 4 * tx + j;
            if (s >= g.nb) continue;
            const int64_t o = g.o + (int64_t)r * g.ld + s;
            if (a.mode == 1) {   // this slice's counts
                if (mm[i][j]) atomicAdd(a.acc + 2 * o, (int)mm[i][j]);
                if (cc[i][j]) atomicAdd(a.acc + 2 * o + 1, (int)cc[i][j]);
                continue;
            }
            if (a.mode == 2) {
                mm[i][j] = (uint32_t)a.acc[2 * o];
                cc[i][j] = (uint32_t)a.acc[2 * o + 1];
            }
            double d = cc[i][j] > 0u ? (double)mm[i][j] / (double)cc[i][j] : 1.0;
            if (g.diag0 && r == s) d = 0.0;
            a.D[o] = d;
            if (a.mism) a.mism[o] = (int32_t)mm[i][j];
            if (a.comp) a.comp[o] = (int32_t)cc[i][j];
        }
    }
}

// A block copied out of a shared distance tile: the sz x sz block at src
// (row stride ld) to the contiguous sz x sz matrix at dst.
struct PdExtract {
    int64_t src, ld, dst;
    int sz;
};

// one workgroup per block
__global__ void __launch_bounds__(256) pd_extract_kernel(double *D, const PdExtract *ex) {
    const PdExtract e = ex[blockIdx.x];
    const int nn = e.sz * e.sz;
    for (int x = threadIdx.x; x < nn; x += blockDim.x) {
        const int r = x / e.sz, c = x - r * e.sz;
        D[e.dst + x] = D[e.src + (int64_t)r * e.ld + c];
    }
}

// label[i] = the first j with the smallest D[i * ld + j], j < nb (one lane per row).
__global__ void __launch_bounds__(256) nearest_kernel(const double *D, int64_t ld, int na, int nb, int32_t *label) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na) return;
    const double *row = D + (int64_t)i * ld;
    double best = row[0];
    int bj = 0;
    for (int j = 1; j < nb; ++j) {
        const double v = row[j];
        if (v < best) {
            best = v;
            bj = j;
        }
    }
    label[i] = bj;
}

// One neighbour-joining problem: n x n matrix D (modified), tree out as
// parent / blen over 2n nodes (leaves first), scratch r, act, id of n.
struct NjGroup {
    int n;
    int64_t d0;     // offset of D in NjArgs::D
    int64_t s0;     // offset of the n-entry scratch
    int64_t t0;     // offset of the tree (2n + 1 entries)
};

struct NjArgs {
    const NjGroup *groups;
    double *D;
    double *r;
    uint8_t *act;
    int32_t *id;
    int32_t *parent;
    double *blen;
    int32_t *nodes;   // per group: node count
};

struct NjBest {
    double q;
    int i, j;
};

__device__ __forceinline__ bool nj_before(const NjBest &x, const NjBest &y) {   // x before y
    if (y.i < 0) return x.i >= 0;
    if (x.i < 0) return false;
    if (x.q < y.q) return true;
    if (y.q < x.q) return false;
    return x.i < y.i || (x.i == y.i && x.j < y.j);
}

constexpr int kNjLdsMax = 6144;   // nodes whose row sums and flags fit in LDS (else global scratch)
constexpr int kNjAhead = 32;      // matrix loads in flight per lane

// LDS bytes of nj_kernel for problems of at most nmax nodes (0: global scratch)
inline size_t nj_lds_bytes(int nmax) { return nmax <= kNjLdsMax ? (size_t)9 * nmax + 8 : 0; }

// One workgroup per problem: each join recomputes the row sums (one lane per
// row, summing its column in slot order, which equals the row bit for bit as
// D is kept symmetric), finds the smallest Q (the matrix spread row-major over
// the lanes, then a workgroup reduction in (Q, i, j) order),
// writes the two branch lengths and updates row and column i for the new
// node, and clears the row of the slot that leaves.  Row sums and active
// flags sit in LDS when the problem fits.
__global__ void __launch_bounds__(1024) nj_kernel(NjArgs a, int lds) {
#pragma clang fp contract(off)
    extern __shared__ double nj_lds[];
    __shared__ NjBest red[32];
    __shared__ int sh_i, sh_j;
    const NjGroup g = a.groups[blockIdx.x];
    const int n = g.n, tid = threadIdx.x, bs = blockDim.x;
    double *D = a.D + g.d0;
    double *r = lds ? nj_lds : a.r + g.s0;
    uint8_t *act = lds ? reinterpret_cast<uint8_t *>(nj_lds + n) : a.act + g.s0;
    int32_t *id = a.id + g.s0;
    int32_t *parent = a.parent + g.t0;
    double *blen = a.blen + g.t0;
    for (int s = tid; s < n; s += bs) {
        act[s] = 1;
        id[s] = s;
    }
    __syncthreads();
    int next = n, m = n;
    while (m > 3) {
        for (int i = tid; i < n; i += bs) {
            if (!act[i]) continue;
            // inactive slots' rows and columns hold +0.0, which leaves the sum
            // (it starts at +0.0 and so is never -0.0) bit for bit: the chain
            // is the sum over the active slots, without branches
            double sum = 0.0;
            for (int k0 = 0; k0 < n; k0 += kNjAhead) {   // column i, kNjAhead loads in flight
                double v[kNjAhead];
#pragma unroll
                for (int u = 0; u < kNjAhead; ++u) v[u] = k0 + u < n ? D[(int64_t)(k0 + u) * n + i] : 0.0;
#pragma unroll
                for (int u = 0; u < kNjAhead; ++u) sum = sum + v[u];
            }
            r[i] = sum;
        }
        __syncthreads();
        const double f = (double)(m - 2);
        NjBest b{0.0, -1, -1};
        // the matrix row-major over all lanes, (i, j) stepped along with
        // the index, kNjAhead loads in flight: pairs j > i of active rows
        {
            const int64_t nn = (int64_t)n * n;
            int i = tid / n, j = tid - (tid / n) * n;
            const int di = bs / n, dj = bs - (bs / n) * n;
            for (int64_t e0 = tid; e0 < nn; e0 += (int64_t)bs * kNjAhead) {
                double v[kNjAhead];
#pragma unroll
                for (int u = 0; u < kNjAhead; ++u) {
                    const int64_t e = e0 + (int64_t)u * bs;
                    v[u] = e < nn ? D[e] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kNjAhead; ++u) {
                    // an inactive slot's sum is -inf: its pairs score +inf and
                    // never come first (an active pair scores finite)
                    if (i < n && j > i) {
                        const NjBest c{f * v[u] - r[i] - r[j], i, j};
                        if (nj_before(c, b)) b = c;
                    }
                    i += di;
                    j += dj;
                    if (j >= n) {
                        j -= n;
                        ++i;
                    }
                }
            }
        }
        // the workgroup's first pair in (Q, i, j) order
        for (int o = 32; o >= 1; o >>= 1) {
            NjBest y{__shfl_xor(b.q, o, 64), __shfl_xor(b.i, o, 64), __shfl_xor(b.j, o, 64)};
            if (nj_before(y, b)) b = y;
        }
        if ((tid & 63) == 0) red[tid >> 6] = b;
        __syncthreads();
        if (tid == 0) {
            NjBest w = red[0];
            for (int x = 1; x < (bs >> 6); ++x)
                if (nj_before(red[x], w)) w = red[x];
            const int bi = w.i, bj = w.j;
            const double dij = D[(int64_t)bi * n + bj];
            const double li = 0.5 * dij + (r[bi] - r[bj]) / (2.0 * f);
            const double lj = dij - li;
            parent[id[bi]] = next;
            blen[id[bi]] = li;
            parent[id[bj]] = next;
            blen[id[bj]] = lj;
            sh_i = bi;
            sh_j = bj;
        }
        __syncthreads();
        const int bi = sh_i, bj = sh_j;
        const double dij = D[(int64_t)bi * n + bj];
        for (int k = tid; k < n; k += bs) {
            if (!act[k] || k == bi || k == bj) continue;
            const double v = (D[(int64_t)bi * n + k] + D[(int64_t)bj * n + k] - dij) * 0.5;
            D[(int64_t)bi * n + k] = v;
            D[(int64_t)k * n + bi] = v;
        }
        __syncthreads();
        // slot j leaves: its row to +0.0 (it enters every other column's
        // sum; column j only enters j's own, which is not kept), its sum to -inf
        for (int k = tid; k < n; k += bs) D[(int64_t)bj * n + k] = 0.0;
        if (tid == 0) {
            act[bj] = 0;
            id[bi] = next;
            r[bj] = -__builtin_inf();
        }
        ++next;
        --m;
        __syncthreads();
    }
    if (tid == 0) {
        int s[3], c = 0;
        for (int i = 0; i < n && c < 3; ++i)
            if (act[i]) s[c++] = i;
        if (m == 3) {
            const double dab = D[(int64_t)s[0] * n + s[1]], dac = D[(int64_t)s[0] * n + s[2]],
                         dbc = D[(int64_t)s[1] * n + s[2]];
            parent[id[s[0]]] = next;
            blen[id[s[0]]] = (dab + dac - dbc) * 0.5;
            parent[id[s[1]]] = next;
            blen[id[s[1]]] = (dab + dbc - dac) * 0.5;
            parent[id[s[2]]] = next;
            blen[id[s[2]]] = (dac + dbc - dab) * 0.5;
            parent[next] = -1;
            blen[next] = 0.0;
            ++next;
        } else if (m == 2) {
            const double dab = D[(int64_t)s[0] * n + s[1]];
            parent[id[s[0]]] = next;
            blen[id[s[0]]] = dab * 0.5;
            parent[id[s[1]]] = next;
            blen[id[s[1]]] = dab * 0.5;
            parent[next] = -1;
            blen[next] = 0.0;
            ++next;
        } else {
            parent[id[s[0]]] = -1;
            blen[id[s[0]]] = 0.0;
        }
        a.nodes[blockIdx.x] = next;
    }
}

// ---- one large problem spread over the chip: three kernels per join ------
// State of the join loop on the device: active nodes, the next node number,
// the pair chosen.
struct NjCtrl {
    int m, next;
};

struct NjBigArgs {
    int n;
    double *D;
    double *r;
    uint8_t *act;
    int32_t *id;
    int32_t *parent;
    double *blen;
    NjBest *part;   // per workgroup of the Q pass
    double *part_d; // D(i, j) of each part's pair
    int nparts;
    NjCtrl *ctrl;
};

__global__ void __launch_bounds__(256) nj_big_init_kernel(NjBigArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.n) {
        a.act[s] = 1;
        a.id[s] = s;
    }
    if (s == 0) *a.ctrl = NjCtrl{a.n, a.n};
}

// row sums: a workgroup per 16 rows i0 .. i0 + 15; its 256 lanes stage the
// columns i0 .. i0 + 15 of 256 rows k at a time in LDS (coalesced, all loads
// in flight together), then lane t < 16 adds column i0 + t in slot order (the
// bits of the row, D being symmetric).  The rows of slots that have left
// hold +0.0 (the join clears them): the sum starts at +0.0 and so is
// never -0.0 (round to nearest gives x + (-x) = +0.0), and adding +0.0 to it
// leaves every bit, so the chain is the sum over the active slots alone and
// runs without flags or branches.
constexpr int kNjRowsCols = 16, kNjRowsChunk = 256;

__global__ void __launch_bounds__(256) nj_big_rows_kernel(NjBigArgs a) {
#pragma clang fp contract(off)
    __shared__ double blk[kNjRowsChunk * kNjRowsCols];
    const int n = a.n, tid = threadIdx.x;
    const int i0 = blockIdx.x * kNjRowsCols;
    const int ci = tid & (kNjRowsCols - 1), kr = tid / kNjRowsCols;   // this lane's column and first row in a chunk
    const int i = i0 + ci;
    double sum = 0.0;
    for (int k0 = 0; k0 < n; k0 += kNjRowsChunk) {
        double v[kNjRowsChunk / 16];
#pragma unroll
        for (int u = 0; u < kNjRowsChunk / 16; ++u) {
            const int k = k0 + kr + 16 * u;
            v[u] = (k < n && i < n) ? a.D[(int64_t)k * n + i] : 0.0;
        }
        __syncthreads();   // the previous chunk's sums are done with blk
#pragma unroll
        for (int u = 0; u < kNjRowsChunk / 16; ++u) blk[(kr + 16 * u) * kNjRowsCols + ci] = v[u];
        __syncthreads();
        if (tid < kNjRowsCols) {
            const int kn = min(kNjRowsChunk, (n - k0 + 15) & ~15);   // rows past n were staged as 0.0
            for (int q0 = 0; q0 < kn; q0 += 16) {
                double t[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) t[q] = blk[(q0 + q) * kNjRowsCols + tid];
#pragma unroll
                for (int q = 0; q < 16; ++q) sum = sum + t[q];
            }
        }
    }
    if (tid < kNjRowsCols && i0 + tid < n && a.act[i0 + tid]) a.r[i0 + tid] = sum;
}

// Q: workgroup b takes elements [b per, (b + 1) per) of the matrix row-major;
// its first (Q, i, j) goes to part[b]
__global__ void __launch_bounds__(256) nj_big_q_kernel(NjBigArgs a) {
#pragma clang fp contract(off)
    __shared__ NjBest red[4];
    __shared__ double redd[4];
    const int n = a.n, tid = threadIdx.x;
    const int64_t nn = (int64_t)n * n, per = (nn + a.nparts - 1) / a.nparts;
    const int64_t e0 = (int64_t)blockIdx.x * per, e1 = min(nn, e0 + per);
    const double f = (double)(a.ctrl->m - 2);
    NjBest b{0.0, -1, -1};
    double bd = 0.0;
    for (int64_t e = e0 + tid; e < e1; e += blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        // a slot that has left has the sum -inf: its pairs score +inf (f D is
        // finite) and never come first, so no flags are read
        if (j <= i) continue;
        const double d = a.D[e], ri = a.r[i], rj = a.r[j];
        const NjBest c{f * d - ri - rj, i, j};
        if (nj_before(c, b)) {
            b = c;
            bd = d;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        NjBest y{__shfl_xor(b.q, o, 64), __shfl_xor(b.i, o, 64), __shfl_xor(b.j, o, 64)};
        const double yd = __shfl_xor(bd, o, 64);
        if (nj_before(y, b)) {
            b = y;
            bd = yd;
        }
    }
    if ((tid & 63) == 0) {
        red[tid >> 6] = b;
        redd[tid >> 6] = bd;
    }
    __syncthreads();
    if (tid == 0) {
        NjBest w = red[0];
        double wd = redd[0];
        for (int x = 1; x < (int)(blockDim.x >> 6); ++x)
            if (nj_before(red[x], w)) {
                w = red[x];
                wd = redd[x];
            }
        a.part[blockIdx.x] = w;
        a.part_d[blockIdx.x] = wd;
    }
}

constexpr int kNjPickAhead = 8;   // parts loaded per lane before comparing (2,048 parts in one batch)

// the join: the first pair over the parts (every part's load in flight before
// the first compare; D(i, j) comes with the pair), lengths, row and column i
// updated, slot j's row cleared to +0.0 and its sum set to -inf for the next
// row sums and Q
__global__ void __launch_bounds__(256) nj_big_join_kernel(NjBigArgs a) {
#pragma clang fp contract(off)
    __shared__ NjBest red[4];
    __shared__ double redd[4];
    const int n = a.n, tid = threadIdx.x;
    NjBest b{0.0, -1, -1};
    double bd = 0.0;
    for (int x0 = 0; x0 < a.nparts; x0 += kNjPickAhead * (int)blockDim.x) {
        NjBest p[kNjPickAhead];
        double pd[kNjPickAhead];
#pragma unroll
        for (int h = 0; h < kNjPickAhead; ++h) {
            const int x = x0 + h * (int)blockDim.x + tid;
            p[h] = x < a.nparts ? a.part[x] : NjBest{0.0, -1, -1};
            pd[h] = x < a.nparts ? a.part_d[x] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < kNjPickAhead; ++h)
            if (nj_before(p[h], b)) {
                b = p[h];
                bd = pd[h];
            }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        NjBest y{__shfl_xor(b.q, o, 64), __shfl_xor(b.i, o, 64), __shfl_xor(b.j, o, 64)};
        const double yd = __shfl_xor(bd, o, 64);
        if (nj_before(y, b)) {
            b = y;
            bd = yd;
        }
    }
    if ((tid & 63) == 0) {
        red[tid >> 6] = b;
        redd[tid >> 6] = bd;
    }
    __syncthreads();
    NjBest w = red[0];
    double dij = redd[0];
    for (int x = 1; x < (int)(blockDim.x >> 6); ++x)
        if (nj_before(red[x], w)) {
            w = red[x];
            dij = redd[x];
        }
    const NjCtrl c = *a.ctrl;
    const int bi = w.i, bj = w.j;
    if (tid == 0) {
        const double f = (double)(c.m - 2);
        const double li = 0.5 * dij + (a.r[bi] - a.r[bj]) / (2.0 * f);
        const double lj = dij - li;
        a.parent[a.id[bi]] = c.next;
        a.blen[a.id[bi]] = li;
        a.parent[a.id[bj]] = c.next;
        a.blen[a.id[bj]] = lj;
    }
    // lane k alone reads and writes entry k of rows i and j and of column i
    // (D(i, j) came with the pair), so clearing row j needs no barrier.  Row
    // j must read +0.0 in the other slots' row sums; column j only enters
    // slot j's own sum, which is not kept, and pairs with j score +inf in Q.
    for (int k = tid; k < n; k += blockDim.x) {
        if (a.act[k] && k != bi && k != bj) {
            const double v = (a.D[(int64_t)bi * n + k] + a.D[(int64_t)bj * n + k] - dij) * 0.5;
            a.D[(int64_t)bi * n + k] = v;
            a.D[(int64_t)k * n + bi] = v;
        }
        a.D[(int64_t)bj * n + k] = 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        a.act[bj] = 0;
        a.id[bi] = c.next;
        a.r[bj] = -__builtin_inf();
        *a.ctrl = NjCtrl{c.m - 1, c.next + 1};
    }
}

__global__ void nj_big_finish_kernel(NjBigArgs a, int32_t *nodes) {
#pragma clang fp contract(off)
    const int n = a.n;
    const NjCtrl c = *a.ctrl;
    int next = c.next;
    int s[3], k = 0;
    for (int i = 0; i < n && k < 3; ++i)
        if (a.act[i]) s[k++] = i;
    const double *D = a.D;
    if (c.m == 3) {
        const double dab = D[(int64_t)s[0] * n + s[1]], dac = D[(int64_t)s[0] * n + s[2]],
                     dbc = D[(int64_t)s[1] * n + s[2]];
        a.parent[a.id[s[0]]] = next;
        a.blen[a.id[s[0]]] = (dab + dac - dbc) * 0.5;
        a.parent[a.id[s[1]]] = next;
        a.blen[a.id[s[1]]] = (dab + dbc - dac) * 0.5;
        a.parent[a.id[s[2]]] = next;
        a.blen[a.id[s[2]]] = (dac + dbc - dab) * 0.5;
        a.parent[next] = -1;
        a.blen[next] = 0.0;
        ++next;
    } else if (c.m == 2) {
        const double dab = D[(int64_t)s[0] * n + s[1]];
        a.parent[a.id[s[0]]] = next;
        a.blen[a.id[s[0]]] = dab * 0.5;
        a.parent[a.id[s[1]]] = next;
        a.blen[a.id[s[1]]] = dab * 0.5;
        a.parent[next] = -1;
        a.blen[next] = 0.0;
        ++next;
    } else {
        a.parent[a.id[s[0]]] = -1;
        a.blen[a.id[s[0]]] = 0.0;
    }
    *nodes = next;
}

}  // namespace hk
