// Learned center proposer: 3-mer features, a BF16 MLP on MFMA (FP32
// accumulation), its backward, Adam, candidate scores and top-k.
//
// The paper picks the center as the sequence most similar to all others; the
// exhaustive search is O(N^2) SW alignments.  The proposer maps each
// sequence to an embedding e so that e_a . e_b approximates SW(a, b) / 100;
// u_i = e_i . (sum_j e_j - e_i) then approximates sum_j SW(i, j) / 100, and
// its top candidates are judged exactly.
//
// All reductions run in a fixed order (no float atomics), so every result is
// run-to-run deterministic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int kFeat = 8000, kHid = 256, kEmb = 64;

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// X[r][400a + 20b + c] = count of the 3-mer abc (all codes < 20) in sequence
// rows[r] (rows == null: r), as bf16 bits.  One workgroup per row, counts in LDS.
__global__ void __launch_bounds__(256)
featurize_kernel(const uint8_t *res, const int64_t *off, const int32_t *rows, int nrows, uint16_t *X) {
    __shared__ int cnt[kFeat];
    const int r = blockIdx.x;
    if (r >= nrows) return;
    const int k = rows ? rows[r] : r;
    const uint8_t *s = res + off[k];
    const int n = (int)(off[k + 1] - off[k]);
    for (int x = threadIdx.x; x < kFeat; x += 256) cnt[x] = 0;
    __syncthreads();
    for (int p = threadIdx.x; p + 2 < n; p += 256) {
        const int a = s[p], b = s[p + 1], c = s[p + 2];
        if (a < 20 && b < 20 && c < 20) atomicAdd(&cnt[400 * a + 20 * b + c], 1);
    }
    __syncthreads();
    uint16_t *row = X + (int64_t)r * kFeat;
    for (int x = threadIdx.x; x < kFeat / 8; x += 256) {
        uint32_t w[4];
#pragma unroll
        for (int y = 0; y < 4; ++y)
            w[y] = (uint32_t)f2bf((float)cnt[8 * x + 2 * y]) | ((uint32_t)f2bf((float)cnt[8 * x + 2 * y + 1]) << 16);
        reinterpret_cast<uint4 *>(row)[x] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

__global__ void iota_kernel(int32_t *p, int n) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = x;
}

__global__ void gather_f32_kernel(const float *src, const int32_t *idx, int n, float *dst) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) dst[x] = src[idx[x]];
}

// Gather rows of a bf16 matrix: dst[r] = src[idx[r]] (width in elements).
__global__ void gather_rows_kernel(const uint16_t *src, const int32_t *idx, int nrows, int width, uint16_t *dst) {
    const int r = blockIdx.x;
    if (r >= nrows) return;
    const uint16_t *s = src + (int64_t)idx[r] * width;
    uint16_t *d = dst + (int64_t)r * width;
    for (int x = threadIdx.x; x < width; x += blockDim.x) d[x] = s[x];
}

// ---------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] . op(B)[K x N] on v_mfma_f32_32x32x16_bf16.
//   op(A)(m, k) = TA ? A[k*lda + m] : A[m*lda + k]
//   op(B)(k, n) = TB ? B[n*ldb + k] : B[k*ldb + n]
// Workgroup tile 64 x 64, four waves of 32 x 32, K staged through LDS in 32s
// (k contiguous for both operands).  Epilogues:
//   0: C = acc (+ bias[n])
//   1: C = acc + bias[n] (pre-activation), Hb = bf16(relu(C))
//   2: D = acc * (Hpre > 0) (relu backward), Db = bf16(D)
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

struct GemmArgs {
    const uint16_t *A;
    const uint16_t *B;
    int M, N, K, lda, ldb;
    float *C;
    int ldc;
    const float *bias;
    uint16_t *Cb;          // bf16 output (epilogues 1, 2)
    int ldcb;
    const float *Hpre;     // epilogue 2 mask source
    int ldh;
};

constexpr int kBK = 32, kLdsK = kBK + 8;

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256)
gemm_bf16_kernel(GemmArgs g) {
    __shared__ uint16_t As[64][kLdsK];
    __shared__ uint16_t Bs[64][kLdsK];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x16_t acc;
#pragma unroll
    for (int x = 0; x < 16; ++x) acc[x] = 0.f;
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        // stage A (64 x 32) and B (32 x 64): 8 elements per thread each
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int q = tid * 8 + e;           // 0 .. 2047
            int mm, kk;
            if (TA) { kk = q >> 6; mm = q & 63; }   // consecutive threads walk m (contiguous in memory)
            else { mm = q >> 5; kk = q & 31; }      // consecutive threads walk k
            const int gm = m0 + mm, gk = k0 + kk;
            uint16_t v = 0;
            if (gm < g.M && gk < g.K) v = TA ? g.A[(int64_t)gk * g.lda + gm] : g.A[(int64_t)gm * g.lda + gk];
            As[mm][kk] = v;
            int nn;
            if (TB) { nn = q >> 5; kk = q & 31; }
            else { kk = q >> 6; nn = q & 63; }
            const int gn = n0 + nn, gk2 = k0 + kk;
            uint16_t w = 0;
            if (gn < g.N && gk2 < g.K) w = TB ? g.B[(int64_t)gn * g.ldb + gk2] : g.B[(int64_t)gk2 * g.ldb + gn];
            Bs[nn][kk] = w;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            const uint4 av = *reinterpret_cast<const uint4 *>(&As[wm + (lane & 31)][kk]);
            const uint4 bv = *reinterpret_cast<const uint4 *>(&Bs[wn + (lane & 31)][kk]);
            bf16x8_t a8, b8;
            __builtin_memcpy(&a8, &av, 16);
            __builtin_memcpy(&b8, &bv, 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b8, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[x]: row (x/4)*8 + (lane/32)*4 + x%4, column lane%32 of the wave tile
    const int gn = n0 + wn + (lane & 31);
    if (gn >= g.N) return;
#pragma unroll
    for (int x = 0; x < 16; ++x) {
        const int gm = m0 + wm + (x >> 2) * 8 + (lane >> 5) * 4 + (x & 3);
        if (gm >= g.M) continue;
        float v = acc[x];
        if (EPI == 0) {
            if (g.bias) v += g.bias[gn];
            g.C[(int64_t)gm * g.ldc + gn] = v;
        } else if (EPI == 1) {
            v += g.bias ? g.bias[gn] : 0.f;
            if (g.C) g.C[(int64_t)gm * g.ldc + gn] = v;
            g.Cb[(int64_t)gm * g.ldcb + gn] = f2bf(v > 0.f ? v : 0.f);
        } else {
            const float z = g.Hpre[(int64_t)gm * g.ldh + gn];
            const float d = z > 0.f ? v : 0.f;
            g.C[(int64_t)gm * g.ldc + gn] = d;
            g.Cb[(int64_t)gm * g.ldcb + gn] = f2bf(d);
        }
    }
}

// Column sums in a fixed order: partial sums over row blocks of 1024, then
// the partials in block order.
__global__ void colsum_partial_kernel(const float *A, int rows, int cols, int lda, float *part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const int r0 = blockIdx.y * 1024, r1 = min(rows, r0 + 1024);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += A[(int64_t)r * lda + c];
    part[(int64_t)blockIdx.y * cols + c] = s;
}
__global__ void colsum_final_kernel(const float *part, int nblk, int cols, float *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * cols + c];
    out[c] = s;
}

// Pair loss: pairs (r, r + P).  dE (fp32) and its bf16 copy; per-pair squared
// errors go to sq[P] for a fixed-order loss reduction.
__global__ void pair_loss_kernel(const float *E, const float *target, int P, float *dE, uint16_t *dEb, float *sq) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P) return;
    const float *a = E + (int64_t)r * kEmb, *b = E + (int64_t)(r + P) * kEmb;
    float pred = 0.f;
    for (int d = 0; d < kEmb; ++d) pred += a[d] * b[d];
    const float diff = pred - target[r];
    sq[r] = diff * diff;
    const float gsc = 2.f * diff / (float)P;
    float *da = dE + (int64_t)r * kEmb, *db = dE + (int64_t)(r + P) * kEmb;
    uint16_t *dab = dEb + (int64_t)r * kEmb, *dbb = dEb + (int64_t)(r + P) * kEmb;
    for (int d = 0; d < kEmb; ++d) {
        const float ga = gsc * b[d], gb = gsc * a[d];
        da[d] = ga;
        db[d] = gb;
        dab[d] = f2bf(ga);
        dbb[d] = f2bf(gb);
    }
}

// out[0] = sum(v[0..n)) / n in a fixed order (one workgroup).
__global__ void __launch_bounds__(256) mean_kernel(const float *v, int n, float *out) {
    __shared__ float part[256];
    float s = 0.f;
    const int per = (n + 255) / 256;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    for (int x = lo; x < hi; ++x) s += v[x];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int x = 0; x < 256; ++x) t += part[x];
        out[0] = n > 0 ? t / (float)n : 0.f;
    }
}

// Pair loss with a per-group term: groups of K consecutive pairs (K <= 64,
// one wavefront per group), loss = mean(diff^2) + lam * mean over groups of
// (mean diff of the group)^2.  dpred = 2 diff / P + 2 lam gmean / (G K).
__global__ void __launch_bounds__(64) pair_group_loss_kernel(const float *E, const float *target, int P, int K,
                                                             float lam, float *dE, uint16_t *dEb, float *sq,
                                                             float *gsq) {
    const int g = blockIdx.x, l = threadIdx.x;
    const int G = P / K;
    const int r = g * K + l;
    float diff = 0.f, pred = 0.f;
    const float *a = E + (int64_t)r * kEmb, *b = E + (int64_t)(r + P) * kEmb;
    if (l < K) {
        for (int d = 0; d < kEmb; ++d) pred += a[d] * b[d];
        diff = pred - target[r];
        sq[r] = diff * diff;
    }
    float sum = diff;   // fixed-order tree over the wavefront
    for (int sh = 32; sh > 0; sh >>= 1) sum += __shfl_xor(sum, sh);
    const float gm = sum / (float)K;
    if (l == 0) gsq[g] = gm * gm;
    if (l >= K) return;
    const float gsc = 2.f * diff / (float)P + 2.f * lam * gm / ((float)G * (float)K);
    float *da = dE + (int64_t)r * kEmb, *db = dE + (int64_t)(r + P) * kEmb;
    uint16_t *dab = dEb + (int64_t)r * kEmb, *dbb = dEb + (int64_t)(r + P) * kEmb;
    for (int d = 0; d < kEmb; ++d) {
        const float ga = gsc * b[d], gb = gsc * a[d];
        da[d] = ga;
        db[d] = gb;
        dab[d] = f2bf(ga);
        dbb[d] = f2bf(gb);
    }
}

// out[0] = mean(v[0..n)) + lam * mean(w[0..m)), each sum in a fixed order.
__global__ void __launch_bounds__(256) mean2_kernel(const float *v, int n, const float *w, int m, float lam,
                                                    float *out) {
    __shared__ float part[256];
    float res = 0.f;
    for (int which = 0; which < 2; ++which) {
        const float *x = which ? w : v;
        const int c = which ? m : n;
        float s = 0.f;
        const int per = (c + 255) / 256;
        const int lo = min(c, (int)threadIdx.x * per), hi = min(c, lo + per);
        for (int q = lo; q < hi; ++q) s += x[q];
        part[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int q = 0; q < 256; ++q) t += part[q];
            res += (which ? lam : 1.f) * (c > 0 ? t / (float)c : 0.f);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = res;
}

// Adam with bias correction on fp32 masters; optional bf16 copy.
__global__ void adam_kernel(float *p, const float *gr, float *m, float *v, uint16_t *pb, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const float gx = gr[x];
        const float mx = b1 * m[x] + (1.f - b1) * gx;
        const float vx = b2 * v[x] + (1.f - b2) * gx * gx;
        m[x] = mx;
        v[x] = vx;
        const float mh = mx / c1, vh = vx / c2;
        const float px = p[x] - lr * mh / (sqrtf(vh) + eps);
        p[x] = px;
        if (pb) pb[x] = f2bf(px);
    }
}

// exponential moving average of parameters: e = d * e + (1 - d) * p
__global__ void ema_kernel(const float *p, float *e, int64_t n, float d) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        e[x] = d * e[x] + (1.f - d) * p[x];
}

__global__ void f32_to_bf16_kernel(const float *src, uint16_t *dst, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        dst[x] = f2bf(src[x]);
}

// targets: t[q] = score[q] / 100
__global__ void scale_targets_kernel(const int32_t *score, int n, float *t) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) t[q] = (float)score[q] / 100.f;
}

// u_i = e_i . (S - e_i) with S = sum_j e_j
__global__ void center_score_kernel(const float *E, const float *S, int n, float *u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *e = E + (int64_t)i * kEmb;
    float a = 0.f, b = 0.f;
    for (int d = 0; d < kEmb; ++d) { a += e[d] * S[d]; b += e[d] * e[d]; }
    const float r = a - b;
    u[i] = (r == r) ? r : -3.0e38f;   // NaN sorts last
}

// Top-k (largest first, ties to the lower index) by k rounds of block argmax.
// Pass 1: each workgroup reduces `chunk` entries of (val, idx) to its top k;
// pass 2 runs the same kernel over the partial results.
__device__ __forceinline__ bool topk_better(float v, int i, float w, int j) {
    return v > w || (v == w && i < j);
}
constexpr int kTopkChunk = 4096;
__global__ void __launch_bounds__(256)
topk_kernel(const float *val, const int32_t *idx, int n, int k, float *oval, int32_t *oidx) {
    __shared__ float sv[kTopkChunk];
    __shared__ int si[kTopkChunk];
    __shared__ float rv[256];
    __shared__ int ri[256], rp[256];
    const int base = blockIdx.x * kTopkChunk;
    const int cnt = min(kTopkChunk, n - base);
    for (int x = threadIdx.x; x < kTopkChunk; x += 256) {
        sv[x] = x < cnt ? val[base + x] : -3.4e38f;
        si[x] = x < cnt ? (idx ? idx[base + x] : base + x) : 0x7fffffff;
    }
    __syncthreads();
    for (int r = 0; r < k; ++r) {
        float bv = -3.4e38f;
        int bi = 0x7fffffff, bp = -1;
        for (int x = threadIdx.x; x < kTopkChunk; x += 256)
            if (si[x] != 0x7fffffff && topk_better(sv[x], si[x], bv, bi)) { bv = sv[x]; bi = si[x]; bp = x; }
        rv[threadIdx.x] = bv;
        ri[threadIdx.x] = bi;
        rp[threadIdx.x] = bp;
        __syncthreads();
        for (int d = 128; d > 0; d >>= 1) {
            if ((int)threadIdx.x < d && topk_better(rv[threadIdx.x + d], ri[threadIdx.x + d], rv[threadIdx.x], ri[threadIdx.x])) {
                rv[threadIdx.x] = rv[threadIdx.x + d];
                ri[threadIdx.x] = ri[threadIdx.x + d];
                rp[threadIdx.x] = rp[threadIdx.x + d];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            oval[blockIdx.x * k + r] = rv[0];
            oidx[blockIdx.x * k + r] = ri[0];
            if (rp[0] >= 0) si[rp[0]] = 0x7fffffff;   // taken
        }
        __syncthreads();
    }
}

}  // namespace hk
