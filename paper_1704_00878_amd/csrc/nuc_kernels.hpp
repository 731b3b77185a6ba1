// Nucleotide center star for gfx950 (Methods, trie section): the center's
// segments of k bases are indexed, each sequence is scanned for them, the
// largest co-linear chain of non-overlapping matches becomes its anchors, and
// only the stretches between anchors are aligned (end to end, affine gaps).
//
// The paper indexes the segments in a trie with failure links, which reports
// every occurrence of every segment in one left-to-right pass.  Here the same
// set of occurrences comes from a hash table of the segments' 2-bit packed
// strings (one probe per position of the sequence); the table sits in LDS.
//
// One lane per sequence throughout: sequences are many and their work is
// sequential (a scan, a chain, small dynamic programs), so lanes, not
// cooperative tiles, carry the parallelism.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int kNucNeg = -(1 << 29);

struct NucArgs {
    const uint8_t *res;       // residue codes (0..3 = A C G T, 4 = other)
    const int64_t *off;       // [N + 1]
    int nseq;
    const uint8_t *center;    // the center's codes
    int m, k;
    // segment table: T slots (power of two), key (2-bit packed string) and
    // segment index (-1 = empty); segscore[q] = sum of S over segment q
    const unsigned long long *tkey;
    const int32_t *tseg;
    int lg_t;
    const int32_t *segscore;
    const int8_t *mat;        // alpha x alpha scores
    int alpha, go, ge;
    // count pass: nmatch[x]; chain pass: matches of x at moff[x] ..
    int32_t *nmatch;
    const int64_t *moff;
    int32_t *mq, *mp, *mbest, *mpred;   // per match
    int32_t *tails;           // per sequence: moff[x] + x .. (count + 1 entries): chain
    int32_t *nchain;          // [N] anchors of x
    int64_t *rowlen;          // [N] largest stretch width + 1 (row buffer entries)
    int64_t *codelen;         // [N] code words of the largest stretch of x
    // align pass: scratch at rowoff[x] (int2 entries) and codeoff[x] (words)
    const int64_t *rowoff, *codeoff;
    int2 *rows;
    uint32_t *codes;
    int32_t *score;           // [N]
    uint16_t *ins;            // [N][m + 1] (zeroed)
    uint32_t *aligned;        // [N][aw] (zeroed)
    int aw;
    int32_t *G;               // optional merge: max of ins over the sequences
    int gskip;                // sequence kept out of G
};

__device__ __forceinline__ uint32_t nuc_hash(unsigned long long key, int lg_t) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - lg_t));
}

// segment q whose packed string is key, or -1
__device__ __forceinline__ int nuc_lookup(const unsigned long long *tk, const int32_t *ts, int lg_t,
                                          unsigned long long key) {
    const uint32_t mask = (1u << lg_t) - 1u;
    uint32_t h = nuc_hash(key, lg_t);
    for (;;) {
        const int q = ts[h];
        if (q < 0) return -1;
        if (tk[h] == key) return q;
        h = (h + 1) & mask;
    }
}

// Scan of sequence x for the indexed segments: fn(q, p) for every match, in
// order of p.  Bytes come four at a time from aligned words (a word holding
// a byte of the sequence never leaves its page).
template <class Fn>
__device__ __forceinline__ void nuc_scan(const uint8_t *s, int n, int k, const unsigned long long *tk,
                                         const int32_t *ts, int lg_t, Fn fn) {
    const unsigned long long kmask = k >= 32 ? ~0ull : ((1ull << (2 * k)) - 1ull);
    const uintptr_t a0 = (uintptr_t)s;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(a0 & ~(uintptr_t)3);
    const int sh0 = (int)(a0 & 3);
    unsigned long long key = 0;
    int valid = 0;
    uint32_t word = n > 0 ? w[0] : 0u;
    for (int j = 0; j < n; ++j) {
        const int at = sh0 + j;
        if (j > 0 && (at & 3) == 0) word = w[at >> 2];
        const uint32_t b = (word >> (8 * (at & 3))) & 0xffu;
        if (b > 3) {
            valid = 0;
            continue;
        }
        key = ((key << 2) | b) & kmask;
        if (++valid >= k) {
            const int q = nuc_lookup(tk, ts, lg_t, key);
            if (q >= 0) fn(q, j - k + 1);
        }
    }
}

// Table in LDS when it fits (48 KiB), else read from global memory.
constexpr int kNucLdsSlots = 4096;

#define NUC_TABLE_SETUP                                                                  \
    __shared__ unsigned long long s_tk[kNucLdsSlots];                                    \
    __shared__ int32_t s_ts[kNucLdsSlots];                                               \
    const int T = 1 << a.lg_t;                                                           \
    const bool tl = T <= kNucLdsSlots;                                                   \
    if (tl)                                                                              \
        for (int x = threadIdx.x; x < T; x += blockDim.x) {                              \
            s_tk[x] = a.tkey[x];                                                         \
            s_ts[x] = a.tseg[x];                                                         \
        }                                                                                \
    __syncthreads();                                                                     \
    const unsigned long long *tk = tl ? s_tk : a.tkey;                                   \
    const int32_t *ts = tl ? s_ts : a.tseg;

// First pass: matches per sequence.
__global__ void __launch_bounds__(256) nuc_count_kernel(NucArgs a) {
    NUC_TABLE_SETUP
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nseq) return;
    const int64_t so = a.off[x];
    int cnt = 0;
    nuc_scan(a.res + so, (int)(a.off[x + 1] - so), a.k, tk, ts, a.lg_t, [&](int, int) { ++cnt; });
    a.nmatch[x] = cnt;
}

// Second pass: the matches again, stored, and the anchor chain.  Matches come
// in order of p.  A match is inserted into the chain table once p_i >= p_j + k
// for the match i being queried; tails[L] is the inserted match of chain
// length L with the smallest (q, p) (q increases with L).  A query takes the
// longest L whose tail has q < q_i: best = L + 1, predecessor = tails[L].
// Then the stretch sizes: the row buffer of the widest stretch and the codes
// of the largest (the stretches take turns in the scratch).
__global__ void __launch_bounds__(256) nuc_chain_kernel(NucArgs a) {
    NUC_TABLE_SETUP
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nseq) return;
    const int64_t so = a.off[x];
    const int n = (int)(a.off[x + 1] - so);
    const int k = a.k;
    const int64_t mb = a.moff[x];
    int32_t *mq = a.mq + mb, *mp = a.mp + mb, *mbest = a.mbest + mb, *mpred = a.mpred + mb;
    int32_t *tails = a.tails + mb + x;   // entries 1 .. count
    int cnt = 0, L = 0, ins_next = 0;
    int lastq = -1;                     // q of tails[L]
    auto insert = [&](int j) __attribute__((always_inline)) {
        const int bj = mbest[j];
        if (bj > L) {
            tails[bj] = j;
            L = bj;
            lastq = mq[j];
        } else if (mq[j] < mq[tails[bj]]) {
            tails[bj] = j;
            if (bj == L) lastq = mq[j];
        }
    };
    nuc_scan(a.res + so, n, k, tk, ts, a.lg_t, [&](int q, int p) {
        while (ins_next < cnt && mp[ins_next] + k <= p) insert(ins_next++);
        int lq = 0;
        if (L > 0 && lastq < q) {
            lq = L;
        } else {
            int lo = 1, hi = L;   // largest l in [1, L] with q(tails[l]) < q
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                if (mq[tails[mid]] < q) { lq = mid; lo = mid + 1; }
                else hi = mid - 1;
            }
        }
        mq[cnt] = q;
        mp[cnt] = p;
        mbest[cnt] = lq + 1;
        mpred[cnt] = lq > 0 ? tails[lq] : -1;
        ++cnt;
    });
    while (ins_next < cnt) insert(ins_next++);
    // the chain, in order, into tails[0 .. L-1] (tails[L] is its last match)
    int e = L > 0 ? tails[L] : -1;
    for (int t = L - 1; t >= 0; --t) {
        tails[t] = e;
        e = mpred[e];
    }
    a.nchain[x] = L;
    // stretch sizes: before the first anchor, between anchors, after the last
    // (one stretch at a time reuses the scratch, so the largest counts)
    int64_t words = 0;
    int wmax = 0, ci = 0, sj = 0;
    for (int t = 0; t <= L; ++t) {
        const int qc = t < L ? mq[tails[t]] * k : a.m;
        const int ps = t < L ? mp[tails[t]] : n;
        const int dc = qc - ci, ds = ps - sj;
        words = max(words, (int64_t)dc * ((ds + 7) >> 3));
        wmax = max(wmax, ds);
        ci = qc + k;
        sj = ps + k;
    }
    a.rowlen[x] = wmax + 1;
    a.codelen[x] = words;
}

// Third pass: every stretch aligned end to end (Gotoh's global form,
// H(0,0) = 0, H(i,0) = F(i,0) = -(go + ge*i), H(0,j) = E(0,j) = -(go + ge*j)),
// codes per cell (bit 0 diagonal not taken, 1 E not taken, 2 E extended, 3 F
// extended), then the traceback with the local alignment's priorities into
// the center-star vector; anchors are aligned as they stand.
__global__ void __launch_bounds__(256) nuc_align_kernel(NucArgs a) {
    __shared__ int8_t smat[32 * 32];
    for (int x = threadIdx.x; x < 1024; x += blockDim.x) {
        const int r = x >> 5, q = x & 31;
        smat[x] = (r < a.alpha && q < a.alpha) ? a.mat[r * a.alpha + q] : (int8_t)0;
    }
    __syncthreads();
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.nseq) return;
    const int64_t so = a.off[x];
    const uint8_t *s = a.res + so;
    const uint8_t *c = a.center;
    const int n = (int)(a.off[x + 1] - so);
    const int m = a.m, k = a.k, go = a.go, ge = a.ge, goe = go + ge;
    const int64_t mb = a.moff[x];
    const int32_t *mq = a.mq + mb, *mp = a.mp + mb;
    const int32_t *chain = a.tails + mb + x;
    const int L = a.nchain[x];
    int2 *row = a.rows + a.rowoff[x];
    uint32_t *code0 = a.codes + a.codeoff[x];
    uint16_t *ins = a.ins + (int64_t)x * (m + 1);
    uint32_t *al = a.aligned + (int64_t)x * a.aw;
    int32_t *gmax = (a.G && x != a.gskip) ? a.G : nullptr;
    int total = 0;
    int ci = 0, sj = 0;
    for (int t = 0; t <= L; ++t) {
        const int qc = t < L ? mq[chain[t]] * k : m;
        const int ps = t < L ? mp[chain[t]] : n;
        const int dc = qc - ci, ds = ps - sj;
        const int cw = (ds + 7) >> 3;   // code words per row
        const uint8_t *cc = c + ci, *ss = s + sj;
        // forward: row buffer holds (H, F) of the row above
        for (int j = 0; j <= ds; ++j) row[j] = make_int2(j == 0 ? 0 : -(go + ge * j), kNucNeg);
        for (int i = 1; i <= dc; ++i) {
            const int cr = cc[i - 1] * 32;
            int hdiag = row[0].x;
            int hleft = -(go + ge * i), eleft = kNucNeg;
            row[0] = make_int2(hleft, hleft);
            uint32_t *crow = code0 + (int64_t)(i - 1) * cw;
            uint32_t word = 0;
            for (int j = 1; j <= ds; ++j) {
                const int2 up = row[j];
                const int e = max(eleft - ge, hleft - goe);
                const int f = max(up.y - ge, up.x - goe);
                const int d = hdiag + smat[cr + ss[j - 1]];
                const int h = max(d, max(e, f));
                const uint32_t nib = (uint32_t)(h != d) | ((uint32_t)(h != e) << 1) |
                                     ((uint32_t)(eleft - ge > hleft - goe) << 2) |
                                     ((uint32_t)(up.y - ge > up.x - goe) << 3);
                word |= nib << (4 * ((j - 1) & 7));
                if (((j - 1) & 7) == 7 || j == ds) {
                    crow[(j - 1) >> 3] = word;
                    word = 0;
                }
                hdiag = up.x;
                row[j] = make_int2(h, f);
                hleft = h;
                eleft = e;
            }
        }
        total += row[ds].x;   // H(dc, ds): the last row written (row 0 when dc = 0)
        // traceback from (dc, ds) to (0, 0)
        int i = dc, j = ds, st = 0;   // 0 H, 1 E, 2 F
        int slot = -1, scount = 0;
        auto flush = [&]() __attribute__((always_inline)) {
            if (slot >= 0) {
                ins[slot] = (uint16_t)scount;
                if (gmax) atomicMax(gmax + slot, scount);
            }
        };
        while (i > 0 || j > 0) {
            const uint32_t nib = (i > 0 && j > 0)
                                     ? (code0[(int64_t)(i - 1) * cw + ((j - 1) >> 3)] >> (4 * ((j - 1) & 7))) & 15u
                                     : 0u;
            if (st == 0) {
                if (i > 0 && j > 0) {
                    if (!(nib & 1u)) {
                        const int p = ci + i - 1;
                        atomicOr(al + (p >> 5), 1u << (p & 31));
                        --i;
                        --j;
                    } else {
                        st = (nib & 2u) ? 2 : 1;
                    }
                } else {
                    st = i == 0 ? 1 : 2;
                }
            } else if (st == 1) {
                // s_j after center position ci + i: slot ci + i
                const int sl = ci + i;
                if (sl != slot) {
                    flush();
                    slot = sl;
                    scount = 0;
                }
                ++scount;
                const bool ext = (i > 0) ? (nib & 4u) != 0 : (j > 1 && go > 0);
                --j;
                if (!ext) st = 0;
            } else {
                const bool ext = (j > 0) ? (nib & 8u) != 0 : (i > 1 && go > 0);
                --i;
                if (!ext) st = 0;
            }
        }
        flush();
        if (t < L) {
            // the anchor: k center positions aligned, its matches scored
            for (int u = 0; u < k; ++u) {
                const int p = qc + u;
                atomicOr(al + (p >> 5), 1u << (p & 31));
            }
            total += a.segscore[mq[chain[t]]];
            ci = qc + k;
            sj = ps + k;
        }
    }
    a.score[x] = total;
}

#undef NUC_TABLE_SETUP

// Exclusive prefix sums of n int64 values (one workgroup of 1024 lanes, each
// a contiguous chunk), and the total.
__global__ void __launch_bounds__(1024) scan_i64_kernel(const int64_t *in, int n, int64_t add, int64_t *out,
                                                         int64_t *total) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int lo = min(n, tid * per), hi = min(n, lo + per);
    int64_t sum = 0;
    for (int p = lo; p < hi; ++p) sum += in[p] + add;
    part[tid] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t acc = tid > 0 ? part[tid - 1] : 0;
    for (int p = lo; p < hi; ++p) {
        out[p] = acc;
        acc += in[p] + add;
    }
    if (tid == 1023) *total = part[1023];
}

// int32 counts to int64 (for the scan)
__global__ void widen_kernel(const int32_t *in, int n, int64_t *out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) out[x] = in[x];
}

}  // namespace hk
