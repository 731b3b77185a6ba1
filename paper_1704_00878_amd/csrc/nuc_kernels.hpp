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
// Lanes, not cooperative tiles, carry the parallelism: sequences are many and
// their work is sequential (a scan, a chain, small dynamic programs).  The
// scan takes one lane per chunk of match starts, the chain one workgroup per
// sequence (its matches staged in LDS), each stretch one lane.
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
    // scan chunks: sequence x owns chunks cbase[x] .. cbase[x+1]-1, chunk c of
    // x holding the match starts p in [c * kNucChunk, (c + 1) * kNucChunk)
    const int64_t *cbase;     // [N + 1]
    int64_t nchunk;
    int32_t *ccount;          // [nchunk] matches per chunk
    const int64_t *cmoff;     // [nchunk + 1] first match of each chunk
    int32_t *mq, *mp, *mbest, *mpred;   // per match, in order of p per sequence
    // per sequence x, slots base(x) = cmoff[cbase[x]] + x .. + count_x:
    // chain table, then the chain; and one stretch per slot
    int32_t *tails;
    int4 *sdesc;              // per slot: center start, center length (-1: none), sequence start, its length
    int32_t *sseq;            // per slot: the sequence
    int64_t *srow, *scode;    // per slot: row buffer entries, code words
    const int64_t *srowoff, *scodeoff;
    int64_t nslot;
    int2 *rows;
    uint32_t *codes;
    int32_t *score;           // [N]
    uint16_t *ins;            // [N][m + 1] (zeroed)
    uint32_t *aligned;        // [N][aw] (zeroed)
    int aw;
    int32_t *G;               // optional merge: max of ins over the sequences
    int gskip;                // sequence kept out of G
    int chain_cap;            // matches per sequence chained in LDS (<= kChainLdsMax)
};

constexpr int kNucChunk = 256;   // match starts per scan lane

// The table's hash of a packed segment (the host fills the table with it).
__host__ __device__ __forceinline__ uint32_t nuc_hash(unsigned long long key, int lg_t) {
    const uint32_t h = (uint32_t)key ^ (uint32_t)(key >> 32) * 0x85EBCA6Bu;
    return (h * 0x9E3779B1u) >> (32 - lg_t);
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

// The chunk of scan lane g: its sequence x (binary search over cbase) and
// chunk c within it.  Returns false past the last chunk.
__device__ __forceinline__ bool nuc_chunk(const NucArgs &a, int64_t g, int &x, int &c) {
    if (g >= a.nchunk) return false;
    int lo = 0, hi = a.nseq - 1;   // last x with cbase[x] <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.cbase[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    x = lo;
    c = (int)(g - a.cbase[x]);
    return true;
}

// fn(q, p) for every match with start p in chunk c of sequence x, in order
// of p.  Bytes come four at a time from aligned words (a word holding a byte
// of the sequence never leaves its page).
template <class Fn>
__device__ __forceinline__ void nuc_scan_chunk(const NucArgs &a, const unsigned long long *tk, const int32_t *ts,
                                               int x, int c, Fn fn) {
    const int64_t so = a.off[x];
    const int n = (int)(a.off[x + 1] - so);
    const int k = a.k;
    const int p0 = c * kNucChunk, j1 = min(n, p0 + kNucChunk + k - 1);
    const unsigned long long kmask = k >= 32 ? ~0ull : ((1ull << (2 * k)) - 1ull);
    const uintptr_t a0 = (uintptr_t)(a.res + so + p0);
    const uint32_t *w = reinterpret_cast<const uint32_t *>(a0 & ~(uintptr_t)3);
    const int sh0 = (int)(a0 & 3);
    unsigned long long key = 0;
    int valid = 0;
    uint32_t word = p0 < j1 ? w[0] : 0u;
    for (int j = p0; j < j1; ++j) {
        const int at = sh0 + (j - p0);
        if (j > p0 && (at & 3) == 0) word = w[at >> 2];
        const uint32_t b = (word >> (8 * (at & 3))) & 0xffu;
        if (b > 3) {
            valid = 0;
            continue;
        }
        key = ((key << 2) | b) & kmask;
        if (++valid >= k) {
            const int q = nuc_lookup(tk, ts, a.lg_t, key);
            if (q >= 0) fn(q, j - k + 1);
        }
    }
}

// First pass: matches per chunk.
__global__ void __launch_bounds__(256) nuc_count_kernel(NucArgs a) {
    NUC_TABLE_SETUP
    int x, c;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!nuc_chunk(a, g, x, c)) return;
    int cnt = 0;
    nuc_scan_chunk(a, tk, ts, x, c, [&](int, int) { ++cnt; });
    a.ccount[g] = cnt;
}

// Second pass: the matches stored at their chunk's offset (so each sequence's
// matches lie in order of p).
__global__ void __launch_bounds__(256) nuc_store_kernel(NucArgs a) {
    NUC_TABLE_SETUP
    int x, c;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!nuc_chunk(a, g, x, c)) return;
    int64_t at = a.cmoff[g];
    nuc_scan_chunk(a, tk, ts, x, c, [&](int q, int p) {
        a.mq[at] = q;
        a.mp[at] = p;
        ++at;
    });
}

// Third pass: the anchor chain over a sequence's matches (in order of p).  A
// match is inserted into the chain table once p_i >= p_j + k for the match i
// being queried; tails[L] is the inserted match of chain length L with the
// smallest (q, p) (q increases with L).  A query takes the longest L whose
// tail has q < q_i: best = L + 1, predecessor = tails[L].  Sequential in the
// matches; returns L with the chain in tails[0 .. L-1].
template <typename TM, typename TI>
__device__ __forceinline__ int nuc_chain_seq(const TM *mq, const TM *mp, TI *mbest, TI *mpred, TI *tails, int cnt,
                                             int k) {
    int L = 0, ins_next = 0;
    int lastq = -1;   // q of tails[L]
    auto insert = [&](int j) __attribute__((always_inline)) {
        const int bj = (int)mbest[j];
        const int qj = (int)mq[j];
        if (bj > L) {
            tails[bj] = (TI)j;
            L = bj;
            lastq = qj;
        } else if (qj < (int)mq[tails[bj]]) {
            tails[bj] = (TI)j;
            if (bj == L) lastq = qj;
        }
    };
    int qn = cnt > 0 ? (int)mq[0] : 0, pn = cnt > 0 ? (int)mp[0] : 0;
    for (int i = 0; i < cnt; ++i) {
        const int q = qn, p = pn;
        if (i + 1 < cnt) {   // the next match's fields, loaded a match ahead
            qn = (int)mq[i + 1];
            pn = (int)mp[i + 1];
        }
        while (ins_next < i && (int)mp[ins_next] + k <= p) insert(ins_next++);
        int lq = 0;
        if (L > 0 && lastq < q) {
            lq = L;
        } else {
            int lo = 1, hi = L;   // largest l in [1, L] with q(tails[l]) < q
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                if ((int)mq[tails[mid]] < q) { lq = mid; lo = mid + 1; }
                else hi = mid - 1;
            }
        }
        mbest[i] = (TI)(lq + 1);
        mpred[i] = (TI)(lq > 0 ? (int)tails[lq] : 0);   // unused for lq = 0
    }
    while (ins_next < cnt) insert(ins_next++);
    // the chain, in order, into tails[0 .. L-1] (tails[L] is its last match)
    int e = L > 0 ? (int)tails[L] : 0;
    for (int t = L - 1; t >= 0; --t) {
        tails[t] = (TI)e;
        e = (int)mpred[e];
    }
    return L;
}

constexpr int kChainLdsMax = 4096;   // matches of a sequence chained in LDS at most

// LDS of the chain kernel for cap matches: five 16-bit arrays
inline size_t nuc_chain_lds_bytes(int cap) { return (size_t)2 * (5 * (size_t)cap + 1); }

// One 64-lane workgroup per sequence.  A sequence with at most a.chain_cap
// matches has them staged in LDS (q, p < 65536 as 16-bit fields) and chained
// there by lane 0; a larger one is chained by lane 0 in the global arrays.
// Then the lanes share the slots: the anchors (aligned bits, scores) and one
// stretch per slot (before the first anchor, between anchors, after the last;
// slots past the chain get an empty descriptor).
__global__ void __launch_bounds__(64) nuc_chain_kernel(NucArgs a) {
    extern __shared__ uint16_t chain_lds[];
    const int cap = a.chain_cap;
    uint16_t *lq = chain_lds, *lp = lq + cap, *lbest = lp + cap, *lpred = lbest + cap, *ltails = lpred + cap;
    __shared__ int sh_L, sh_total;
    const int x = blockIdx.x, lane = threadIdx.x;
    const int n = (int)(a.off[x + 1] - a.off[x]);
    const int k = a.k, m = a.m;
    const int64_t mb = a.cmoff[a.cbase[x]];
    const int cnt = (int)(a.cmoff[a.cbase[x + 1]] - mb);
    const int32_t *mq = a.mq + mb, *mp = a.mp + mb;
    const int64_t sb = mb + x;   // this sequence's slots: sb .. sb + cnt
    int32_t *tails = a.tails + sb;
    const bool inl = cnt <= cap;
    if (inl) {
        for (int i = lane; i < cnt; i += 64) {
            lq[i] = (uint16_t)mq[i];
            lp[i] = (uint16_t)mp[i];
        }
    }
    if (lane == 0) sh_total = 0;
    __syncthreads();
    if (lane == 0)
        sh_L = inl ? nuc_chain_seq(lq, lp, lbest, lpred, ltails, cnt, k)
                   : nuc_chain_seq(mq, mp, a.mbest + mb, a.mpred + mb, tails, cnt, k);
    __syncthreads();
    const int L = sh_L;
    auto anchor = [&](int t) __attribute__((always_inline)) -> int {   // match index of anchor t < L
        return inl ? (int)ltails[t] : tails[t];
    };
    auto qof = [&](int j) __attribute__((always_inline)) -> int { return inl ? (int)lq[j] : mq[j]; };
    auto pof = [&](int j) __attribute__((always_inline)) -> int { return inl ? (int)lp[j] : mp[j]; };
    uint32_t *al = a.aligned + (int64_t)x * a.aw;
    int part = 0;
    for (int t = lane; t <= cnt; t += 64) {
        if (t > L) {
            a.sdesc[sb + t] = make_int4(0, -1, 0, 0);
            a.srow[sb + t] = 0;
            a.scode[sb + t] = 0;
            continue;
        }
        int ci = 0, sj = 0;   // just past the previous anchor
        if (t > 0) {
            const int jp = anchor(t - 1);
            ci = qof(jp) * k + k;
            sj = pof(jp) + k;
        }
        const int jt = t < L ? anchor(t) : 0;
        const int qc = t < L ? qof(jt) * k : m;
        const int ps = t < L ? pof(jt) : n;
        const int dc = qc - ci, ds = ps - sj;
        a.sdesc[sb + t] = make_int4(ci, dc, sj, ds);
        a.sseq[sb + t] = x;
        a.srow[sb + t] = ds + 1;
        a.scode[sb + t] = (int64_t)dc * ((ds + 7) >> 3);
        if (t < L) {
            // center positions qc .. qc + k - 1 aligned
            for (int w = qc >> 5; w <= (qc + k - 1) >> 5; ++w) {
                const int b0 = max(qc, w << 5) - (w << 5), b1 = min(qc + k, (w + 1) << 5) - (w << 5);
                const uint32_t bits = (b1 - b0 == 32) ? ~0u : (((1u << (b1 - b0)) - 1u) << b0);
                atomicOr(al + w, bits);
            }
            part += a.segscore[qof(jt)];
        }
    }
    atomicAdd(&sh_total, part);
    __syncthreads();
    if (lane == 0) a.score[x] = sh_total;
}

// Fourth pass, one lane per stretch: the stretch aligned end to end (Gotoh's
// global form, H(0,0) = 0, H(i,0) = F(i,0) = -(go + ge*i), H(0,j) = E(0,j) =
// -(go + ge*j)), codes per cell (bit 0 diagonal not taken, 1 E not taken,
// 2 E extended, 3 F extended), then the traceback with the local alignment's
// priorities into the center-star vector.  Stretches of a sequence touch
// disjoint insertion slots; aligned words and the score are shared (atomics).
__global__ void __launch_bounds__(256) nuc_stretch_kernel(NucArgs a) {
    __shared__ int8_t smat[32 * 32];
    for (int x = threadIdx.x; x < 1024; x += blockDim.x) {
        const int r = x >> 5, q = x & 31;
        smat[x] = (r < a.alpha && q < a.alpha) ? a.mat[r * a.alpha + q] : (int8_t)0;
    }
    __syncthreads();
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= a.nslot) return;
    const int4 d = a.sdesc[slot];
    const int dc = d.y;
    if (dc < 0) return;
    const int ci = d.x, sj = d.z, ds = d.w;
    if (dc == 0 && ds == 0) return;   // adjacent anchors: nothing between them
    const int x = a.sseq[slot];
    const uint8_t *cc = a.center + ci, *ss = a.res + a.off[x] + sj;
    const int m = a.m, go = a.go, ge = a.ge, goe = go + ge;
    int2 *row = a.rows + a.srowoff[slot];
    uint32_t *code0 = a.codes + a.scodeoff[slot];
    uint16_t *ins = a.ins + (int64_t)x * (m + 1);
    uint32_t *al = a.aligned + (int64_t)x * a.aw;
    int32_t *gmax = (a.G && x != a.gskip) ? a.G : nullptr;
    const int cw = (ds + 7) >> 3;   // code words per row
    // forward: the row buffer holds (H, F) of the row above
    for (int j = 0; j <= ds; ++j) row[j] = make_int2(j == 0 ? 0 : -(go + ge * j), kNucNeg);
    for (int i = 1; i <= dc; ++i) {
        const int cr = cc[i - 1] * 32;
        int hdiag = row[0].x;
        int hleft = -(go + ge * i), eleft = kNucNeg;
        row[0] = make_int2(hleft, hleft);
        uint32_t *crow = code0 + (int64_t)(i - 1) * cw;
        uint32_t word = 0;
        int2 upn = ds >= 1 ? row[1] : make_int2(0, 0);
        for (int j = 1; j <= ds; ++j) {
            const int2 up = upn;
            if (j < ds) upn = row[j + 1];   // a cell ahead
            const int e = max(eleft - ge, hleft - goe);
            const int f = max(up.y - ge, up.x - goe);
            const int dd = hdiag + smat[cr + ss[j - 1]];
            const int h = max(dd, max(e, f));
            const uint32_t nib = (uint32_t)(h != dd) | ((uint32_t)(h != e) << 1) |
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
    atomicAdd(a.score + x, row[ds].x);   // H(dc, ds): the last row written (row 0 when dc = 0)
    // traceback from (dc, ds) to (0, 0)
    int i = dc, j = ds, st = 0;   // 0 H, 1 E, 2 F
    int sl = -1, scount = 0;
    int curw = -1;
    uint32_t bits = 0;
    while (i > 0 || j > 0) {
        const uint32_t nib = (i > 0 && j > 0)
                                 ? (code0[(int64_t)(i - 1) * cw + ((j - 1) >> 3)] >> (4 * ((j - 1) & 7))) & 15u
                                 : 0u;
        if (st == 0) {
            if (i > 0 && j > 0) {
                if (!(nib & 1u)) {
                    const int p = ci + i - 1;
                    if ((p >> 5) != curw) {
                        if (curw >= 0) atomicOr(al + curw, bits);
                        curw = p >> 5;
                        bits = 0;
                    }
                    bits |= 1u << (p & 31);
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
            if (ci + i != sl) {
                if (sl >= 0) {
                    ins[sl] = (uint16_t)scount;
                    if (gmax) atomicMax(gmax + sl, scount);
                }
                sl = ci + i;
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
    if (sl >= 0) {
        ins[sl] = (uint16_t)scount;
        if (gmax) atomicMax(gmax + sl, scount);
    }
    if (curw >= 0) atomicOr(al + curw, bits);
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

// Scans of many values: tiles of kScanTile (1024 lanes x 8 values) scanned
// in place with their totals in part[], the totals scanned by
// scan_i64_kernel, then added back.
constexpr int kScanTile = 8192;

__global__ void __launch_bounds__(1024) scan_tile_kernel(const int64_t *in, int64_t n, int64_t add, int64_t *out,
                                                          int64_t *part) {
    __shared__ int64_t sh[1024];
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * 8;
    int64_t v[8], sum = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        v[u] = t0 + u < n ? in[t0 + u] + add : 0;
        sum += v[u];
    }
    sh[tid] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t w = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += w;
        __syncthreads();
    }
    int64_t acc = tid > 0 ? sh[tid - 1] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (t0 + u < n) out[t0 + u] = acc;
        acc += v[u];
    }
    if (tid == 1023) part[blockIdx.x] = sh[1023];
}

__global__ void scan_add_kernel(int64_t *out, int64_t n, const int64_t *part_off) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) out[x] += part_off[x / kScanTile];
}

// int32 counts to int64 (for the scan)
__global__ void widen_kernel(const int32_t *in, int n, int64_t *out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) out[x] = in[x];
}

}  // namespace hk
