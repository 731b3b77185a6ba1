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
    // segment table: T slots (power of two), key (2-bit packed string, base
    // t at bits 2t and 2t + 1) and segment index (-1 = empty); segscore[q] =
    // sum of S over segment q
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
    int64_t *srow, *scode;    // per slot: boundary entries (wide stretches), code words
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
    // non-empty stretches: slots of the narrow ones (one lane each; lcount[0]
    // of at most kNucTinyW x kNucTinyW from the front of slist, lcount[2]
    // others from its back, nslot entries) and the wide ones (one wavefront
    // each; lcount[1] in blist); counts zeroed before the chain kernel
    int32_t *slist, *blist;
    int32_t *lcount;
};

constexpr int kNucChunk = 256;   // match starts per scan chunk
constexpr int kNucSmallW = 32;   // stretches at most this many columns wide: one lane, the row in registers
constexpr int kNucTinyW = 20;    // narrow stretches at most this size both ways are listed apart
constexpr int kNucTallH = 40;    // stretches taller than this take a wavefront too (rows across lanes)

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
        key = (key >> 2) | ((unsigned long long)b << (2 * (k - 1)));   // base j - k + 1 + t at bits 2t
        if (++valid >= k) {
            const int q = nuc_lookup(tk, ts, a.lg_t, key);
            if (q >= 0) fn(q, j - k + 1);
        }
    }
}

constexpr int kNucWaveMaxK = 29;   // the wavefront scan's window: k + 3 bases in 64 bits

// The match starts p = p0 + 4 lane + r (r < 4) of chunk c of a sequence (its
// residues at so, n of them), the
// lanes of a wavefront sharing the chunk: returns q_r (the segment, or -1) in
// q[r].  The chunk's bytes come in coalesced aligned words (one per lane, nine
// more for the last k - 1 bases), are realigned to the chunk's start, turned
// into 2-bit codes plus an invalid bit per base, and each lane gathers the
// codes of its 32 bases (4 lane .. 4 lane + 31) from the next seven lanes.
__device__ __forceinline__ void nuc_scan_wave(const NucArgs &a, const unsigned long long *tk, const int32_t *ts,
                                              int64_t so, int n, int c, int lane, int q[4]) {
    const int k = a.k;
    const int p0 = c * kNucChunk;
    const uint8_t *base = a.res + so;
    const uintptr_t ad = (uintptr_t)(base + p0);
    const uintptr_t A = ad & ~(uintptr_t)3;
    const uint32_t sh = (uint32_t)(ad & 3);
    const uintptr_t lim = (uintptr_t)(base + n);   // a word starting before it holds a byte of the sequence
    const uint32_t d0 = A + 4 * (uintptr_t)lane < lim ? *reinterpret_cast<const uint32_t *>(A + 4 * lane) : 0u;
    const uint32_t d1 =
        (lane < 9 && A + 256 + 4 * (uintptr_t)lane < lim) ? *reinterpret_cast<const uint32_t *>(A + 256 + 4 * lane) : 0u;
    // bytes p0 + 4 lane .. + 3 (e0) and p0 + 256 + 4 lane .. + 3 (e1, lanes < 8)
    const uint32_t n0 = __shfl(d0, (lane + 1) & 63, 64), n1 = __shfl(d1, 0, 64), n1b = __shfl(d1, (lane + 1) & 63, 64);
    const uint32_t e0 = (uint32_t)((((uint64_t)(lane < 63 ? n0 : n1) << 32) | d0) >> (8 * sh));
    const uint32_t e1 = (uint32_t)((((uint64_t)n1b << 32) | d1) >> (8 * sh));
    auto codes = [](uint32_t e) __attribute__((always_inline)) -> uint32_t {   // 2-bit codes | invalid bits << 8
        uint32_t v = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t b = (e >> (8 * j)) & 255u;
            v |= (b & 3u) << (2 * j);
            v |= (uint32_t)(b > 3u) << (8 + j);
        }
        return v;
    };
    const uint32_t ca = codes(e0), cb = codes(e1);
    uint64_t W = 0;   // base 4 lane + t at bits 2t
    uint32_t V = 0;   // its invalid bit at bit t
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int src = lane + d;
        const uint32_t va = __shfl(ca, src & 63, 64), vb = __shfl(cb, src & 63, 64);
        const uint32_t v = src < 64 ? va : vb;
        W |= (uint64_t)(v & 255u) << (8 * d);
        V |= (v >> 8) << (4 * d);
    }
    const uint64_t kmask = (1ull << (2 * k)) - 1ull;
    const uint32_t vmask = (1u << k) - 1u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = p0 + 4 * lane + r;
        const bool ok = p + k <= n && ((V >> r) & vmask) == 0u;
        q[r] = ok ? nuc_lookup(tk, ts, a.lg_t, (W >> (2 * r)) & kmask) : -1;
    }
}

static_assert(kNucChunk == 4 * 64, "the wavefront scan takes four match starts per lane");

// The wavefront's chunks [g, g1): an equal share of a.nchunk, contiguous so
// that one search finds the first chunk's sequence and the rest follow it.
__device__ __forceinline__ void nuc_wave_range(const NucArgs &a, int64_t &g, int64_t &g1) {
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t per = (a.nchunk + nw - 1) / nw;
    g = min(a.nchunk, w * per);
    g1 = min(a.nchunk, g + per);
}

// First pass, wavefront form (k <= kNucWaveMaxK): matches per chunk.
__global__ void __launch_bounds__(1024) nuc_count_wave_kernel(NucArgs a) {
    NUC_TABLE_SETUP   // shared by the workgroup's 16 wavefronts
    const int lane = threadIdx.x & 63;
    int64_t g, g1;
    nuc_wave_range(a, g, g1);
    int x = 0, c = 0;
    if (g < g1) nuc_chunk(a, g, x, c);
    int64_t so = a.off[x], nb = a.cbase[x + 1];
    int n = (int)(a.off[x + 1] - so);
    for (; g < g1; ++g) {
        if (g >= nb) {   // the next sequence with chunks
            do ++x;
            while (g >= a.cbase[x + 1]);
            c = 0;
            so = a.off[x];
            n = (int)(a.off[x + 1] - so);
            nb = a.cbase[x + 1];
        }
        int q[4];
        nuc_scan_wave(a, tk, ts, so, n, c, lane, q);
        int cnt = (q[0] >= 0) + (q[1] >= 0) + (q[2] >= 0) + (q[3] >= 0);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) a.ccount[g] = cnt;
        ++c;
    }
}

// Second pass, wavefront form: the matches at their chunk's offset, in order
// of p (lane by lane, then r).
__global__ void __launch_bounds__(1024) nuc_store_wave_kernel(NucArgs a) {
    NUC_TABLE_SETUP   // shared by the workgroup's 16 wavefronts
    const int lane = threadIdx.x & 63;
    int64_t g, g1;
    nuc_wave_range(a, g, g1);
    int x = 0, c = 0;
    if (g < g1) nuc_chunk(a, g, x, c);
    int64_t so = a.off[x], nb = a.cbase[x + 1];
    int n = (int)(a.off[x + 1] - so);
    for (; g < g1; ++g) {
        if (g >= nb) {   // the next sequence with chunks
            do ++x;
            while (g >= a.cbase[x + 1]);
            c = 0;
            so = a.off[x];
            n = (int)(a.off[x + 1] - so);
            nb = a.cbase[x + 1];
        }
        int q[4];
        nuc_scan_wave(a, tk, ts, so, n, c, lane, q);
        const int cnt = (q[0] >= 0) + (q[1] >= 0) + (q[2] >= 0) + (q[3] >= 0);
        int inc = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        int64_t at = a.cmoff[g] + inc - cnt;
        const int p = c * kNucChunk + 4 * lane;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (q[r] >= 0) {
                a.mq[at] = q[r];
                a.mp[at] = p + r;
                ++at;
            }
        ++c;
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
    int lastq = -1, lastj = 0;   // q and index of tails[L]
    // the previous match's fields stay in registers: it is usually the next
    // one inserted (matches lie about k apart in p)
    int qprev = 0, pprev = 0, bprev = 0;
    int qn = cnt > 0 ? (int)mq[0] : 0, pn = cnt > 0 ? (int)mp[0] : 0;
    for (int i = 0; i < cnt; ++i) {
        const int q = qn, p = pn;
        if (i + 1 < cnt) {   // the next match's fields, loaded a match ahead
            qn = (int)mq[i + 1];
            pn = (int)mp[i + 1];
        }
        while (ins_next < i) {
            const bool reg = ins_next == i - 1;
            const int pj = reg ? pprev : (int)mp[ins_next];
            if (pj + k > p) break;
            const int j = ins_next++;
            const int bj = reg ? bprev : (int)mbest[j];
            const int qj = reg ? qprev : (int)mq[j];
            if (bj > L) {
                tails[bj] = (TI)j;
                L = bj;
                lastq = qj;
                lastj = j;
            } else if (qj < (int)mq[tails[bj]]) {
                tails[bj] = (TI)j;
                if (bj == L) {
                    lastq = qj;
                    lastj = j;
                }
            }
        }
        int lq = 0, pred = 0;   // pred unused for lq = 0
        if (L > 0 && lastq < q) {
            lq = L;
            pred = lastj;
        } else {
            int lo = 1, hi = L;   // largest l in [1, L] with q(tails[l]) < q
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                if ((int)mq[tails[mid]] < q) { lq = mid; lo = mid + 1; }
                else hi = mid - 1;
            }
            if (lq > 0) pred = (int)tails[lq];
        }
        mbest[i] = (TI)(lq + 1);
        mpred[i] = (TI)pred;
        qprev = q;
        pprev = p;
        bprev = lq + 1;
    }
    while (ins_next < cnt) {
        const int j = ins_next++;
        const int bj = (int)mbest[j];
        const int qj = (int)mq[j];
        if (bj > L) {
            tails[bj] = (TI)j;
            L = bj;
        } else if (qj < (int)mq[tails[bj]]) {
            tails[bj] = (TI)j;
        }
    }
    // the chain, in order, into tails[0 .. L-1] (tails[L] is its last match)
    int e = L > 0 ? (int)tails[L] : 0;
    for (int t = L - 1; t >= 0; --t) {
        tails[t] = (TI)e;
        e = (int)mpred[e];
    }
    return L;
}

constexpr int kChainLdsMax = 4096;   // matches of a sequence chained in LDS at most

// LDS of the chain kernel (16-bit units): q, p, best, pred [cap] each, tails
// [2 cap + 2], cut flags (bytes) [cap], then the aligned words (4-byte aligned)
__host__ __device__ inline size_t nuc_chain_lal_off(int cap) { return ((6 * (size_t)cap + 2 + ((size_t)cap + 1) / 2) + 1) & ~(size_t)1; }
inline size_t nuc_chain_lds_bytes(int cap, int aw) { return 2 * nuc_chain_lal_off(cap) + 4 * (size_t)aw; }

// One 64-lane workgroup per sequence.  A sequence with at most a.chain_cap
// matches has them staged in LDS (q, p < 65536 as 16-bit fields) and chained
// there, segment by segment (below); a larger one is chained by lane 0 in the
// global arrays.
// Then the lanes share the slots: the anchors (aligned bits, scores) and one
// stretch per slot (before the first anchor, between anchors, after the last;
// slots past the chain get an empty descriptor).
__global__ void __launch_bounds__(64) nuc_chain_kernel(NucArgs a) {
    extern __shared__ uint16_t chain_lds[];
    const int cap = a.chain_cap;
    uint16_t *lq = chain_lds, *lp = lq + cap, *lbest = lp + cap, *lpred = lbest + cap, *ltails = lpred + cap;
    uint8_t *lcut = reinterpret_cast<uint8_t *>(ltails + 2 * cap + 2);
    __shared__ int sh_L;
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
    __syncthreads();
    auto qof = [&](int j) __attribute__((always_inline)) -> int { return inl ? (int)lq[j] : mq[j]; };
    auto pof = [&](int j) __attribute__((always_inline)) -> int { return inl ? (int)lp[j] : mp[j]; };
    // When every match follows the one before it (q larger, p at least k
    // further), all of them form the one chain of length cnt, which is then
    // the longest: checked by all lanes, no sequential pass.
    bool ok = true;
    for (int i = lane; i + 1 < cnt; i += 64) ok = ok && qof(i + 1) > qof(i) && pof(i + 1) >= pof(i) + k;
    const bool ident = __ballot(!ok) == 0;
    if (!ident && !inl) {
        if (lane == 0) sh_L = nuc_chain_seq(mq, mp, a.mbest + mb, a.mpred + mb, tails, cnt, k);
    } else if (!ident) {
        // Cuts: b splits the matches when every match before it precedes every
        // match from it on (max q before b < min q from b, p[b-1] + k <= p[b]).
        // Then every match before b is inserted before b is queried, each query
        // from b on finds the prefix's whole chain below its q, and later
        // inserts touch only longer lengths: the chain is the prefix's chain
        // followed by the rest's.  So each segment between cuts is chained on
        // its own (lanes take the segments starting in their block), and the
        // segments' chains are joined in order.
        const int per = (cnt + 63) / 64, lo = min(cnt, lane * per), hi = min(cnt, lo + per);
        int bmax = -1, bmin = 0x7fffffff;
        for (int i = lo; i < hi; ++i) {
            bmax = max(bmax, (int)lq[i]);
            bmin = min(bmin, (int)lq[i]);
        }
        int pm = bmax, sm = bmin;   // inclusive prefix max, suffix min over the lanes
        for (int d = 1; d < 64; d <<= 1) {
            const int t1 = __shfl_up(pm, d, 64), t2 = __shfl_down(sm, d, 64);
            if (lane >= d) pm = max(pm, t1);
            if (lane + d < 64) sm = min(sm, t2);
        }
        int runmax = __shfl_up(pm, 1, 64), runmin = __shfl_down(sm, 1, 64);
        if (lane == 0) runmax = -1;
        if (lane == 63) runmin = 0x7fffffff;
        for (int i = hi - 1; i >= lo; --i) {   // min q from i on (lbest as scratch)
            runmin = min(runmin, (int)lq[i]);
            lbest[i] = (uint16_t)runmin;
        }
        for (int i = lo; i < hi; ++i) {
            lcut[i] = (i == 0 || (runmax < (int)lbest[i] && (int)lp[i - 1] + k <= (int)lp[i])) ? 1 : 0;
            runmax = max(runmax, (int)lq[i]);
        }
        __syncthreads();
        for (int b = lo; b < hi; ++b) {
            if (!lcut[b]) continue;
            int e = b + 1;
            while (e < cnt && !lcut[e]) ++e;
            const int Ls = nuc_chain_seq(lq + b, lp + b, lbest + b, lpred + b, ltails + 2 * b, e - b, k);
            lbest[b] = (uint16_t)Ls;   // the segment's chain length (its own best no longer needed)
        }
        __syncthreads();
        int sl = 0;
        for (int b = lo; b < hi; ++b)
            if (lcut[b]) sl += lbest[b];
        int inc = sl;
        for (int d = 1; d < 64; d <<= 1) {
            const int t1 = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t1;
        }
        int o = inc - sl;
        for (int b = lo; b < hi; ++b) {   // the chain, in order, into lpred (preds no longer needed)
            if (!lcut[b]) continue;
            const int Ls = lbest[b];
            for (int t = 0; t < Ls; ++t) lpred[o + t] = (uint16_t)(b + ltails[2 * b + t]);
            o += Ls;
        }
        if (lane == 63) sh_L = inc;
    }
    __syncthreads();
    const int L = ident ? cnt : sh_L;
    auto anchor = [&](int t) __attribute__((always_inline)) -> int {   // match index of anchor t < L
        return ident ? t : (inl ? (int)lpred[t] : tails[t]);
    };
    uint32_t *al = a.aligned + (int64_t)x * a.aw;
    uint32_t *lal = reinterpret_cast<uint32_t *>(chain_lds + nuc_chain_lal_off(cap));   // [aw]: the aligned bits
    for (int w = lane; w < a.aw; w += 64) lal[w] = 0u;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;   // lanes under this one
    // slot t of the chain (t <= L): the stretch from just past anchor t - 1 to
    // anchor t (or the ends)
    auto stretch = [&](int t, int &ci, int &sj, int &dc, int &ds, int &jt) __attribute__((always_inline)) {
        ci = 0;
        sj = 0;
        if (t > 0) {
            const int jp = anchor(t - 1);
            ci = qof(jp) * k + k;
            sj = pof(jp) + k;
        }
        jt = t < L ? anchor(t) : 0;
        dc = (t < L ? qof(jt) * k : m) - ci;
        ds = (t < L ? pof(jt) : n) - sj;
    };
    // narrow stretches (at most kNucSmallW columns and kNucTallH rows): up to
    // kNucTinyW x kNucTinyW from the front of the lane list, the others from
    // its back, so most wavefronts get stretches of one size; the rest take
    // a wavefront each
    auto tiny = [&](int dc, int ds) __attribute__((always_inline)) { return dc <= kNucTinyW && ds <= kNucTinyW; };
    int part = 0, nsm = 0, nwd = 0, nti = 0;
    for (int t = lane; t <= L; t += 64) {
        int ci, sj, dc, ds, jt;
        stretch(t, ci, sj, dc, ds, jt);
        const bool work = dc > 0 || ds > 0;
        const bool wide = work && (ds > kNucSmallW || dc > kNucTallH);
        nti += work && !wide && tiny(dc, ds);
        nsm += work && !wide && !tiny(dc, ds);
        nwd += wide;
        a.sdesc[sb + t] = make_int4(ci, dc, sj, ds);
        a.sseq[sb + t] = x;
        a.srow[sb + t] = wide ? dc + 1 : 0;   // the wavefront kernel's boundary column
        a.scode[sb + t] = (int64_t)dc * ((ds + 7) >> 3);
        if (t < L) {
            // center positions qc .. qc + k - 1 aligned
            const int qc = ci + dc;
            for (int w = qc >> 5; w <= (qc + k - 1) >> 5; ++w) {
                const int b0 = max(qc, w << 5) - (w << 5), b1 = min(qc + k, (w + 1) << 5) - (w << 5);
                const uint32_t bits = (b1 - b0 == 32) ? ~0u : (((1u << (b1 - b0)) - 1u) << b0);
                atomicOr(lal + w, bits);
            }
            part += a.segscore[qof(jt)];
        }
    }
    for (int t = L + 1 + lane; t <= cnt; t += 64) {   // slots past the chain
        a.sdesc[sb + t] = make_int4(0, -1, 0, 0);
        a.srow[sb + t] = 0;
        a.scode[sb + t] = 0;
    }
    // the sequence's list entries: one global atomic per list, then the
    // non-empty stretches in slot order (narrow: one lane each; wide: a
    // wavefront each)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        part += __shfl_xor(part, o, 64);
        nsm += __shfl_xor(nsm, o, 64);
        nwd += __shfl_xor(nwd, o, 64);
        nti += __shfl_xor(nti, o, 64);
    }
    int os = 0, ow = 0, ot = 0;
    if (lane == 0) {
        a.score[x] = part;
        if (nti) ot = atomicAdd(a.lcount, nti);
        if (nwd) ow = atomicAdd(a.lcount + 1, nwd);
        if (nsm) os = atomicAdd(a.lcount + 2, nsm);
    }
    ot = __shfl(ot, 0, 64);
    os = __shfl(os, 0, 64);
    ow = __shfl(ow, 0, 64);
    int32_t *sback = a.slist + a.nslot - 1;   // the back of the lane list, filled downwards
    for (int t0 = 0; t0 <= L; t0 += 64) {   // uniform trip count (ballots)
        const int t = t0 + lane;
        int ci = 0, sj = 0, dc = 0, ds = 0, jt = 0;
        if (t <= L) stretch(t, ci, sj, dc, ds, jt);
        const bool work = t <= L && (dc > 0 || ds > 0);
        const bool wide = work && (ds > kNucSmallW || dc > kNucTallH);
        const bool ti = work && !wide && tiny(dc, ds);
        const bool sm = work && !wide && !ti;
        const uint64_t bt = __ballot(ti), bs = __ballot(sm), bw = __ballot(wide);
        if (ti) a.slist[ot + __popcll(bt & below)] = (int32_t)(sb + t);
        if (sm) sback[-(int64_t)(os + __popcll(bs & below))] = (int32_t)(sb + t);
        if (wide) a.blist[ow + __popcll(bw & below)] = (int32_t)(sb + t);
        ot += __popcll(bt);
        os += __popcll(bs);
        ow += __popcll(bw);
    }
    __syncthreads();
    for (int w = lane; w < a.aw; w += 64) al[w] = lal[w];   // the row was zeroed; stretches OR in later
}

// Fourth pass: each stretch aligned end to end (Gotoh's global form,
// H(0,0) = 0, H(i,0) = -(go + ge*i), H(0,j) = -(go + ge*j), E(i,0) = F(0,j) =
// -inf), codes per cell (bit 0 diagonal not taken, 1 E not taken, 2 E
// extended, 3 F extended; eight cells per word, cw = ceil(ds / 8) words a
// row), then the traceback with the local alignment's priorities into the
// center-star vector.  Stretches of a sequence touch disjoint insertion slots;
// aligned words and the score are shared (atomics).
#define NUC_SMAT_SETUP                                                              \
    __shared__ int8_t smat[32 * 32];                                                \
    for (int x_ = threadIdx.x; x_ < 1024; x_ += blockDim.x) {                       \
        const int r_ = x_ >> 5, q_ = x_ & 31;                                       \
        smat[x_] = (r_ < a.alpha && q_ < a.alpha) ? a.mat[r_ * a.alpha + q_] : (int8_t)0; \
    }                                                                               \
    __syncthreads();

// The traceback from (dc, ds) to (0, 0) over a stretch's codes: diagonal
// steps mark center positions aligned, E steps count residues into the
// insertion slot after their center position (a slot's count is written once,
// with the merge's running max).
__device__ __forceinline__ void nuc_traceback(const NucArgs &a, int x, int ci, int dc, int ds, const uint32_t *code0) {
    const int cw = (ds + 7) >> 3;
    uint16_t *ins = a.ins + (int64_t)x * (a.m + 1);
    uint32_t *al = a.aligned + (int64_t)x * a.aw;
    int32_t *gmax = (a.G && x != a.gskip) ? a.G : nullptr;
    const int go = a.go;
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

// Stretches at most kNucSmallW columns wide and kNucTallH rows tall, one lane
// each (over the list a.slist: lcount[0] entries from its front, lcount[2]
// from its back): the row of (H, F) sits in registers, the codes go to the
// stretch's code region, then the lane's traceback reads them back.
__global__ void __launch_bounds__(256) nuc_stretch_small_kernel(NucArgs a) {
    NUC_SMAT_SETUP
    const int nt = a.lcount[0], ns = nt + a.lcount[2];   // the front's entries, then the back's
    const int go = a.go, ge = a.ge, goe = go + ge;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < ns; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t li = base + threadIdx.x;
        const bool act = li < ns;
        const int64_t slot = act ? a.slist[li < nt ? li : a.nslot - 1 - (li - nt)] : 0;
        const int4 d = act ? a.sdesc[slot] : make_int4(0, 0, 0, 0);
        const int ci = d.x, dc = d.y, sj = d.z, ds = d.w;
        const int x = act ? a.sseq[slot] : 0;
        // the widest stretch of the wavefront bounds the unrolled columns
        int wmax = ds;
        for (int o = 32; o >= 1; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, 64));
        wmax = __builtin_amdgcn_readfirstlane(wmax);
        const uint8_t *cc = a.center + ci, *ss = a.res + a.off[x] + sj;
        uint32_t *code0 = a.codes + a.scodeoff[slot];
        const int cw = (ds + 7) >> 3;
        uint32_t sw[kNucSmallW / 4];   // the stretch's residues, four per word
#pragma unroll
        for (int w = 0; w < kNucSmallW / 4; ++w) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int jj = 4 * w + b;
                if (jj < ds) v |= (uint32_t)ss[jj] << (8 * b);
            }
            sw[w] = v;
        }
        int H[kNucSmallW + 1], F[kNucSmallW + 1];
#pragma unroll
        for (int j = 0; j <= kNucSmallW; ++j) {
            H[j] = j == 0 ? 0 : -(go + ge * j);
            F[j] = kNucNeg;
        }
        // the center's bases eight rows at a time, the next eight loaded a
        // group ahead
        auto load8 = [&](int i0) __attribute__((always_inline)) -> uint64_t {
            uint64_t v = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < dc) v |= (uint64_t)cc[i0 + u] << (8 * u);
            return v;
        };
        uint64_t cwin = load8(0), cnext = load8(8);
        for (int i = 1; i <= dc; ++i) {
            if (((i - 1) & 7) == 0 && i > 1) {
                cwin = cnext;
                cnext = load8(i + 7);
            }
            const int cr = (int)((cwin >> (8 * ((i - 1) & 7))) & 255u) * 32;
            int hdiag = H[0];
            int hleft = -(go + ge * i), eleft = kNucNeg;
            H[0] = hleft;
            uint32_t *crow = code0 + (int64_t)(i - 1) * cw;
            uint32_t word = 0;
#pragma unroll
            for (int j = 1; j <= kNucSmallW; ++j) {
                if (j > wmax) continue;   // uniform: past the wavefront's widest stretch
                const int e = max(eleft - ge, hleft - goe);
                const int f = max(F[j] - ge, H[j] - goe);
                const int dd = hdiag + smat[cr + ((sw[(j - 1) >> 2] >> (8 * ((j - 1) & 3))) & 255u)];
                const int h = max(dd, max(e, f));
                const uint32_t nib = (uint32_t)(h != dd) | ((uint32_t)(h != e) << 1) |
                                     ((uint32_t)(eleft - ge > hleft - goe) << 2) |
                                     ((uint32_t)(F[j] - ge > H[j] - goe) << 3);
                word |= nib << (4 * ((j - 1) & 7));
                if ((j & 7) == 0 || j == wmax) {
                    if (((j - 1) >> 3) < cw) crow[(j - 1) >> 3] = word;
                    word = 0;
                }
                hdiag = H[j];
                H[j] = h;
                F[j] = f;
                hleft = h;
                eleft = e;
            }
        }
        int hend = H[0];   // H(dc, ds): the last row computed (row 0 when dc = 0)
#pragma unroll
        for (int j = 1; j <= kNucSmallW; ++j)
            if (j == ds) hend = H[j];
        if (act) {
            atomicAdd(a.score + x, hend);
            nuc_traceback(a, x, ci, dc, ds, code0);
        }
    }
}

// inclusive prefix max over the 64 lanes
__device__ __forceinline__ int wave_prefix_max(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v = max(v, t);
    }
    return v;
}

// Wider (or taller) stretches, one wavefront each (over the list a.blist[0 ..
// a.lcount[1])), in strips of 64 columns, lane L owning column 64 b + 1 + L of
// strip b and keeping (H, F) of the row above in registers.  E along a row is a
// max-plus scan: with Ht = max(D, F) and A(j) = Ht(i, j) + ge j,
//   E(i, j) + ge j = max(E(i, jb) + ge jb, H(i, jb) + ge jb - go,
//                        max over jb < j' < j of A(j') - go)
// for the strip's left boundary jb (since E - ge >= E - go - ge, extending from
// an E-derived H never beats the gap it continues).  The boundary column (H, E)
// per row passes from strip to strip through the stretch's row region
// (dc + 1 entries), 64 rows per coalesced load or store.
__global__ void __launch_bounds__(64) nuc_stretch_wave_kernel(NucArgs a) {
    NUC_SMAT_SETUP
    const int lane = threadIdx.x;
    const int nb = a.lcount[1];
    const int go = a.go, ge = a.ge, goe = go + ge;
    constexpr int kLow = -(1 << 30);
    for (int li = blockIdx.x; li < nb; li += gridDim.x) {
        const int64_t slot = a.blist[li];
        const int4 d = a.sdesc[slot];
        const int ci = d.x, dc = d.y, sj = d.z, ds = d.w;
        const int x = a.sseq[slot];
        const uint8_t *cc = a.center + ci, *ss = a.res + a.off[x] + sj;
        int2 *bnd = a.rows + a.srowoff[slot];
        uint32_t *code0 = a.codes + a.scodeoff[slot];
        const int cw = (ds + 7) >> 3;
        const int nstrip = (ds + 63) >> 6;
        for (int b = 0; b < nstrip; ++b) {
            const int jb = 64 * b;
            const int j = jb + 1 + lane;
            const bool inj = j <= ds;
            const int sres = inj ? ss[j - 1] : 0;
            int hp = -(go + ge * j), fp = kNucNeg;         // (H, F)(0, j)
            int bh_prev = b == 0 ? 0 : -(go + ge * jb);    // H(0, jb)
            for (int i0 = 1; i0 <= dc; i0 += 64) {
                const int nr = min(64, dc - i0 + 1);
                const int2 ld = (b > 0 && lane < nr) ? bnd[i0 + lane] : make_int2(0, 0);
                const int crs = lane < nr ? cc[i0 - 1 + lane] : 0;
                int2 out = make_int2(0, 0);
                for (int r = 0; r < nr; ++r) {
                    const int i = i0 + r;
                    const int bh = b == 0 ? -(go + ge * i) : __shfl(ld.x, r, 64);   // H(i, jb)
                    const int be = b == 0 ? kNucNeg : __shfl(ld.y, r, 64);          // E(i, jb)
                    const int cr = __shfl(crs, r, 64) * 32;
                    int hd = __shfl_up(hp, 1, 64);   // H(i-1, j-1)
                    if (lane == 0) hd = bh_prev;
                    const int dd = hd + smat[cr + sres];
                    const int f = max(fp - ge, hp - goe);
                    const int ht = max(dd, f);
                    const int inc = wave_prefix_max(ht + ge * j, lane);
                    int ex = __shfl_up(inc, 1, 64);
                    if (lane == 0) ex = kLow;
                    const int ehat = max(max(be + ge * jb, bh + ge * jb - go), ex - go);
                    const int e = ehat - ge * j;
                    const int h = max(ht, e);
                    int el = __shfl_up(e, 1, 64), hl = __shfl_up(h, 1, 64);   // (E, H)(i, j-1)
                    if (lane == 0) {
                        el = be;
                        hl = bh;
                    }
                    uint32_t nib = (uint32_t)(h != dd) | ((uint32_t)(h != e) << 1) |
                                   ((uint32_t)(el - ge > hl - goe) << 2) | ((uint32_t)(fp - ge > hp - goe) << 3);
                    if (!inj) nib = 0;
                    uint32_t v = nib << (4 * (lane & 7));
                    v |= __shfl_xor(v, 1, 64);
                    v |= __shfl_xor(v, 2, 64);
                    v |= __shfl_xor(v, 4, 64);
                    const int w = 8 * b + (lane >> 3);
                    if ((lane & 7) == 0 && w < cw) code0[(int64_t)(i - 1) * cw + w] = v;
                    const int oh = __shfl(h, 63, 64), oe = __shfl(e, 63, 64);   // (H, E)(i, jb + 64)
                    if (lane == r) out = make_int2(oh, oe);
                    if (i == dc && j == ds) atomicAdd(a.score + x, h);   // H(dc, ds)
                    bh_prev = bh;
                    hp = h;
                    fp = f;
                }
                if (b + 1 < nstrip && lane < nr) bnd[i0 + lane] = out;
            }
        }
        if (dc == 0 && lane == 0) atomicAdd(a.score + x, -(go + ge * ds));   // H(0, ds)
        if (ds == 0 && lane == 0) atomicAdd(a.score + x, -(go + ge * dc));   // H(dc, 0): no strips
        __syncthreads();   // the codes, written by every lane, before lane 0 reads them
        if (lane == 0) nuc_traceback(a, x, ci, dc, ds, code0);
    }
}

#undef NUC_SMAT_SETUP
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
