// Traceback walk for gfx950: one 16-lane DPP row per pair over the 4-bit codes
// written by the wavefront kernel (sw_kernels.hpp) or the strip kernel
// (strip_kernels.hpp), emitting the center-star vector of each pair.
#pragma once
#include "sw_kernels.hpp"

namespace hk {

// ---------------------------------------------------------------------------
// Traceback walk.  From the end cell, in state H: stop when the running value
// is 0, else take the diagonal if notd is clear, else the horizontal gap if
// note is clear, else the vertical gap; in a gap state, extend while the ext
// bit is set (open wins ties).  The running value is H (or the gap value) of
// the current cell, kept exactly from the score.  Emits the center-star
// vector: ins[k][0..m], aligned bits, cells.
//
// A path is a chain of runs: diagonal runs in H, horizontal runs in E and
// vertical runs in F.  Sixteen lanes (one DPP row) serve one pair: lane k
// looks at the k-th cell ahead along the current run, so one iteration
// decides up to sixteen moves.  The first lane whose cell ends the run (a
// stop, a gap, the end of a gap, missing data) is found with a ballot; the
// score change over the diagonal cells before it is a row prefix sum.
//
// Code words arrive in chunks: 8 steps of one lane of the wavefront layout
// (R rows x 8 columns) or 4 columns of one lane of the strip layout (16 rows
// x 4 columns).  Each pair caches 16 chunks in LDS, direct mapped by (block
// mod NB, chunk column mod NG), NB * NG = 16.  On a miss the pair's lanes load,
// one chunk each, the NB blocks at and above the current one times the NG
// chunk columns at and left of where the path (diagonal, or straight up in a
// vertical gap) meets each block, with a 64-byte window of the sequence, in
// one round trip.
// ---------------------------------------------------------------------------
struct WalkArgs {
    const int8_t *mat;
    int alpha;
    const uint8_t *center;
    int m;
    const uint8_t *res;
    const int64_t *off;
    const int32_t *pids;      // pairs to walk (indices into N)
    int npairs;
    int ge, goe;
    const int32_t *score;
    const int32_t *endcell;   // [N][2]
    const uint32_t *codes;
    // layout per pair id: kind 0 = wavefront (R rows/lane), 1 = strip (16 rows)
    const int64_t *cbase;     // strip, per walk entry: word base of the group
    const int32_t *ccol;      // strip, per walk entry: lane in the group
    const int32_t *cstride;   // strip, per walk entry: nmax of the group
    int R;                    // wavefront rows per lane
    uint32_t rmagic;          // ceil(2^32 / R) for R >= 2: row / R = umulhi(row, rmagic) for rows < 2^16
    int kind;
    int32_t *cells;           // [N][4]
    uint16_t *ins;            // [N][m+1] (zeroed)
    uint32_t *aligned;        // [N][aw] (zeroed)
    int aw;
    int32_t *G;               // optional [m+1]: max of ins over the walked pairs
    int gskip;                // pair id kept out of G
    // wavefront layout: the walk runs over slots; slot q holds pair
    // slot_pid[q] at stream column slot_col[q] of the stream s with
    // slot0[s] <= q < slot0[s+1] (streams hold at least one pair each;
    // empty pairs sit in slots after the streamed ones)
    const int32_t *slot_pid;
    const int64_t *slot_col;
    const int64_t *sbeg;      // [nstreams + 1]
    const int32_t *slot0;     // [nstreams]
    const int32_t *slot_stream;   // [slots] the stream s of each slot
    const int64_t *scb;       // [nstreams] code word base
    int nstreams;
    int lg_ls;                // log2 of the lanes per stream (wavefront layout)
    int W;                    // code words per step (wavefront layout)
    int lg_nb;                // log2 of NB, the cached blocks per pair (NG = 16 / NB)
    int glds;                 // 1: G is gathered per workgroup in LDS, then added with one
                              // atomicMax per slot (G != NULL and m < kWalkGLds)
};

constexpr int kWalkCenterLds = 8192;   // centers up to this length are staged in LDS
constexpr int kWalkPairs = 16;         // pairs per 256-thread workgroup (16 lanes each)
constexpr int kWalkSlots = 16;         // cached code chunks per pair
constexpr int kWalkGLds = 2048;        // centers shorter than this gather G in LDS

// LDS bytes of one workgroup: substitution table, sequence windows, chunk
// tags, chunk cache (8 * W words per chunk), the center if staged, and the
// workgroup's G if gathered there
__host__ __device__ inline size_t walk_lds_bytes(int W, int m, bool cen_lds, bool glds) {
    return 1024 + kWalkPairs * 64 + kWalkPairs * kWalkSlots * 8 +
           (size_t)kWalkPairs * kWalkSlots * 8 * W * 4 + (cen_lds ? (size_t)((m + 15) & ~15) : 0) +
           (glds ? (size_t)(m + 1) * 4 : 0);
}

// inclusive prefix sum over the 16 lanes of a DPP row
__device__ inline int row_prefix16(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    return x;
}

// Reasons a run ends at a cell (the first that holds): the walk stops there,
// the codes are bad, the cell's chunk is not cached, the sequence window does
// not hold its residue (diagonal moves only), the move out of the cell is not
// the run's own (a gap from H), the gap ends (E or F).
enum : int { kRunFin = 1, kRunBad = 2, kRunMiss = 3, kRunSmiss = 4, kRunTurn = 5, kRunEnd = 6 };

template <bool STRIP, bool CEN_LDS, bool PK>
__global__ void __launch_bounds__(256)
walk_kernel(WalkArgs a) {
    extern __shared__ uint32_t wlds[];
    const int W = STRIP ? 1 : a.W;
    const int cws = 8 * W;                 // words per cached chunk
    int8_t *smat = reinterpret_cast<int8_t *>(wlds);
    uint32_t *swin_all = wlds + 256;                                    // [pairs][16] words
    int2 *ctag_all = reinterpret_cast<int2 *>(wlds + 256 + kWalkPairs * 16);   // [pairs][slots]
    uint32_t *cache_all = wlds + 256 + kWalkPairs * 16 + kWalkPairs * kWalkSlots * 2;
    uint8_t *scen = reinterpret_cast<uint8_t *>(cache_all + kWalkPairs * kWalkSlots * cws);
    const int m = a.m;
    // the merge: G[x] = max over pairs of ins[x], gathered per workgroup in
    // LDS (the flank slots 0 and m take one value from every pair) and added
    // into G after the workgroup's walks
    int *sG = reinterpret_cast<int *>(scen + (CEN_LDS ? ((m + 15) & ~15) : 0));
    const bool glds = a.glds != 0;
    if (glds)
        for (int x = threadIdx.x; x <= m; x += 256) sG[x] = 0;
    for (int x = threadIdx.x; x < 1024; x += 256) {
        const int r = x >> 5, q = x & 31;
        smat[x] = (r < a.alpha && q < a.alpha) ? a.mat[r * a.alpha + q] : (int8_t)0;
    }
    if (CEN_LDS)
        for (int x = threadIdx.x; x < m; x += 256) scen[x] = a.center[x] & 31;
    ctag_all[threadIdx.x] = make_int2(-1, -1);   // 256 = pairs x slots
    __syncthreads();
    // one pair per 16-lane row; a lambda so that its early exits still reach
    // the workgroup's G flush below
    auto walk_pair = [&]() __attribute__((always_inline)) {
        const int gp = threadIdx.x >> 4;       // pair of the workgroup
        const int k = threadIdx.x & 15;        // lane of the pair's row
        const int gbase = threadIdx.x & 48;    // the row's first lane in the wavefront
        const int w = blockIdx.x * kWalkPairs + gp;
        if (w >= a.npairs) return;
        uint32_t *win = swin_all + gp * 16;
        int2 *ctag = ctag_all + gp * kWalkSlots;
        uint32_t *ccache = cache_all + gp * kWalkSlots * cws;
        const int pid = STRIP ? a.pids[w] : a.slot_pid[w];
        const int64_t so = a.off[pid];
        const int n = (int)(a.off[pid + 1] - so);
        uint16_t *ins = a.ins + (int64_t)pid * (m + 1);
        uint32_t *al = a.aligned + (int64_t)pid * a.aw;
        int v = a.score[pid];
        int4 *cp = reinterpret_cast<int4 *>(a.cells) + pid;
        int32_t *gmax = (a.G && pid != a.gskip) ? (glds ? sG : a.G) : nullptr;
        if (v <= 0) {
            if (k == 0) {
                ins[0] = (uint16_t)n;
                if (gmax && n > 0) atomicMax(gmax, n);
                *cp = make_int4(0, 0, 0, 0);
            }
            return;
        }
        const int i1 = a.endcell[2 * pid], j1 = a.endcell[2 * pid + 1];
        int64_t base;
        int half = 0;   // packed wavefront layout: the stream's half of each code word
        int ccol, stride;
        if (STRIP) {
            base = a.cbase[w];
            ccol = a.ccol[w];
            stride = a.cstride[w];
        } else {   // stream of slot w
            const int lo = a.slot_stream[w];
            base = a.scb[lo];
            ccol = (int)(a.slot_col[w] - a.sbeg[lo]);
            int cs = (int)(a.sbeg[lo + 1] - a.sbeg[lo]);
            if (PK) {   // the stream pair shares the longer stream's tiles
                const int o = lo ^ 1;
                if (o < a.nstreams) cs = max(cs, (int)(a.sbeg[o + 1] - a.sbeg[o]));
                half = lo & 1;
            }
            stride = cs + (1 << a.lg_ls) - 1;
        }
        constexpr bool strip = STRIP;
        const int R = strip ? 16 : a.R;
        const uint32_t rmagic = a.rmagic;
        const int G = strip ? (stride + 3) >> 2 : (stride + 7) >> 3;   // chunk columns per block row
        const int lg = strip ? 6 : a.lg_ls, LSm = (1 << lg) - 1;
        const int n0 = min(R, 8);           // rows in the first word of a step
        const int lgnb = a.lg_nb, lgng = 4 - lgnb, nbm = (1 << lgnb) - 1, ngm = (1 << lgng) - 1;
        // row -> (block, row in block); block = pass * LS + lane (wavefront) or strip
        auto split_row = [&](int row, int &b, int &t) __attribute__((always_inline)) {
            if (strip) { b = row >> 4; t = row & 15; }
            else {
                b = R == 1 ? row : (int)__umulhi((uint32_t)row, rmagic);
                t = row - b * R;
            }
        };
        // chunk column of (block b, column col)
        auto grp_of = [&](int b, int col) __attribute__((always_inline)) -> int {
            return strip ? col >> 2 : (ccol + col + (b & LSm)) >> 3;
        };
        auto chunk_addr = [&](int b, int g) __attribute__((always_inline)) -> int64_t {
            return strip ? base + (((int64_t)b * G + g) * 64 + ccol) * 8
                         : base + ((((int64_t)(b >> lg) * G + g) << lg) + (b & LSm)) * 8 * W;
        };
        int i = i1, j = j1;
        int state = 0;              // 0 = H, 1 = E, 2 = F
        int run = 0;                // horizontal moves of the open insertion run
        int insrow = -1, inssum = 0;
        int curw = -1;              // aligned word being accumulated
        uint32_t bits = 0;
        int64_t swb = 0;
        int qoff = -(1 << 30);      // so - swb once a window is loaded
        bool bad = (i1 < 1 || i1 > m || j1 < 1 || j1 > n);
        bool fin = false;
        // a path has at most m + n steps; the guard keeps a corrupted code
        // stream from reading outside the matrix or looping
        int guard = 0;
        const int glim = m + n + 2;
        for (;;) {
            if (__ballot(!bad && !fin) == 0) break;
            // why the pair left the iteration loop: 0 still in it, else a kRun*
            // reason; 7 done before the round
            int why = (bad || fin) ? 7 : 0;
            for (;;) {
                // ---- the cell of lane k: k moves ahead along the current run
                const int ci = i - (state != 1 ? k : 0), cj = j - (state != 2 ? k : 0);
                const int row = max(ci - 1, 0), col = max(cj - 1, 0);
                int b, t;
                split_row(row, b, t);
                const int g = grp_of(b, col);
                const int slot = (g & ngm) | ((b & nbm) << lgng);
                int wi, sh;
                if (strip) { wi = (col & 3) * 2 + (t >> 3); sh = 4 * (7 - (t & 7)); }
                else {
                    const int st8 = (ccol + col + (b & LSm)) & 7;
                    if (PK) { wi = st8 * W + (t >> 2); sh = 8 * half + 2 * (t & 3); }
                    else { wi = st8 * W + (t >> 3); sh = t < 8 ? 4 * (n0 - 1 - t) : 4 * (R - 1 - t); }
                }
                const uint32_t cword = ccache[slot * cws + wi];
                const int2 tg = ctag[slot];
                const int gq = qoff + col;
                const int gqc = min(max(gq, 0), 63);
                const int ic = min(row, m - 1);
                const int cr = CEN_LDS ? (int)scen[ic] : (int)(a.center[ic] & 31);
                const int sr = (int)((win[gqc >> 2] >> (8 * (gqc & 3))) & 31u);
                int sd = (int)smat[cr * 32 + sr];
                // read for every lane and iteration: no branch guards the reads
                asm volatile("" : "+v"(sd));
                // notd, note, eext, fext in bits 0-3 (packed layout: two bit pairs 16 apart)
                const uint32_t nib = PK ? ((cword >> (sh & 15)) & 3u) | (((cword >> ((sh & 15) + 16)) & 3u) << 2)
                                        : (cword >> (sh & 31)) & 15u;
                const int hit = (tg.x == b) & (tg.y == g);
                const int cbad = (ci < 1) | (cj < 1) | (guard + k > glim);
                // score change over the diagonal cells before this one
                const int pre = row_prefix16(sd) - sd;
                int reason;
                if (state == 0) {
                    const int dg = (int)(~nib & 1u);
                    reason = (v - pre == 0) ? kRunFin : cbad ? kRunBad : !hit ? kRunMiss
                           : !dg ? kRunTurn : ((unsigned)gq >= 64u) ? kRunSmiss : 0;
                } else {
                    const int ext = (int)(nib >> (state == 1 ? 2 : 3)) & 1;
                    reason = cbad ? kRunBad : !hit ? kRunMiss : !ext ? kRunEnd : 0;
                }
                // ---- the first lane of the row that ends the run
                const unsigned long long fm = __ballot(reason != 0);
                const uint32_t rb = (uint32_t)(fm >> gbase) & 0xffffu;
                const int r = __builtin_ctz(rb | 0x10000u);
                const int q = min(r, 15);
                const uint32_t pk = ((uint32_t)(pre + 0x8000) & 0xffffu) | ((uint32_t)(sd & 0xff) << 16) |
                                    (nib << 24) | ((uint32_t)reason << 28);
                const uint32_t got = (uint32_t)__builtin_amdgcn_ds_bpermute((gbase + q) << 2, (int)pk);
                const int preq = (int)(got & 0xffffu) - 0x8000;
                const int sdq = (int)(int8_t)(got >> 16);
                const uint32_t nibq = (got >> 24) & 15u;
                const int rq = r < 16 ? (int)(got >> 28) : 0;
                if (why == 0) {
                    // ---- r moves of the run
                    if (state == 0) {
                        if (r > 0) {
                            // aligned bits of center positions i - r .. i - 1
                            const int hi = i - 1, lo = i - r;
                            const int wh = hi >> 5, wlo = lo >> 5;
                            if (wh != curw) {
                                if (curw >= 0 && k == 0) al[curw] = bits;
                                curw = wh;
                                bits = 0;
                            }
                            bits |= (0xffffffffu >> (31 - (hi & 31))) & (0xffffffffu << (wlo == wh ? (lo & 31) : 0));
                            if (wlo != wh) {
                                if (k == 0) al[wh] = bits;
                                curw = wlo;
                                bits = 0xffffffffu << (lo & 31);
                            }
                        }
                        v -= preq + (r == 16 ? sdq : 0);
                        i -= r;
                        j -= r;
                    } else {
                        v += r * a.ge;
                        if (state == 1) { j -= r; run += r; } else i -= r;
                    }
                    guard += r;
                    // ---- the move out of cell r when the run ends there
                    if (rq == kRunTurn || rq == kRunEnd) {
                        const bool hm = state == 1 || (state == 0 && (nibq & 3u) == 1u);
                        const bool ext = rq == kRunTurn && ((hm ? (nibq >> 2) : (nibq >> 3)) & 1u);
                        v += ext ? a.ge : a.goe;
                        ++guard;
                        state = ext ? (hm ? 1 : 2) : 0;
                        if (hm) {
                            --j;
                            ++run;
                            if (!ext) {   // the insertion run ends: it belongs to slot i
                                if (insrow == i) inssum += run;
                                else {
                                    if (insrow >= 0 && k == 0) {
                                        ins[insrow] = (uint16_t)inssum;
                                        if (gmax) atomicMax(gmax + insrow, inssum);
                                    }
                                    insrow = i;
                                    inssum = run;
                                }
                                run = 0;
                            }
                        } else {
                            --i;
                        }
                    } else if (rq != 0) {
                        why = rq;
                    }
                }
                if (__ballot(why == 0) == 0) break;
            }
            if (why == 7) continue;
            fin = why == kRunFin;
            bad = why == kRunBad;
            if (why != kRunMiss && why != kRunSmiss) continue;
            // ---- refill: lane k loads chunk (block b0 - qb, column gq0 - u), k = qb * NG + u
            const int row0 = i - 1, col0 = j - 1;
            int b0, t0;
            split_row(row0, b0, t0);
            const int qb = k >> lgng, u = k & ngm;
            const int bq = b0 - qb;
            const int cq = (state == 2 || qb == 0) ? col0 : max(col0 - (t0 + 1) - (qb - 1) * R, 0);
            const int gg = grp_of(max(bq, 0), cq) - u;
            const bool ok = bq >= 0 && gg >= 0;
            const int slot = (gg & ngm) | ((bq & nbm) << lgng);
            const int64_t gs = so + col0;
            int64_t nswb = (gs & ~(int64_t)15) - 48;
            if (nswb < 0) nswb = 0;
            // 16 lanes x 4 bytes, none past the aligned 16-byte chunk that holds
            // residue gs (dwords above it repeat that chunk's last one; the path
            // never reads columns right of j - 1)
            const uint32_t wv = *reinterpret_cast<const uint32_t *>(
                a.res + min(nswb + 4 * k, (gs & ~(int64_t)15) + 12));
            uint4 cq4[8];
    #pragma unroll
            for (int h = 0; h < 8; ++h) cq4[h] = make_uint4(0, 0, 0, 0);
            if (ok) {
                const uint4 *src = reinterpret_cast<const uint4 *>(a.codes + chunk_addr(bq, gg));
    #pragma unroll
                for (int h = 0; h < 8; ++h)
                    if (h < 2 * W) cq4[h] = src[h];
            }
            win[k] = wv;
            swb = nswb;
            qoff = (int)(so - swb);
            if (ok) {
                uint4 *dst = reinterpret_cast<uint4 *>(ccache + slot * cws);
    #pragma unroll
                for (int h = 0; h < 8; ++h)
                    if (h < 2 * W) dst[h] = cq4[h];
            }
            ctag[slot] = ok ? make_int2(bq, gg) : make_int2(-1, -1);
        }
        if (k != 0) return;
        if (bad) {
            *cp = make_int4(-1, -1, -1, -1);
            return;
        }
        if (insrow >= 0) {
            ins[insrow] = (uint16_t)inssum;
            if (gmax) atomicMax(gmax + insrow, inssum);
        }
        if (curw >= 0) al[curw] = bits;
        // core insertions sit in slots 1..m-1, so slots 0 and m hold the flanks only
        ins[0] = (uint16_t)j;
        ins[m] = (uint16_t)(n - j1);
        if (gmax) {
            if (j > 0) atomicMax(gmax, j);
            if (n - j1 > 0) atomicMax(gmax + m, n - j1);
        }
        *cp = make_int4(i, j, i1, j1);
    };
    walk_pair();
    if (glds) {
        __syncthreads();
        for (int x = threadIdx.x; x <= m; x += 256) {
            const int gv = sG[x];
            // G only grows, so a stale read can only let an atomic through
            if (gv > 0 && gv > __hip_atomic_load(a.G + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(a.G + x, gv);
        }
    }
}

}  // namespace hk
