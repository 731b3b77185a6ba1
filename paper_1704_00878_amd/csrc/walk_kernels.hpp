// Traceback walk for gfx950: one lane per pair over the 4-bit codes written
// by the wavefront kernel (sw_kernels.hpp) or the strip kernel
// (strip_kernels.hpp), emitting the center-star vector of each pair.
#pragma once
#include "sw_kernels.hpp"

namespace hk {

// ---------------------------------------------------------------------------
// Traceback walk: one lane per pair.  From the end cell, in state H: stop when
// the running value is 0, else take the diagonal if notd is clear, else the
// horizontal gap if note is clear, else the vertical gap; in a gap state,
// extend while the ext bit is set (open wins ties).  The running value is
// H (or the gap value) of the current cell, kept exactly from the score.
// Emits the center-star vector: ins[k][0..m], aligned bits, cells.
//
// Code words arrive in 32-byte chunks (8 steps of one lane of the wavefront
// layout, or 4 columns of one lane of the strip layout) held in a two-entry
// per-lane LDS cache, so a diagonal run costs one line fetch per chunk.
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
};

constexpr int kWalkCenterLds = 8192;   // centers up to this length are staged in LDS

// One lane per pair.  Each lane keeps four 32-byte code chunks and a 64-byte
// window of its sequence in LDS: on a miss it loads the chunk it needs, the
// one to its left and the two that a diagonal path meets in the block above
// (and refreshes the sequence window), in one round trip.  Lanes advance
// through their cached data until each misses or ends, so that one memory
// round trip serves the misses of every lane of the wavefront.
template <bool STRIP, bool CEN_LDS, bool PK>
__global__ void __launch_bounds__(64)
walk_kernel(WalkArgs a) {
    constexpr int CW = PK ? 32 : 16;   // words per cached chunk (8 steps x W, W <= 4 packed, <= 2 otherwise)
    constexpr int HQ = CW / 4;
    __shared__ uint32_t cache[4][CW][64];
    __shared__ uint32_t swin[16][64];
    __shared__ int8_t smat[32 * 32];
    __shared__ uint8_t scen[kWalkCenterLds];
    const int lane = threadIdx.x;
    const int m = a.m;
    constexpr bool cen_lds = CEN_LDS;
    for (int x = lane; x < 1024; x += 64) {
        const int r = x >> 5, q = x & 31;
        smat[x] = (r < a.alpha && q < a.alpha) ? a.mat[r * a.alpha + q] : (int8_t)0;
    }
    if (cen_lds)
        for (int x = lane; x < m; x += 64) scen[x] = a.center[x] & 31;
    __syncthreads();
    const int w = blockIdx.x * 64 + lane;
    if (w >= a.npairs) return;
    const int pid = STRIP ? a.pids[w] : a.slot_pid[w];
    const int64_t so = a.off[pid];
    const int n = (int)(a.off[pid + 1] - so);
    // window of residue bytes [swb, swb + 64) of the residue array, read as
    // four aligned 16-byte chunks that each hold a byte at or below the
    // position in use (so no read leaves the array's last page)
    int64_t swb = -1024;
    uint16_t *ins = a.ins + (int64_t)pid * (m + 1);
    uint32_t *al = a.aligned + (int64_t)pid * a.aw;
    int v = a.score[pid];
    int4 *cp = reinterpret_cast<int4 *>(a.cells) + pid;
    int32_t *gmax = (a.G && pid != a.gskip) ? a.G : nullptr;
    if (v <= 0) {
        ins[0] = (uint16_t)n;
        if (gmax && n > 0) atomicMax(gmax, n);
        *cp = make_int4(0, 0, 0, 0);
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
    const int G = strip ? (stride + 3) >> 2 : (stride + 7) >> 3;   // groups per pass / strip
    // wavefront layout: LS lanes per stream, W words (8 steps x W words per chunk)
    const int lg = strip ? 6 : a.lg_ls, LSm = (1 << lg) - 1;
    const int W = strip ? 1 : a.W;
    const int n0 = min(R, 8);           // rows in the first word of a step
    int i = i1, j = j1;
    // row decomposition of i-1: block (pass*LS + lane, or strip) and row t in block
    int blk = 0, t = 0;
    {
        const int row = i - 1;
        if (strip) { blk = row >> 4; t = row & 15; }
        else {
            const int span = R << lg, ps = row / span, rr = row - ps * span;
            blk = (ps << lg) + rr / R;
            t = rr % R;
        }
    }
    // chunk (block b, group g): group of 4 columns (strip) or 8 wavefront steps
    auto grp_of = [&](int b, int jj) __attribute__((always_inline)) -> int {
        return strip ? (jj - 1) >> 2 : (ccol + jj - 1 + (b & LSm)) >> 3;
    };
    auto chunk_addr = [&](int b, int g) __attribute__((always_inline)) -> int64_t {
        return strip ? base + (((int64_t)b * G + g) * 64 + ccol) * 8
                     : base + ((((int64_t)(b >> lg) * G + g) << lg) + (b & LSm)) * 8 * W;
    };
    int tb0 = -1, tg0 = -1, tb1 = -1, tg1 = -1, tb2 = -1, tg2 = -1, tb3 = -1, tg3 = -1;
    int state = 0;              // 0 = H, 1 = E, 2 = F
    int run = 0;                // pending insertions at row i
    int insrow = -1, inssum = 0;
    int curw = -1;              // aligned word being accumulated
    uint32_t bits = 0;
    // stores found inside the stepping loop wait in one pending slot each and
    // are issued between rounds, so the loop itself touches only LDS
    int pw = -1, pir = -1, piv = 0;
    uint32_t pb = 0;
    bool bad = (i1 < 1 || i1 > m || j1 < 1 || j1 > n);
    bool fin = false;
    int guard = 0;
    // a path has at most m + n steps; the guard keeps a corrupted code
    // stream from reading outside the matrix or looping
    while (!bad && !fin) {
        bool smiss = false;
        bool cmiss = false;
        while (true) {
            // everything about the current cell, then one exit test
            const int grp = grp_of(blk, j);
            const bool h0 = tb0 == blk && tg0 == grp, h1 = tb1 == blk && tg1 == grp;
            const bool h2 = tb2 == blk && tg2 == grp, h3 = tb3 == blk && tg3 == grp;
            const int sl = h0 ? 0 : (h1 ? 1 : (h2 ? 2 : 3));
            int wi, sh;
            if (strip) { wi = ((j - 1) & 3) * 2 + (t >> 3); sh = 4 * (7 - (t & 7)); }
            else {
                if (PK) {
                    wi = ((ccol + j - 1 + (blk & LSm)) & 7) * W + (t >> 2);
                    sh = 8 * half + 2 * (t & 3);
                } else {
                    wi = ((ccol + j - 1 + (blk & LSm)) & 7) * W + (t >> 3);
                    sh = t < 8 ? 4 * (n0 - 1 - t) : 4 * (R - 1 - t);
                }
            }
            const uint32_t cword = cache[sl][wi & (CW - 1)][lane];
            // notd, note, eext, fext in bits 0-3 (packed layout: two bit pairs 16 apart)
            const uint32_t nib = PK ? ((cword >> (sh & 15)) & 3u) | (((cword >> ((sh & 15) + 16)) & 3u) << 2)
                                    : (cword >> (sh & 31)) & 15u;
            const int gq = (int)(so + j - 1 - swb);
            const int gqc = min(max(gq, 0), 63);
            const int ic = min(max(i - 1, 0), m - 1);
            const int cr = cen_lds ? (int)scen[ic] : (int)(a.center[ic] & 31);
            const int sr = (int)((swin[gqc >> 2][lane] >> (8 * (gqc & 3))) & 31u);
            const int sd = (int)smat[cr * 32 + sr];
            const bool stop = state == 0 && v == 0;
            const bool badc = guard > m + n + 2 || i < 1 || j < 1;
            const bool miss = !(h0 || h1 || h2 || h3);
            // the move out of this cell: diagonal, horizontal (E) or vertical
            // (F); a switch from H into E or F moves in the same step
            const bool dm = state == 0 && !(nib & 1u);
            const bool hm = state == 1 || (state == 0 && (nib & 3u) == 1u);
            const bool sm = dm && (gq < 0 || gq >= 64);
            const bool ext = hm ? (nib & 4u) != 0 : (nib & 8u) != 0;
            const bool fa = dm && curw >= 0 && ((i - 1) >> 5) != curw && pw >= 0;
            const bool fi = hm && !ext && insrow >= 0 && insrow != i && pir >= 0;
            if (stop || badc || miss || sm || fa || fi) {
                fin = stop;
                bad = !stop && badc;
                cmiss = !stop && !badc && miss;
                smiss = !stop && !badc && !miss && sm;
                break;
            }
            ++guard;
            v += dm ? -sd : (ext ? a.ge : a.goe);
            if (dm) {
                const int p = i - 1;
                if ((p >> 5) != curw) {
                    if (curw >= 0) { pw = curw; pb = bits; }
                    curw = p >> 5;
                    bits = 0;
                }
                bits |= 1u << (p & 31);
            }
            run += hm ? 1 : 0;
            if (hm && !ext) {   // the insertion run ends: it belongs to slot i
                if (insrow == i) {
                    inssum += run;
                } else {
                    if (insrow >= 0) { pir = insrow; piv = inssum; }
                    insrow = i;
                    inssum = run;
                }
                run = 0;
            }
            state = dm ? 0 : (ext ? (hm ? 1 : 2) : 0);
            const bool di = !hm, dj = hm || dm;
            i -= di ? 1 : 0;
            j -= dj ? 1 : 0;
            const bool wrap = di && t == 0;
            t = wrap ? R - 1 : t - (di ? 1 : 0);
            blk -= wrap ? 1 : 0;
        }
        if (pw >= 0) { al[pw] = pb; pw = -1; }
        if (pir >= 0) {
            ins[pir] = (uint16_t)piv;
            if (gmax) atomicMax(gmax + pir, piv);
            pir = -1;
        }
        if (bad || fin) break;
        if (!cmiss && !smiss) continue;   // the loop stopped only to issue stores
        // the sequence window: moved when it no longer holds the 16 residues
        // at and below j - 1; reloaded with every code miss (one round trip)
        const int64_t gs = so + j - 1;
        int64_t nswb = swb;
        if (smiss || gs - 15 < swb || gs >= swb + 64) {
            nswb = (gs & ~(int64_t)15) - 48;
            if (nswb < 0) nswb = 0;
        }
        const uint4 *src = reinterpret_cast<const uint4 *>(a.res + nswb);
        const uint4 s0 = src[0], s1 = src[1], s2 = src[2], s3 = src[3];
        if (smiss) {
            swin[0][lane] = s0.x; swin[1][lane] = s0.y; swin[2][lane] = s0.z; swin[3][lane] = s0.w;
            swin[4][lane] = s1.x; swin[5][lane] = s1.y; swin[6][lane] = s1.z; swin[7][lane] = s1.w;
            swin[8][lane] = s2.x; swin[9][lane] = s2.y; swin[10][lane] = s2.z; swin[11][lane] = s2.w;
            swin[12][lane] = s3.x; swin[13][lane] = s3.y; swin[14][lane] = s3.z; swin[15][lane] = s3.w;
            swb = nswb;
            continue;
        }
        // miss at (blk, grp(j)): load it, its left neighbour, and the two
        // chunks of the block above where a diagonal path enters it
        const int g0 = grp_of(blk, j);
        const int jn = j - (t + 1);
        const int g2 = (blk >= 1 && jn >= 1) ? grp_of(blk - 1, jn) : -1;
        const int64_t ad0 = chunk_addr(blk, g0);
        const int64_t ad1 = g0 >= 1 ? chunk_addr(blk, g0 - 1) : ad0;
        const int64_t ad2 = g2 >= 0 ? chunk_addr(blk - 1, g2) : ad0;
        const int64_t ad3 = g2 >= 1 ? chunk_addr(blk - 1, g2 - 1) : ad0;
        uint4 cq[4][HQ];
#pragma unroll
        for (int h = 0; h < HQ; ++h) cq[0][h] = cq[1][h] = cq[2][h] = cq[3][h] = make_uint4(0, 0, 0, 0);
        {
            const uint4 *q0 = reinterpret_cast<const uint4 *>(a.codes + ad0);
            const uint4 *q1 = reinterpret_cast<const uint4 *>(a.codes + ad1);
            const uint4 *q2 = reinterpret_cast<const uint4 *>(a.codes + ad2);
            const uint4 *q3 = reinterpret_cast<const uint4 *>(a.codes + ad3);
            cq[0][0] = q0[0]; cq[0][1] = q0[1];
            cq[1][0] = q1[0]; cq[1][1] = q1[1];
            cq[2][0] = q2[0]; cq[2][1] = q2[1];
            cq[3][0] = q3[0]; cq[3][1] = q3[1];
            if (PK) {
#pragma unroll
                for (int h = 2; h < HQ; ++h)
                    if (h < 2 * W) {
                        cq[0][h] = q0[h];
                        cq[1][h] = q1[h];
                        cq[2][h] = q2[h];
                        cq[3][h] = q3[h];
                    }
            } else if (W == 2) {
                cq[0][2] = q0[2]; cq[0][3] = q0[3];
                cq[1][2] = q1[2]; cq[1][3] = q1[3];
                cq[2][2] = q2[2]; cq[2][3] = q2[3];
                cq[3][2] = q3[2]; cq[3][3] = q3[3];
            }
        }
        swin[0][lane] = s0.x; swin[1][lane] = s0.y; swin[2][lane] = s0.z; swin[3][lane] = s0.w;
        swin[4][lane] = s1.x; swin[5][lane] = s1.y; swin[6][lane] = s1.z; swin[7][lane] = s1.w;
        swin[8][lane] = s2.x; swin[9][lane] = s2.y; swin[10][lane] = s2.z; swin[11][lane] = s2.w;
        swin[12][lane] = s3.x; swin[13][lane] = s3.y; swin[14][lane] = s3.z; swin[15][lane] = s3.w;
        swb = nswb;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int h = 0; h < HQ; ++h) {
                if (h < 2 || (PK ? h < 2 * W : W == 2)) {
                    cache[c][4 * h + 0][lane] = cq[c][h].x;
                    cache[c][4 * h + 1][lane] = cq[c][h].y;
                    cache[c][4 * h + 2][lane] = cq[c][h].z;
                    cache[c][4 * h + 3][lane] = cq[c][h].w;
                }
            }
        }
        tb0 = blk; tg0 = g0;
        tb1 = g0 >= 1 ? blk : -1; tg1 = g0 - 1;
        tb2 = g2 >= 0 ? blk - 1 : -1; tg2 = g2;
        tb3 = g2 >= 1 ? blk - 1 : -1; tg3 = g2 - 1;
    }
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
}

}  // namespace hk
