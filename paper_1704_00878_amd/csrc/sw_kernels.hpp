// Smith-Waterman forward kernels and the traceback walk for gfx950.
//
// Recurrence (eq. 1-2 of the paper with W_k = go + ge*k, in Gotoh's affine
// form): E(i,j) = max(E(i,j-1) - ge, H(i,j-1) - goe), F(i,j) = max(F(i-1,j) -
// ge, H(i-1,j) - goe), H(i,j) = max(0, H(i-1,j-1) + S[c_i][s_j], E, F), goe =
// go + ge, H(i,0) = H(0,j) = 0.
//
// Register form used by every kernel (exact for H):
//   Hg = H - goe is carried instead of H, so the profile holds S + goe and the
//   diagonal term is Hg(i-1,j-1) + P;  E and F are carried clamped at 0
//   (E* = max(E, 0), F* = max(F, 0)), which leaves H unchanged because H >= 0.
// Per cell: 7 VALU ops (sub, max3, sub, max3, add, max3, sub).
//
// Traceback code (4 bits per cell, a pure function of the DP values):
//   bit0 notd = H != H(i-1,j-1) + S      (diagonal not a source)
//   bit1 note = H != E                  (horizontal gap not a source)
//   bit2 eext = E(i,j-1) - ge > H(i,j-1) - goe   (strict: open wins ties)
//   bit3 fext = F(i-1,j) - ge > H(i-1,j) - goe
// Each bit is the sign of a difference shifted in with one v_alignbit.  With
// clamped E/F these bits can differ from the unclamped ones only at cells
// whose gap value is <= 0, which the walk never visits (a cell is entered in
// a gap state only when that gap value equals H > 0).
//
// End cell: max H, ties to the smallest j, then the smallest i.  Kernels form
// key = (H << 5) | (31 - t) for the T rows of a column, take the max over the
// column (max H, then min row); the running best moves on a strictly larger H,
// or on an equal H at a smaller j (a later strip or pass, which holds larger i).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int kPad = 31;             // residue code of padding columns / alphabet filler
constexpr int kAlphaMax = 32;
constexpr int kNegProf = -(1 << 22); // profile value of padding: never a source

// shift the sign bit of d into the low end of w
__device__ __forceinline__ uint32_t push_sign(uint32_t w, int d) {
    return __builtin_amdgcn_alignbit(w, (uint32_t)d, 31);
}

// One DP cell.  hg: Hg(i,j-1) in, Hg(i,j) out.  e: E*(i,j-1) in, E*(i,j) out.
// diag: Hg(i-1,j-1) in, replaced by Hg(i,j-1) (the next row's diagonal).
// upg/upf: Hg(i-1,j), F*(i-1,j) in; replaced by this cell's Hg, F* (next row).
template <bool TB>
__device__ __forceinline__ int sw_cell(int &hg, int &e, int &diag, int &upg, int &upf,
                                       int p, int ge, int goe, uint32_t &word) {
    const int eext = e - ge;
    const int en = max(max(eext, hg), 0);
    const int fext = upf - ge;
    const int fn = max(max(fext, upg), 0);
    const int hd = diag + p;
    const int h = max(max(hd, en), fn);
    if (TB) {
        word = push_sign(word, upg - fext);   // fext
        word = push_sign(word, hg - eext);    // eext
        word = push_sign(word, en - h);       // note
        word = push_sign(word, hd - h);       // notd
    }
    diag = hg;
    hg = h - goe;
    e = en;
    upg = hg;
    upf = fn;
    return h;
}

struct BestCell {   // running end cell of one lane
    int h, j, i;
};

__device__ __forceinline__ bool better(int h, int j, int i, const BestCell &b) {
    return h > b.h || (h == b.h && (j < b.j || (j == b.j && i < b.i)));
}

// ---------------------------------------------------------------------------
// Intra-task kernel: one pair per wavefront.  Lane l owns center rows
// [row0 + l*R, row0 + l*R + R) of a pass of 64*R rows and works on column
// j = k - l + 1 at step k (a skewed wavefront).  The bottom row of lane l-1
// reaches lane l through DPP wave_shr:1 one step later; the residue stream
// enters at lane 0 and moves down the same way.  Passes over m > 64*R chain
// through a per-pair boundary row in global scratch.
//
// The query profile P[r][i] = S[c_i][r] + goe (int32, 32 x mpad) is built once
// per workgroup in LDS and shared by its waves; wave w of the grid takes the
// w-th pair of the (longest first) order.
//
// Codes: word (u32, R nibbles) per (pass, step k, lane):
//   codes[cbase + (pass*(n+63) + k)*64 + lane], row t nibble at 4*(R-1-t).
// ---------------------------------------------------------------------------
struct IntraArgs {
    const int8_t *mat;        // alpha x alpha
    int alpha;
    const uint8_t *center;    // m residues
    int m, mpad, passes;
    const uint8_t *res;
    const int64_t *off;
    const int32_t *order;     // pair indices, processing order
    int npairs;
    int ge, goe;
    int *counter;             // work counter (zeroed before launch)
    int32_t *score;           // [N]
    int32_t *endcell;         // [N][2] (i1, j1) or null
    uint32_t *codes;          // code words or null
    const int64_t *code_base; // per pair (indexed by pair id) or null
    int2 *bound;              // boundary rows for passes > 0
    const int64_t *bound_base;// per pair or null
};

template <int R, bool TB, bool ENDC>
__global__ void __launch_bounds__(512)
sw_intra_kernel(IntraArgs a) {
    extern __shared__ int prof[];   // [32][mpad]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nthreads = blockDim.x;
    // build P'[r][i] = S[c_i][r] + goe, padding -> kNegProf
    for (int x = tid; x < kAlphaMax * a.mpad; x += nthreads) {
        const int r = x / a.mpad, i = x - r * a.mpad;
        int v = kNegProf;
        if (r < a.alpha && i < a.m) v = (int)a.mat[a.center[i] * a.alpha + r] + a.goe;
        prof[x] = v;
    }
    __syncthreads();

    const int ge = a.ge, goe = a.goe;
    // one pair per wave, longest pairs in the lowest workgroups
    const int w = blockIdx.x * (nthreads >> 6) + (tid >> 6);
    if (w < a.npairs) {
        // every lane loads the same value: readfirstlane only moves it to SGPRs
        const int pid = __builtin_amdgcn_readfirstlane(a.order[w]);
        const int64_t so = a.off[pid];
        const int n = __builtin_amdgcn_readfirstlane((int)(a.off[pid + 1] - so));
        const uint8_t *s = a.res + so;
        const int steps = n + 63;
        BestCell best{0, 0x7fffffff, 0x7fffffff};
        int hmax = 0;
        for (int pass = 0; pass < a.passes; ++pass) {
            const int row0 = pass * 64 * R;
            const int myrow = row0 + lane * R;
            int hg[R], e[R];
#pragma unroll
            for (int t = 0; t < R; ++t) { hg[t] = -goe; e[t] = 0; }
            int botg = -goe, botf = 0;  // this lane's bottom row values (last step)
            int diag0 = -goe;           // Hg(myrow-1, j-1) for row 0
            int rcur = kPad;            // residue of this lane's column
            int rbuf = kPad;            // residues s[kb .. kb+63] across lanes
            int2 bbuf = make_int2(-goe, 0);
            const int2 *bin = (pass > 0) ? a.bound + a.bound_base[pid] + (int64_t)(pass - 1) * n : nullptr;
            int2 *bout = (pass + 1 < a.passes) ? a.bound + a.bound_base[pid] + (int64_t)pass * n : nullptr;
            uint32_t *cw = TB ? a.codes + a.code_base[pid] + (int64_t)pass * steps * 64 : nullptr;
            const int *prow_base = prof + myrow;
            for (int k = 0; k < steps; ++k) {
                if ((k & 63) == 0) {
                    const int kk = k + lane;
                    rbuf = (kk < n) ? (int)(s[kk] & 31) : kPad;
                    if (bin) bbuf = (kk < n) ? bin[kk] : make_int2(-goe, 0);
                }
                const int rin = __builtin_amdgcn_readlane(rbuf, k & 63);
                int tg = -goe, tf = 0;
                if (bin) {
                    tg = __builtin_amdgcn_readlane(bbuf.x, k & 63);
                    tf = __builtin_amdgcn_readlane(bbuf.y, k & 63);
                }
                // lane l <- lane l-1 (lane 0 keeps the boundary value)
                rcur = __builtin_amdgcn_update_dpp(rin, rcur, 0x138, 0xf, 0xf, false);
                int upg = __builtin_amdgcn_update_dpp(tg, botg, 0x138, 0xf, 0xf, false);
                int upf = __builtin_amdgcn_update_dpp(tf, botf, 0x138, 0xf, 0xf, false);
                int diag = diag0;
                diag0 = upg;
                const int *prow = prow_base + rcur * a.mpad;
                int p[R];
#pragma unroll
                for (int t = 0; t < R; ++t) p[t] = prow[t];
                uint32_t word = 0;
                int colkey = 0;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    const int h = sw_cell<TB>(hg[t], e[t], diag, upg, upf, p[t], ge, goe, word);
                    if (ENDC) colkey = max(colkey, (h << 5) | (31 - t));
                    else hmax = max(hmax, h);
                }
                botg = upg;
                botf = upf;
                const int j = k - lane + 1;
                if (TB) cw[(int64_t)k * 64 + lane] = word;
                if (bout && lane == 63 && j >= 1 && j <= n) bout[j - 1] = make_int2(botg, botf);
                if (ENDC) {
                    // later passes hold larger i: on equal H they win only with a smaller j
                    const int ch = colkey >> 5;
                    if (ch > 0 && (ch > best.h || (ch == best.h && j < best.j))) {
                        best.h = ch;
                        best.j = j;
                        best.i = myrow + (31 - (colkey & 31));
                    }
                }
            }
        }
        if (ENDC) {
            // wave reduction: max h, then min j, then min i
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) {
                const int oh = __shfl_xor(best.h, sh);
                const int oj = __shfl_xor(best.j, sh);
                const int oi = __shfl_xor(best.i, sh);
                if (better(oh, oj, oi, best)) { best.h = oh; best.j = oj; best.i = oi; }
            }
            if (lane == 0) {
                a.score[pid] = best.h;
                if (a.endcell) {
                    a.endcell[2 * pid] = best.h > 0 ? best.i + 1 : 0;
                    a.endcell[2 * pid + 1] = best.h > 0 ? best.j : 0;
                }
            }
        } else {
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) hmax = max(hmax, __shfl_xor(hmax, sh));
            if (lane == 0) a.score[pid] = hmax;
        }
    }
}

// ---------------------------------------------------------------------------
// Inter-task kernel: one pair per lane, 64 pairs per wavefront (one wave per
// workgroup, persistent over groups).  Lane-private state is a strip of T=16
// center rows; the wave sweeps j over the group's longest sequence, strip by
// strip.  The strip's profile (32 x 16 int32, stride 20) is rebuilt in LDS per
// strip from the group's center, so a group may use the batch center or any
// sequence of the set as its center (center selection, training targets).
// Strip boundaries (Hg, F* of the strip's last row for every j) go through a
// per-workgroup scratch row, read with agent-scope loads so that no stale L1
// line is seen.
//
// Codes: u64 (two u32 words: rows 0-7, 8-15) per (strip s, column j, lane):
//   codes[gbase + ((s*nmax + j-1)*64 + lane)*2 + half], row t nibble at
//   4*(7 - t%8).
// ---------------------------------------------------------------------------
constexpr int kT = 16;
constexpr int kPS = kT + 4;  // LDS row stride of the strip profile

struct InterArgs {
    const int8_t *mat;
    int alpha;
    const uint8_t *center;    // batch center (mode 0)
    int m;
    const uint8_t *res;
    const int64_t *off;
    int mode;                 // 0 batch, 1 all pairs (a < b), 2 anchored groups
    const int32_t *order;     // mode 0: 64 * ngroups pair ids (-1 = empty lane)
    const int32_t *gnmax;     // mode 0: per group longest sequence (code layout)
    const int32_t *gcen;      // mode 1: center position in perm; mode 2: center seq id
    const int32_t *gb0;       // modes 1/2: first partner position in perm
    const int32_t *perm;      // modes 1/2: sequence ids sorted by length
    int nseq;
    const int32_t *gslot;     // mode 2: sums slot of the group's center
    int64_t *sums;            // modes 1/2: integer score sums (atomic adds)
    int ngroups;
    int ge, goe;
    int *counter;
    int32_t *score;           // mode 0: per pair id; mode 2: per lane slot (optional)
    int32_t *endcell;
    uint32_t *codes;
    const int64_t *gcode_base;// per group (u32 words)
    int2 *bound;              // per workgroup slot: bstride int2
    int64_t bstride;          // >= 64 * max nmax
};

__device__ __forceinline__ int2 load_agent(const int2 *p) {
    uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    return make_int2((int)(uint32_t)v, (int)(uint32_t)(v >> 32));
}

template <bool TB, bool ENDC>
__global__ void __launch_bounds__(64)
sw_inter_kernel(InterArgs a) {
    __shared__ int prof[kAlphaMax * kPS];
    __shared__ int8_t smat[kAlphaMax * kAlphaMax];
    const int lane = threadIdx.x;
    for (int x = lane; x < kAlphaMax * kAlphaMax; x += 64) {
        const int r = x >> 5, q = x & 31;
        smat[x] = (r < a.alpha && q < a.alpha) ? a.mat[r * a.alpha + q] : (int8_t)0;
    }
    int2 *bnd = a.bound + (int64_t)blockIdx.x * a.bstride;
    const int ge = a.ge, goe = a.goe;
    __shared__ int s_next;
    for (;;) {
        // fetch the next group: one atomic by lane 0, broadcast through LDS
        __syncthreads();
        if (lane == 0) s_next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int g = __builtin_amdgcn_readfirstlane(s_next);
        if (g >= a.ngroups) break;
        int pid = -1;       // output slot (mode 0: pair id)
        int sid = -1;       // sequence of this lane
        const uint8_t *cen = a.center;
        int m = a.m;
        int cid = -1;
        if (a.mode == 0) {
            pid = a.order[(int64_t)g * 64 + lane];
            sid = pid;
        } else {
            const int bpos = a.gb0[g] + lane;
            cid = a.mode == 1 ? a.perm[a.gcen[g]] : a.gcen[g];
            if (bpos < a.nseq) {
                sid = a.perm[bpos];
                pid = g * 64 + lane;          // output slot; a self pair scores 0
                if (sid == cid) sid = -1;
            }
            cen = a.res + a.off[cid];
            m = (int)(a.off[cid + 1] - a.off[cid]);
        }
        const int64_t so = sid >= 0 ? a.off[sid] : 0;
        const int n = sid >= 0 ? (int)(a.off[sid + 1] - so) : 0;
        const uint8_t *s = a.res + so;
        int nmax = n;
        if (a.mode == 0) {
            nmax = a.gnmax[g];
        } else {
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) nmax = max(nmax, __shfl_xor(nmax, sh));
        }
        m = __builtin_amdgcn_readfirstlane(m);        // same in every lane
        nmax = __builtin_amdgcn_readfirstlane(nmax);  // same in every lane
        const int nstrips = (m + kT - 1) / kT;
        uint32_t *cw = TB ? a.codes + a.gcode_base[g] : nullptr;
        BestCell best{0, 0x7fffffff, 0x7fffffff};
        int hmax = 0;
        for (int st = 0; st < nstrips; ++st) {
            const int i0 = st * kT;
            __syncthreads();
            for (int x = lane; x < kAlphaMax * kT; x += 64) {
                const int r = x / kT, t = x - r * kT;
                int v = kNegProf;
                if (r < a.alpha && i0 + t < m) v = (int)smat[(cen[i0 + t] & 31) * 32 + r] + goe;
                prof[r * kPS + t] = v;
            }
            __syncthreads();
            int hg[kT], e[kT];
#pragma unroll
            for (int t = 0; t < kT; ++t) { hg[t] = -goe; e[t] = 0; }
            int diag0 = -goe;
            for (int j = 1; j <= nmax; ++j) {
                const int r = (j <= n) ? (int)(s[j - 1] & 31) : kPad;
                int upg = -goe, upf = 0;
                int2 *bp = bnd + (int64_t)(j - 1) * 64 + lane;
                if (st > 0) { const int2 v = load_agent(bp); upg = v.x; upf = v.y; }
                int diag = diag0;
                diag0 = upg;
                const int *prow = prof + r * kPS;
                int p[kT];
#pragma unroll
                for (int t = 0; t < kT; ++t) p[t] = prow[t];
                uint32_t w0 = 0, w1 = 0;
                int colkey = 0;
#pragma unroll
                for (int t = 0; t < kT; ++t) {
                    const int h = sw_cell<TB>(hg[t], e[t], diag, upg, upf, p[t], ge, goe,
                                              t < 8 ? w0 : w1);
                    if (ENDC) colkey = max(colkey, (h << 5) | (31 - t));
                    else hmax = max(hmax, h);
                }
                if (st + 1 < nstrips) *bp = make_int2(upg, upf);
                if (TB) {
                    uint2 *dst = reinterpret_cast<uint2 *>(cw) + ((int64_t)st * nmax + (j - 1)) * 64 + lane;
                    *dst = make_uint2(w0, w1);
                }
                if (ENDC) {
                    // later strips hold larger i: on equal H they win only with a smaller j
                    const int ch = colkey >> 5;
                    if (ch > 0 && (ch > best.h || (ch == best.h && j < best.j))) {
                        best.h = ch;
                        best.j = j;
                        best.i = i0 + (31 - (colkey & 31));
                    }
                }
            }
        }
        if (ENDC) hmax = best.h;
        if (a.mode == 0) {
            if (pid >= 0) {
                a.score[pid] = hmax;
                if (ENDC && a.endcell) {
                    a.endcell[2 * pid] = best.h > 0 ? best.i + 1 : 0;
                    a.endcell[2 * pid + 1] = best.h > 0 ? best.j : 0;
                }
            }
        } else {
            const int v = sid >= 0 ? hmax : 0;
            if (a.score && pid >= 0) a.score[pid] = v;
            if (a.mode == 1 && sid >= 0) atomicAdd(reinterpret_cast<unsigned long long *>(a.sums + sid), (unsigned long long)v);
            int tot = v;
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) tot += __shfl_xor(tot, sh);
            if (lane == 0) {
                const int slot = a.mode == 1 ? cid : a.gslot[g];
                atomicAdd(reinterpret_cast<unsigned long long *>(a.sums + slot), (unsigned long long)(int64_t)tot);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Traceback walk: one lane per pair.  From the end cell, in state H: stop when
// the running value is 0, else take the diagonal if notd is clear, else the
// horizontal gap if note is clear, else the vertical gap; in a gap state,
// extend while the ext bit is set (open wins ties).  The running value is
// H (or the gap value) of the current cell, kept exactly from the score.
// Emits the center-star vector: ins[k][0..m], aligned bits, cells.
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
    // layout descriptor per pair id: kind 0 = intra (R rows/lane), 1 = inter
    const int64_t *cbase;     // word base per pair
    const int32_t *cstride;   // intra: steps (n+63); inter: nmax
    int R;                    // intra rows per lane
    int kind;
    int32_t *cells;           // [N][4]
    uint16_t *ins;            // [N][m+1] (zeroed)
    uint32_t *aligned;        // [N][aw] (zeroed)
    int aw;
};

__device__ __forceinline__ uint32_t code_at(const WalkArgs &a, int64_t base, int stride, int i, int j) {
    const int row = i - 1;
    if (a.kind == 0) {
        const int span = 64 * a.R;
        const int pass = row / span;
        const int rr = row - pass * span;
        const int ln = rr / a.R, t = rr - ln * a.R;
        const int k = j - 1 + ln;
        const uint32_t w = a.codes[base + ((int64_t)pass * stride + k) * 64 + ln];
        return (w >> (4 * (a.R - 1 - t))) & 15u;
    } else {
        const int st = row >> 4, t = row & 15;
        const uint32_t w = a.codes[base + (((int64_t)st * stride + (j - 1)) * 64) * 2 + (t >> 3)];
        return (w >> (4 * (7 - (t & 7)))) & 15u;
    }
}

__global__ void __launch_bounds__(256)
walk_kernel(WalkArgs a) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= a.npairs) return;
    const int pid = a.pids[w];
    const int64_t so = a.off[pid];
    const int n = (int)(a.off[pid + 1] - so);
    const uint8_t *s = a.res + so;
    const int m = a.m;
    uint16_t *ins = a.ins + (int64_t)pid * (m + 1);
    uint32_t *al = a.aligned + (int64_t)pid * a.aw;
    int v = a.score[pid];
    if (v <= 0) {
        ins[0] = (uint16_t)n;
        int4 *cp = reinterpret_cast<int4 *>(a.cells) + pid;
        *cp = make_int4(0, 0, 0, 0);
        return;
    }
    const int i1 = a.endcell[2 * pid], j1 = a.endcell[2 * pid + 1];
    const int64_t base = a.cbase[pid];
    const int stride = a.cstride[pid];
    int i = i1, j = j1;
    int state = 0;              // 0 = H, 1 = E, 2 = F
    int run = 0;                // pending insertions at row i
    int curw = -1;              // aligned word being accumulated
    uint32_t bits = 0;
    bool bad = (i1 < 1 || i1 > m || j1 < 1 || j1 > n);
    // a path has at most m + n steps; the guard keeps a corrupted code
    // stream from reading outside the matrix or looping
    for (int guard = 0; !bad; ++guard) {
        if (guard > m + n + 2 || i < 0 || j < 0) { bad = true; break; }
        if (state != 0 && (i < 1 || j < 1)) { bad = true; break; }
        if (state == 0) {
            if (v == 0) break;
            if (i < 1 || j < 1) { bad = true; break; }
            const uint32_t nib = code_at(a, base, stride, i, j);
            if (!(nib & 1u)) {
                const int p = i - 1;
                const int wi = p >> 5;
                if (wi != curw) {
                    if (curw >= 0) al[curw] = bits;
                    curw = wi;
                    bits = 0;
                }
                bits |= 1u << (p & 31);
                v -= (int)a.mat[a.center[i - 1] * a.alpha + s[j - 1]];
                --i;
                --j;
            } else if (!(nib & 2u)) {
                state = 1;
            } else {
                state = 2;
            }
        } else if (state == 1) {
            const uint32_t nib = code_at(a, base, stride, i, j);
            ++run;
            --j;
            if (nib & 4u) {
                v += a.ge;
            } else {
                v += a.goe;
                state = 0;
                ins[i] = (uint16_t)(ins[i] + run);
                run = 0;
            }
        } else {
            const uint32_t nib = code_at(a, base, stride, i, j);
            --i;
            if (nib & 8u) v += a.ge;
            else { v += a.goe; state = 0; }
        }
    }
    if (bad) {
        int4 *cp = reinterpret_cast<int4 *>(a.cells) + pid;
        *cp = make_int4(-1, -1, -1, -1);
        return;
    }
    if (curw >= 0) al[curw] = bits;
    ins[0] = (uint16_t)(ins[0] + j);
    ins[m] = (uint16_t)(ins[m] + (n - j1));
    int4 *cp = reinterpret_cast<int4 *>(a.cells) + pid;
    *cp = make_int4(i, j, i1, j1);
}

}  // namespace hk
