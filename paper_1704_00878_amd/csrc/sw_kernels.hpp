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
#include <type_traits>

namespace hk {

constexpr int kPad = 31;             // residue code of padding columns / alphabet filler
constexpr int kAlphaMax = 32;
constexpr int kNegProf = -(1 << 22); // profile value of padding: never a source

// v_max3_i32 (the compiler splits max(max(a,b),c) into a signed and an
// unsigned max once it knows two operands are non-negative)
__device__ __forceinline__ int vmax3(int a, int b, int c) {
    int r;
    asm("v_max3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

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
    const int h = vmax3(hd, en, fn);
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
// Intra-task (wavefront) kernel: each stream of LS lanes (LS = 64, 32 or 16,
// so a wavefront runs 64/LS streams side by side) works through a list of
// pairs.  Lane l of a stream owns center rows [row0 + l*R, row0 + l*R + R)
// of a pass of LS*R rows and works on stream column K = k - l at step k (a
// skewed wavefront).  The columns of the stream are the concatenated
// sequences of its pairs; a pair's first column carries a flag at which each
// lane resets its row state to the column-0 boundary, so consecutive pairs
// overlap in the pipeline and only the stream pays the LS-1 step fill/drain.
// The bottom row of lane l-1 (Hg, F*) and the residue stream reach lane l
// through DPP wave_shr:1; the first lane of each stream takes its inputs by
// readlane / writelane instead.  Passes over m > LS*R run one after the other
// for the whole workgroup; the boundary row between passes goes through
// global scratch per stream.
//
// Profile: int16 [alpha+1][LS lanes][8*W] (W = ceil(R/8); row alpha is the
// padding row) when every score and S + goe fit in 16 bits (P16), one or two
// 16-byte LDS reads per step (the streams of a wavefront read the same
// entries); otherwise int32 [32][LS*R] (LS = 64 only).
//
// End cell: when a lane leaves a pair it publishes its best cell as a 64-bit
// key (H << 32 | (0xffff - j) << 16 | (0xffff - i)) with atomicMax, so the
// pair's maximum over lanes and passes is max H, then min j, then min i,
// independent of the order of the atomics.
//
// Codes: W u32 words per (pass, step k, lane); word q holds rows 8q.. of the
// lane, row t at bit 4*(n_q - 1 - (t - 8q)) with n_q rows in word q.  They
// are tiled so that a lane's 8 consecutive steps share 32*W bytes: with
// G = ceil((C + LS - 1)/8) groups per pass,
//   codes[sbase + ((pass*G + k/8)*LS + l)*8W + (k%8)*W + q].
// Each lane stages its words in LDS and stores 32*W bytes every 8 steps
// (coalesced); the walk then finds a diagonal run of up to 8 steps in one
// line.  For a pair starting at stream column c0, cell (i, j) is at step
// k = c0 + j - 1 + lane(i).
// ---------------------------------------------------------------------------
constexpr uint8_t kFirstCol = 0x80;

struct StreamArgs {
    const int8_t *mat;        // alpha x alpha
    int alpha;
    const uint8_t *center;    // m residues
    int m, passes;
    const uint8_t *sres;      // staged stream residues (bit 7: first column of a pair)
    const int64_t *sbeg;      // per stream: first column in sres (nstreams + 1 entries)
    int nstreams;
    int ge, goe;
    unsigned long long *keys; // per pair-slot end-cell keys (zeroed); score-only: H << 32
    const int32_t *sslot0;    // per stream: slot of its first pair
    uint32_t *codes;          // null: no traceback
    const int64_t *scbase;    // per stream: code word base
    int2 *bound;              // per stream boundary rows: (passes-1) * C entries
    const int64_t *sbbase;    // per stream
};

__device__ __forceinline__ unsigned long long cell_key(const BestCell &b, bool endc) {
    unsigned long long k = (unsigned long long)b.h << 32;
    if (endc) k |= ((unsigned long long)(0xffff - b.j) << 16) | (unsigned long long)(0xffff - b.i);
    return k;
}

// The step loop is unrolled by 8: a lane's 8 steps of code words are staged
// in LDS and go out as one 32*W-byte tile, and the loop runs over whole tiles
// (steps rounded up to a multiple of 8, to the longest stream of the
// wavefront; the extra steps see padding columns).  A lane keeps, for the
// current pair, its max H, the step of the first column that reached it and
// that column's key (smallest row), which is the max-H / min-j / min-i rule
// restricted to its rows.  A stream's last pair is published after the loop:
// padding columns after a stream never raise H above the stream's maximum (E
// and F only decay there).  The loop is compiled twice: with and without
// boundary rows between passes.
template <int R, int LS, bool TB, bool ENDC, bool P16>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(R > 6 ? 4 : 6)))
sw_stream_kernel(StreamArgs a) {
    static_assert(LS == 64 || LS == 32 || LS == 16, "lanes per stream");
    static_assert(P16 || LS == 64, "the int32 profile serves 64-lane streams only");
    constexpr int W = (R + 7) / 8;           // code words per step
    constexpr int NS = 64 / LS;              // streams per wavefront
    constexpr int SPAN = LS * R;             // rows per pass
    extern __shared__ int prof[];   // profile, then code staging [8 waves][8 steps][W][64 lanes]
    const int nprow = P16 ? a.alpha + 1 : kAlphaMax;
    const int prof_words = P16 ? nprow * LS * 4 * W : kAlphaMax * SPAN;
    uint32_t *stage = reinterpret_cast<uint32_t *>(prof + prof_words) + (threadIdx.x >> 6) * 512 * W +
                      (threadIdx.x & 63);   // word (u, q) at stage[64 * (u*W + q)]: no bank conflicts
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int ll = lane & (LS - 1);          // lane within its stream
    const int nthreads = blockDim.x;
    const int ge = a.ge, goe = a.goe;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (nthreads >> 6) + (tid >> 6));
    const int sid = wave * NS + lane / LS;   // this lane's stream
    const bool active = sid < a.nstreams;
    int64_t b0 = 0;
    int C = 0, slot0 = 0;
    if (active) {
        b0 = a.sbeg[sid];
        C = (int)(a.sbeg[sid + 1] - b0);
        slot0 = a.sslot0[sid];
    }
    // the wavefront runs to its longest stream
    int Cmax = C;
#pragma unroll
    for (int s = 0; s < NS; ++s) Cmax = max(Cmax, __builtin_amdgcn_readlane(C, s * LS));
    Cmax = __builtin_amdgcn_readfirstlane(Cmax);
    const uint8_t *sr = a.sres + b0;
    const int steps_s = C + LS - 1;                  // this stream's steps
    const int steps8 = (Cmax + LS - 1 + 7) & ~7;     // the wavefront's steps (whole tiles)
    const int G = (steps_s + 7) >> 3;                // this stream's tiles per pass
    for (int pass = 0; pass < a.passes; ++pass) {
        const int row0 = pass * SPAN;
        __syncthreads();
        if (P16) {
            int16_t *p16 = reinterpret_cast<int16_t *>(prof);
            constexpr int PER = 8 * W;               // halves per (residue, lane)
            for (int x = tid; x < nprow * LS * PER; x += nthreads) {
                const int r = x / (LS * PER), l = (x / PER) & (LS - 1), tt = x % PER;
                const int i = row0 + l * R + tt;
                int v = -32768;
                if (r < a.alpha && tt < R && i < a.m) v = (int)a.mat[(a.center[i] & 31) * a.alpha + r] + goe;
                p16[x] = (int16_t)v;
            }
        } else {
            for (int x = tid; x < kAlphaMax * SPAN; x += nthreads) {
                const int r = x / SPAN, i = row0 + (x - r * SPAN);
                int v = kNegProf;
                if (r < a.alpha && i < a.m) v = (int)a.mat[(a.center[i] & 31) * a.alpha + r] + goe;
                prof[x] = v;
            }
        }
        __syncthreads();
        if (wave * NS >= a.nstreams) continue;   // no stream of this wavefront is active
        const int myrow = row0 + ll * R;
        const int *pbase = prof + ll * R;
        const int2 *bin = (pass > 0 && active) ? a.bound + a.sbbase[sid] + (int64_t)(pass - 1) * C : nullptr;
        int2 *bout = (pass + 1 < a.passes && active) ? a.bound + a.sbbase[sid] + (int64_t)pass * C : nullptr;
        uint32_t *cw = (TB && active) ? a.codes + a.scbase[sid] + (int64_t)pass * G * LS * 8 * W + ll * 8 * W : nullptr;
        // staged residue codes are already clamped to the profile rows; the
        // first-column flag moves to bit 31 (so the profile index shifts it out)
        const int padc = P16 ? a.alpha : kPad;
        auto conv = [&](int b) __attribute__((always_inline)) { return (b & 0x7f) | ((b & 0x80) << 24); };
        // the loop, specialised on whether boundary rows come in or go out
        auto run = [&](auto hb_tag) __attribute__((always_inline)) {
            constexpr bool HB = decltype(hb_tag)::value;
            int hg[R], e[R];
#pragma unroll
            for (int t = 0; t < R; ++t) { hg[t] = -goe; e[t] = 0; }
            int botg = -goe, botf = 0;   // this lane's bottom row values (last step)
            int diag0 = -goe;            // Hg(myrow-1, j-1) for row 0
            int rcur = padc;             // staged residue of this lane's column
            int rbuf = padc;             // staged residues of columns kb .. kb+LS-1 of the stream
            int2 bbuf = make_int2(-goe, 0);
            int pl = -1;                 // this lane's pair index within the stream
            // lane's best cell in the current pair: first column with its max H
            int bh = 0, bcol = 0, bk = 0, kflag = 0;
            auto publish = [&]() __attribute__((always_inline)) {
                if (active && pl >= 0 && bh > 0) {
                    BestCell b{bh, bk - kflag + 1, myrow + (31 - (bcol & 31))};
                    atomicMax(a.keys + slot0 + pl, cell_key(b, ENDC));
                }
            };
            for (int k8 = 0; k8 < steps8; k8 += 8) {
                if ((k8 & (LS - 1)) == 0) {
                    const int kk = k8 + ll;
                    rbuf = (kk < C) ? conv((int)sr[kk]) : padc;
                    if (HB && bin) bbuf = (kk < C) ? bin[kk] : make_int2(-goe, 0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = k8 + u;
                    const int rl = (k8 & (LS - 1)) + u;   // wave-uniform
                    rcur = __builtin_amdgcn_update_dpp(__builtin_amdgcn_readlane(rbuf, rl), rcur, 0x138, 0xf, 0xf,
                                                       false);
#pragma unroll
                    for (int s = 1; s < NS; ++s) {   // the first lane of stream s takes its column directly
                        const int rs = __builtin_amdgcn_readlane(rbuf, s * LS + rl);
                        rcur = lane == s * LS ? rs : rcur;
                    }
                    int upg, upf;
                    if (HB) {
                        int tg = -goe, tf = 0;
                        if (bin) {
                            tg = __builtin_amdgcn_readlane(bbuf.x, rl);
                            tf = __builtin_amdgcn_readlane(bbuf.y, rl);
                        }
                        upg = __builtin_amdgcn_update_dpp(tg, botg, 0x138, 0xf, 0xf, false);
                        upf = __builtin_amdgcn_update_dpp(tf, botf, 0x138, 0xf, 0xf, false);
#pragma unroll
                        for (int s = 1; s < NS; ++s) {
                            int sg = -goe, sf = 0;
                            if (bin) {
                                sg = __builtin_amdgcn_readlane(bbuf.x, s * LS + rl);
                                sf = __builtin_amdgcn_readlane(bbuf.y, s * LS + rl);
                            }
                            upg = lane == s * LS ? sg : upg;
                            upf = lane == s * LS ? sf : upf;
                        }
                    } else {
                        upg = __builtin_amdgcn_update_dpp(-goe, botg, 0x138, 0xf, 0xf, false);
                        upf = __builtin_amdgcn_mov_dpp(botf, 0x138, 0xf, 0xf, true);   // lane 0: 0
#pragma unroll
                        for (int s = 1; s < NS; ++s) {
                            upg = lane == s * LS ? -goe : upg;
                            upf = lane == s * LS ? 0 : upf;
                        }
                    }
                    if (rcur < 0) {
                        // leave the previous pair, enter the next one at its column 1
                        publish();
                        ++pl;
                        bh = 0;
                        bcol = 0;
                        bk = k;
                        kflag = k;
#pragma unroll
                        for (int t = 0; t < R; ++t) { hg[t] = -goe; e[t] = 0; }
                        diag0 = -goe;
                    }
                    int diag = diag0;
                    diag0 = upg;
                    int p[R];
                    if (P16) {
                        constexpr int LG = LS == 64 ? 6 : (LS == 32 ? 5 : 4);
                        const uint4 *pq = reinterpret_cast<const uint4 *>(prof) + (((uint32_t)rcur << LG) + ll) * W;
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            const uint4 q = pq[w];
                            const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                            for (int t = 8 * w; t < R && t < 8 * w + 8; ++t) {
                                const int h = t - 8 * w;
                                p[t] = (h & 1) ? ((int)qw[h >> 1] >> 16) : (int)(int16_t)(qw[h >> 1] & 0xffffu);
                            }
                        }
                    } else {
                        const int *prow = pbase + (rcur & 31) * SPAN;
#pragma unroll
                        for (int t = 0; t < R; ++t) p[t] = prow[t];
                    }
                    uint32_t word[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) word[w] = 0;
                    int colkey = 0, hm = 0;
#pragma unroll
                    for (int t = 0; t < R; t += 2) {
                        const int h0 = sw_cell<TB>(hg[t], e[t], diag, upg, upf, p[t], ge, goe, word[t >> 3]);
                        if (t + 1 < R) {
                            const int h1 = sw_cell<TB>(hg[t + 1], e[t + 1], diag, upg, upf, p[t + 1], ge, goe,
                                                       word[(t + 1) >> 3]);
                            if (ENDC) colkey = vmax3(colkey, (h0 << 5) | (31 - t), (h1 << 5) | (30 - t));
                            else hm = vmax3(hm, h0, h1);
                        } else {
                            if (ENDC) colkey = max(colkey, (h0 << 5) | (31 - t));
                            else hm = max(hm, h0);
                        }
                    }
                    botg = upg;
                    botf = upf;
                    if (TB) {
#pragma unroll
                        for (int w = 0; w < W; ++w) stage[64 * (u * W + w)] = word[w];
                    }
                    if (HB && bout) {
                        const int K = k - ll;   // stream column of this lane
                        if (ll == LS - 1 && K >= 0 && K < C) bout[K] = make_int2(botg, botf);
                    }
                    if (ENDC) {
                        const int ch = colkey >> 5;
                        const bool up = ch > bh;
                        bcol = up ? colkey : bcol;
                        bk = up ? k : bk;
                        bh = max(bh, ch);
                    } else {
                        bh = max(bh, hm);
                    }
                }
                if (TB && cw && k8 < steps_s) {
                    uint4 *dst = reinterpret_cast<uint4 *>(cw + (int64_t)(k8 >> 3) * LS * 8 * W);
#pragma unroll
                    for (int v = 0; v < 2 * W; ++v)
                        dst[v] = make_uint4(stage[64 * (4 * v)], stage[64 * (4 * v + 1)], stage[64 * (4 * v + 2)],
                                            stage[64 * (4 * v + 3)]);
                }
            }
            publish();   // the stream's last pair
        };
        if (pass > 0 || pass + 1 < a.passes) run(std::true_type{});
        else run(std::false_type{});
    }
}

// keys -> score and end cell (i1, j1), 1-based; slot q belongs to pair pid[q].
__global__ void decode_keys_kernel(const unsigned long long *keys, const int32_t *slot_pid, int nslots,
                                   int32_t *score, int32_t *endcell) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nslots) return;
    const unsigned long long k = keys[q];
    const int pid = slot_pid[q];
    const int h = (int)(k >> 32);
    score[pid] = h;
    if (endcell) {
        endcell[2 * pid] = h > 0 ? (0xffff - (int)(k & 0xffff)) + 1 : 0;
        endcell[2 * pid + 1] = h > 0 ? 0xffff - (int)((k >> 16) & 0xffff) : 0;
    }
}

// Stage the residues of every stream: sres[sbase + c0(q) + x] = s_q[x], with
// kFirstCol on x = 0.  One workgroup per pair slot.
__global__ void stage_stream_kernel(const uint8_t *res, const int64_t *off, const int32_t *slot_pid,
                                    const int64_t *slot_col, int nslots, int clamp, uint8_t *sres) {
    const int q = blockIdx.x;
    if (q >= nslots) return;
    const int pid = slot_pid[q];
    const int64_t so = off[pid];
    const int n = (int)(off[pid + 1] - so);
    uint8_t *dst = sres + slot_col[q];
    for (int x = threadIdx.x; x < n; x += blockDim.x)
        dst[x] = (uint8_t)(min((int)(res[so + x] & 31), clamp) | (x == 0 ? kFirstCol : 0));
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
// Codes: u64 (two u32 words: rows 0-7, 8-15; row t nibble at 4*(7 - t%8))
// per (strip s, column j, lane), tiled so that a lane's 4 consecutive columns
// share 32 bytes: with G = ceil(nmax/4),
//   codes[gbase + ((s*G + (j-1)/4)*64 + lane)*8 + ((j-1)%4)*2 + half].
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
    __shared__ uint32_t stage_all[64 * 8];
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
        const int G = (nmax + 3) >> 2;
        uint32_t *cw = TB ? a.codes + a.gcode_base[g] + lane * 8 : nullptr;
        uint32_t *stage = stage_all + lane * 8;
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
                    const int jj = (j - 1) & 3;
                    stage[2 * jj] = w0;
                    stage[2 * jj + 1] = w1;
                    if (jj == 3 || j == nmax) {
                        const uint4 lo = *reinterpret_cast<const uint4 *>(stage);
                        const uint4 hi = *reinterpret_cast<const uint4 *>(stage + 4);
                        uint4 *dst = reinterpret_cast<uint4 *>(cw + ((int64_t)st * G + ((j - 1) >> 2)) * 512);
                        dst[0] = lo;
                        dst[1] = hi;
                    }
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
    const int64_t *cbase;     // word base of the stream / group
    const int32_t *ccol;      // wavefront: first stream column of the pair; strip: lane in group
    const int32_t *cstride;   // wavefront: steps per pass (C+63); strip: nmax of the group
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
template <bool STRIP, bool CEN_LDS>
__global__ void __launch_bounds__(64)
walk_kernel(WalkArgs a) {
    __shared__ uint32_t cache[4][16][64];
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
    int ccol, stride;
    if (STRIP) {
        base = a.cbase[pid];
        ccol = a.ccol[pid];
        stride = a.cstride[pid];
    } else {   // stream of slot w: the last s with slot0[s] <= w
        int lo = 0, hi = a.nstreams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.slot0[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        base = a.scb[lo];
        ccol = (int)(a.slot_col[w] - a.sbeg[lo]);
        stride = (int)(a.sbeg[lo + 1] - a.sbeg[lo]) + (1 << a.lg_ls) - 1;
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
                wi = ((ccol + j - 1 + (blk & LSm)) & 7) * W + (t >> 3);
                sh = t < 8 ? 4 * (n0 - 1 - t) : 4 * (R - 1 - t);
            }
            const uint32_t nib = (cache[sl][wi & 15][lane] >> (sh & 31)) & 15u;
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
        uint4 cq[4][4];
#pragma unroll
        for (int h = 0; h < 4; ++h) cq[0][h] = cq[1][h] = cq[2][h] = cq[3][h] = make_uint4(0, 0, 0, 0);
        {
            const uint4 *q0 = reinterpret_cast<const uint4 *>(a.codes + ad0);
            const uint4 *q1 = reinterpret_cast<const uint4 *>(a.codes + ad1);
            const uint4 *q2 = reinterpret_cast<const uint4 *>(a.codes + ad2);
            const uint4 *q3 = reinterpret_cast<const uint4 *>(a.codes + ad3);
            cq[0][0] = q0[0]; cq[0][1] = q0[1];
            cq[1][0] = q1[0]; cq[1][1] = q1[1];
            cq[2][0] = q2[0]; cq[2][1] = q2[1];
            cq[3][0] = q3[0]; cq[3][1] = q3[1];
            if (W == 2) {
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
            for (int h = 0; h < 4; ++h) {
                if (h < 2 || W == 2) {
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
