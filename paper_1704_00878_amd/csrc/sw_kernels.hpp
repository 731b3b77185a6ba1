// Smith-Waterman recurrence, shared cell helpers and the wavefront (stream)
// forward kernel for gfx950.
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

}  // namespace hk
