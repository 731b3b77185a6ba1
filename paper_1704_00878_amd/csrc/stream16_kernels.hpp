// Packed 16-bit wavefront kernel for gfx950: the traceback forward pass of
// the wavefront kernel (sw_kernels.hpp) with two streams per lane group.
// Lane group g of a wavefront runs stream 2q (A) in the low and stream 2q+1
// (B) in the high half of every register, q = wave * NS + g, with v_pk_* 16-bit
// ops.  The lane group's columns are the longer stream's; the other half runs
// padding columns after its last pair.
//
// Recurrence as in the 32-bit kernels (E* and F* clamped at 0), on values
// held plus a bias so that each of E*, F* and H is one v_pk_maximum3_f16 on
// their bit patterns: 8 packed ops per two cells.  The host uses this kernel
// only when every H stays below 15000 (max S * min(m, longest sequence) <
// 15000, go + ge <= 256), so no value or difference wraps and a padding
// profile entry is never a source.
//
// The four flags of a cell are the signs of four packed differences.
// v_perm_b32 with byte selectors 8..11 turns the signs of two packed
// differences into four 0x00/0xff bytes, one per flag and half, so two perms
// give all eight flags of a row pair, and two v_bfi_b32 with constant masks
// drop them into their bits of a word that holds 4 rows of both pairs:
// WQ = ceil(R/4) words per step, word q holding rows 4q.. of the lane.  Row t
// (k = t mod 4) of half h: byte h holds notd at bit 2k and note at bit 2k + 1,
// byte 2 + h holds eext at bit 2k and fext at bit 2k + 1.  Tiles and the
// step-to-column rule are the wavefront kernel's with WQ words per step; each
// lane stages 4 steps in LDS and stores them as half a tile.  With E* and F*
// clamped as there, every flag equals the 32-bit kernel's.
//
// End cells stay packed: per step one v_pk_maximum3_f16 per two rows gives
// the step maximum of each half, its sign against the running best gives a
// 16-bit mask per half, and where it is set the step and the lane's rows are
// copied (v_bfi_b32).  The first step that reaches the best H is the smallest
// column, and at publication the smallest row of that step holding the best H
// completes the key (max H, then min j, then min i per lane).  This needs R
// more registers; above R = 11 both halves unpack H into 32-bit keys
// (H << 5 | 31 - t) per row instead, as the 32-bit kernel does.
#pragma once
#include "sw_kernels.hpp"
#include "pk16.hpp"

namespace hk {

template <int R, int LS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
sw_stream16_kernel(StreamArgs a) {
    static_assert(LS == 32 || LS == 16, "lanes per stream");
    static_assert(R >= 2 && R <= 16, "rows per lane");
    // packed end cells need R more registers: up to R = 11 they fit the
    // 128 of four waves per SIMD
    constexpr bool SNAP = R <= 11;
    constexpr int W = (R + 7) / 8;           // profile uint4 per (residue, lane)
    constexpr int WQ = (R + 3) / 4;          // code words per step (both halves)
    constexpr int NS = 64 / LS;              // lane groups per wavefront
    constexpr int SPAN = LS * R;             // rows per pass
    constexpr int LG = LS == 32 ? 5 : 4;
    extern __shared__ int prof[];   // profile, then code staging [8 waves][4 steps][WQ][64 lanes]
    const int nprow = a.alpha + 1;
    const int prof_words = nprow * LS * 4 * W;
    uint32_t *stage = reinterpret_cast<uint32_t *>(prof + prof_words) + (threadIdx.x >> 6) * 256 * WQ +
                      (threadIdx.x & 63);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int ll = lane & (LS - 1);
    const int nthreads = blockDim.x;
    const int goe = a.goe;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (nthreads >> 6) + (tid >> 6));
    const int q = wave * NS + lane / LS;     // lane group's stream pair
    const int sA = 2 * q, sB = 2 * q + 1;
    const bool actA = sA < a.nstreams, actB = sB < a.nstreams;
    int64_t bA = 0, bB = 0;
    int CA = 0, CB = 0, slotA = 0, slotB = 0;
    if (actA) {
        bA = a.sbeg[sA];
        CA = (int)(a.sbeg[sA + 1] - bA);
        slotA = a.sslot0[sA];
    }
    if (actB) {
        bB = a.sbeg[sB];
        CB = (int)(a.sbeg[sB + 1] - bB);
        slotB = a.sslot0[sB];
    }
    const int C = max(CA, CB);
    int Cmax = C;
#pragma unroll
    for (int s = 0; s < NS; ++s) Cmax = max(Cmax, __builtin_amdgcn_readlane(C, s * LS));
    Cmax = __builtin_amdgcn_readfirstlane(Cmax);
    const uint8_t *srA = a.sres + bA, *srB = a.sres + bB;
    const int steps_s = C + LS - 1;
    const int steps8 = (Cmax + LS - 1 + 7) & ~7;
    const int G = (steps_s + 7) >> 3;
    const pk16 init2 = pk16{(short)(kBias16 - goe), (short)(kBias16 - goe)};   // -go - ge, biased
    const uint32_t init2u = as_u(init2);
    const pk16 ge2 = pk16{(short)a.ge, (short)a.ge};
    const pk16 goe2 = pk16{(short)goe, (short)goe};
    const pk16 zero2 = pk16{0, 0};
    const pk16 bias2 = pk16{(short)kBias16, (short)kBias16};   // 0, biased
    const int padc = a.alpha;
    const int padrc = padc | (padc << 16);
    for (int pass = 0; pass < a.passes; ++pass) {
        const int row0 = pass * SPAN;
        __syncthreads();
        {
            int16_t *p16 = reinterpret_cast<int16_t *>(prof);
            constexpr int PER = 8 * W;
            for (int x = tid; x < nprow * LS * PER; x += nthreads) {
                const int r = x / (LS * PER), l = (x / PER) & (LS - 1), tt = x % PER;
                const int i = row0 + l * R + tt;
                int v = kPadProf16;
                if (r < a.alpha && tt < R && i < a.m) v = (int)a.mat[(a.center[i] & 31) * a.alpha + r] + goe;
                p16[x] = (int16_t)v;
            }
        }
        __syncthreads();
        if (2 * wave * NS >= a.nstreams) continue;   // no stream of this wavefront is active
        const int myrow = row0 + ll * R;
        const int2 *bin = (pass > 0 && actA) ? a.bound + a.sbbase[sA] + (int64_t)(pass - 1) * C : nullptr;
        int2 *bout = (pass + 1 < a.passes && actA) ? a.bound + a.sbbase[sA] + (int64_t)pass * C : nullptr;
        uint32_t *cw = actA ? a.codes + a.scbase[sA] + (int64_t)pass * G * LS * 8 * WQ + ll * 8 * WQ : nullptr;
        auto run = [&](auto hb_tag) __attribute__((always_inline)) {
            constexpr bool HB = decltype(hb_tag)::value;
            pk16 hg[R], e[R];
#pragma unroll
            for (int t = 0; t < R; ++t) { hg[t] = init2; e[t] = init2; }
            uint32_t botg = init2u, botf = init2u;
            uint32_t diag0 = init2u;
            int rcur = padrc, rbuf = padrc;
            int2 bbuf = make_int2((int)init2u, (int)init2u);
            int plA = -1, plB = -1;
            // running end cell of the current pair, per half.  SNAP: the best
            // H, the step (mod 2^16) that first reached it and the lane's rows
            // (as H - go - ge) at that step, the row resolved at publication.
            // Otherwise 32-bit keys (H << 5 | 31 - t) per step.
            pk16 bh = zero2;
            uint32_t bk = 0;
            pk16 hs[SNAP ? R : 1];
#pragma unroll
            for (int t = 0; t < (SNAP ? R : 1); ++t) hs[t] = init2;
            int bhA = 0, bcolA = 0, bkA = 0;
            int bhB = 0, bcolB = 0, bkB = 0;
            int kfA = 0, kfB = 0;
            auto publish = [&](int h, int kf, int sh, int slot, int pl) __attribute__((always_inline)) {
                int t0 = 0;
#pragma unroll
                for (int t = R - 1; t >= 0; --t)
                    if ((int)(short)(as_u(hs[SNAP ? t : 0]) >> sh) == h - goe) t0 = t;
                // j - 1 < 2^16 for every cell of a pair, so the low 16 bits of
                // the step difference are the column
                BestCell b{h - kBias16, (int)(((bk >> sh) - (uint32_t)kf) & 0xffffu) + 1, myrow + t0};
                atomicMax(a.keys + slot + pl, cell_key(b, true));
            };
            auto publishA = [&]() __attribute__((always_inline)) {
                if constexpr (SNAP) {
                    const int h = (int)(as_u(bh) & 0xffffu);
                    if (actA && plA >= 0 && h > kBias16) publish(h, kfA, 0, slotA, plA);
                } else if (actA && plA >= 0 && bhA > kBias16) {
                    BestCell b{bhA - kBias16, bkA - kfA + 1, myrow + (31 - (bcolA & 31))};
                    atomicMax(a.keys + slotA + plA, cell_key(b, true));
                }
            };
            auto publishB = [&]() __attribute__((always_inline)) {
                if constexpr (SNAP) {
                    const int h = (int)(as_u(bh) >> 16);
                    if (actB && plB >= 0 && h > kBias16) publish(h, kfB, 16, slotB, plB);
                } else if (actB && plB >= 0 && bhB > kBias16) {
                    BestCell b{bhB - kBias16, bkB - kfB + 1, myrow + (31 - (bcolB & 31))};
                    atomicMax(a.keys + slotB + plB, cell_key(b, true));
                }
            };
            for (int k8 = 0; k8 < steps8; k8 += 8) {
                if ((k8 & (LS - 1)) == 0) {
                    const int kk = k8 + ll;
                    const int ra = kk < CA ? (int)srA[kk] : padc;
                    const int rb = kk < CB ? (int)srB[kk] : padc;
                    rbuf = ra | (rb << 16);
                    if (HB && bin) bbuf = kk < C ? bin[kk] : make_int2((int)init2u, (int)init2u);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = k8 + u;
                    const int rl = (k8 & (LS - 1)) + u;   // wave-uniform
                    rcur = __builtin_amdgcn_update_dpp(__builtin_amdgcn_readlane(rbuf, rl), rcur, 0x138, 0xf, 0xf,
                                                       false);
#pragma unroll
                    for (int s = 1; s < NS; ++s) {
                        const int rs = __builtin_amdgcn_readlane(rbuf, s * LS + rl);
                        rcur = lane == s * LS ? rs : rcur;
                    }
                    uint32_t upgu, upfu;
                    if (HB) {
                        int tg = (int)init2u, tf = (int)init2u;
                        if (bin) {
                            tg = __builtin_amdgcn_readlane(bbuf.x, rl);
                            tf = __builtin_amdgcn_readlane(bbuf.y, rl);
                        }
                        upgu = (uint32_t)__builtin_amdgcn_update_dpp(tg, (int)botg, 0x138, 0xf, 0xf, false);
                        upfu = (uint32_t)__builtin_amdgcn_update_dpp(tf, (int)botf, 0x138, 0xf, 0xf, false);
#pragma unroll
                        for (int s = 1; s < NS; ++s) {
                            int sg = (int)init2u, sf = (int)init2u;
                            if (bin) {
                                sg = __builtin_amdgcn_readlane(bbuf.x, s * LS + rl);
                                sf = __builtin_amdgcn_readlane(bbuf.y, s * LS + rl);
                            }
                            upgu = lane == s * LS ? (uint32_t)sg : upgu;
                            upfu = lane == s * LS ? (uint32_t)sf : upfu;
                        }
                    } else {
                        upgu = (uint32_t)__builtin_amdgcn_update_dpp((int)init2u, (int)botg, 0x138, 0xf, 0xf, false);
                        upfu = (uint32_t)__builtin_amdgcn_update_dpp((int)init2u, (int)botf, 0x138, 0xf, 0xf, false);
#pragma unroll
                        for (int s = 1; s < NS; ++s) {
                            upgu = lane == s * LS ? init2u : upgu;
                            upfu = lane == s * LS ? init2u : upfu;
                        }
                    }
                    if (rcur & 0x00800080) {
                        // a pair starts in one half or both: publish the pair left
                        // behind and reset that half to the column-0 boundary
                        const bool fA = (rcur & 0x80) != 0, fB = (rcur & 0x800000) != 0;
                        if (fA) {
                            publishA();
                            ++plA;
                            kfA = k;
                            bhA = 0;
                            bcolA = 0;
                            bkA = k;
                        }
                        if (fB) {
                            publishB();
                            ++plB;
                            kfB = k;
                            bhB = 0;
                            bcolB = 0;
                            bkB = k;
                        }
                        const uint32_t msk = (fA ? 0xffffu : 0u) | (fB ? 0xffff0000u : 0u);
                        bh = as_pk(as_u(bh) & ~msk);
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            hg[t] = as_pk((init2u & msk) | (as_u(hg[t]) & ~msk));
                            e[t] = as_pk((init2u & msk) | (as_u(e[t]) & ~msk));
                        }
                        diag0 = (init2u & msk) | (diag0 & ~msk);
                    }
                    pk16 upg = as_pk(upgu), upf = as_pk(upfu);
                    pk16 diag = as_pk(diag0);
                    diag0 = upgu;
                    const int ra = rcur & 0x7f, rb = (rcur >> 16) & 0x7f;
                    const uint4 *pa = reinterpret_cast<const uint4 *>(prof) + (((uint32_t)ra << LG) + ll) * W;
                    const uint4 *pb = reinterpret_cast<const uint4 *>(prof) + (((uint32_t)rb << LG) + ll) * W;
                    uint32_t wa[4 * W], wb[4 * W];
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const uint4 x = pa[w], y = pb[w];
                        wa[4 * w] = x.x; wa[4 * w + 1] = x.y; wa[4 * w + 2] = x.z; wa[4 * w + 3] = x.w;
                        wb[4 * w] = y.x; wb[4 * w + 1] = y.y; wb[4 * w + 2] = y.z; wb[4 * w + 3] = y.w;
                    }
                    uint32_t word[WQ];
#pragma unroll
                    for (int w = 0; w < WQ; ++w) word[w] = 0;
                    pk16 sm = bias2;   // step maximum over the lane's rows, per half
                    pk16 hprev = bias2;
                    int ckA = 0, ckB = 0, kpA = 0, kpB = 0;
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        const pk16 p = as_pk(__builtin_amdgcn_perm(wb[t >> 1], wa[t >> 1],
                                                                   (t & 1) ? 0x07060302u : 0x05040100u));
                        const pk16 eext = e[t] - ge2;
                        const pk16 en = max3h(eext, hg[t], bias2);   // E* = max(E, 0)
                        const pk16 fext = upf - ge2;
                        const pk16 fn = max3h(fext, upg, bias2);     // F* = max(F, 0)
                        const pk16 hd = diag + p;
                        const pk16 h = max3h(hd, en, fn);
                        // bytes (notd A, notd B, eext A, eext B) and (note A, note B, fext A, fext B)
                        const uint32_t f0 = __builtin_amdgcn_perm(as_u(hg[t] - eext), as_u(hd - h), 0x0b0a0908u);
                        const uint32_t f1 = __builtin_amdgcn_perm(as_u(upg - fext), as_u(en - h), 0x0b0a0908u);
                        const uint32_t m0 = 0x01010101u << (2 * (t & 3)), m1 = m0 << 1;
                        uint32_t wd = word[t >> 2];
                        wd = bfi_s(m0, f0, wd);
                        wd = bfi_s(m1, f1, wd);
                        word[t >> 2] = wd;
                        if constexpr (SNAP) {
                            if (t & 1) sm = max3h(sm, hprev, h);
                            else if (t == R - 1) sm = pmax(sm, h);
                            else hprev = h;
                        } else {
                            const uint32_t hu = as_u(h);
                            const int kA = (int)((hu & 0xffffu) << 5) | (31 - t);
                            const int kB = (int)((hu >> 16) << 5) | (31 - t);
                            if (t & 1) {
                                ckA = vmax3(ckA, kpA, kA);
                                ckB = vmax3(ckB, kpB, kB);
                            } else if (t == R - 1) {
                                ckA = max(ckA, kA);
                                ckB = max(ckB, kB);
                            } else {
                                kpA = kA;
                                kpB = kB;
                            }
                        }
                        diag = hg[t];
                        hg[t] = h - goe2;
                        e[t] = en;
                        upg = hg[t];
                        upf = fn;
                    }
                    botg = as_u(upg);
                    botf = as_u(upf);
#pragma unroll
                    for (int w = 0; w < WQ; ++w) stage[64 * ((u & 3) * WQ + w)] = word[w];
                    if ((u & 3) == 3 && cw && k8 < steps_s) {
                        // half a tile (4 steps, 16*WQ bytes of the lane's 32*WQ)
                        uint4 *dst = reinterpret_cast<uint4 *>(cw + (int64_t)(k8 >> 3) * LS * 8 * WQ) + (u >> 2) * WQ;
#pragma unroll
                        for (int v = 0; v < WQ; ++v)
                            dst[v] = make_uint4(stage[64 * (4 * v)], stage[64 * (4 * v + 1)], stage[64 * (4 * v + 2)],
                                                stage[64 * (4 * v + 3)]);
                    }
                    if (HB && bout) {
                        const int K = k - ll;
                        if (ll == LS - 1 && K >= 0 && K < C) bout[K] = make_int2((int)botg, (int)botf);
                    }
                    if constexpr (SNAP) {
                        // 0xffff in each half whose step maximum beats its best
                        const uint32_t imp = as_u((bh - sm) >> pk16{15, 15});
                        bh = pmax(bh, sm);
                        const uint32_t kw = (uint32_t)(k & 0xffff) * 0x10001u;
                        bk = bfi(imp, kw, bk);
#pragma unroll
                        for (int t = 0; t < R; ++t) hs[t] = as_pk(bfi(imp, as_u(hg[t]), as_u(hs[t])));
                    } else {
                        {
                            const int ch = ckA >> 5;
                            const bool up = ch > bhA;
                            bcolA = up ? ckA : bcolA;
                            bkA = up ? k : bkA;
                            bhA = max(bhA, ch);
                        }
                        {
                            const int ch = ckB >> 5;
                            const bool up = ch > bhB;
                            bcolB = up ? ckB : bcolB;
                            bkB = up ? k : bkB;
                            bhB = max(bhB, ch);
                        }
                    }
                }
            }
            publishA();
            publishB();
        };
        if (pass > 0 || pass + 1 < a.passes) run(std::true_type{});
        else run(std::false_type{});
    }
}

}  // namespace hk
