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

// DPP controls (gfx9 family): shifts within 16-lane rows, the whole-wave
// shift, and the broadcast of lane 15 of each row to the next row.
constexpr int kDppRowShl = 0x100;   // + n: lane l reads lane l + n of its row
constexpr int kDppRowShr1 = 0x111;  // lane l reads lane l - 1 of its row
constexpr int kDppRowBcast15 = 0x142;

// N (<= 4) LDS dwords of a profile entry at p (16-byte aligned for N >= 3,
// 8-byte aligned for N = 2)
template <int N>
__device__ __forceinline__ void lds_words(const uint32_t *p, uint32_t *d) {
    if constexpr (N >= 4) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        d[0] = x.x; d[1] = x.y; d[2] = x.z; d[3] = x.w;
    } else if constexpr (N == 3) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        d[0] = x.x; d[1] = x.y; d[2] = x.z;
    } else if constexpr (N == 2) {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        d[0] = x.x; d[1] = x.y;
    } else {
        d[0] = *p;
    }
}

// A stream's next column enters at its first lane and every other lane takes
// its left neighbour's: lane l of each stream gets x[l - 1], the first lane of
// each stream gets head (both wave-uniform patterns, three DPP moves at most).
template <int LS>
__device__ __forceinline__ int stream_shift(int x, int head) {
    if constexpr (LS == 16) {
        return __builtin_amdgcn_update_dpp(head, x, kDppRowShr1, 0xf, 0xf, false);
    } else {   // 32 lanes: rows 1 and 3 continue rows 0 and 2
        const int t = __builtin_amdgcn_update_dpp(head, x, kDppRowBcast15, 0xa, 0xf, false);
        return __builtin_amdgcn_update_dpp(t, x, kDppRowShr1, 0xf, 0xf, false);
    }
}

// lane l of each 16-lane row takes x[l + U] (the first lane of each stream
// takes the value of lane U of its stream)
template <int U>
__device__ __forceinline__ int row_take(int x) {
    if constexpr (U == 0) return x;
    else return __builtin_amdgcn_update_dpp(x, x, kDppRowShl + U, 0xf, 0xf, false);
}

template <int R, int LS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
sw_stream16_kernel(StreamArgs a) {
    static_assert(LS == 32 || LS == 16, "lanes per stream");
    static_assert(R >= 2 && R <= 16, "rows per lane");
    // packed end cells need R more registers: up to R = 11 they fit the
    // 128 of four waves per SIMD
    constexpr bool SNAP = R <= 11;
    constexpr int NW = (R + 1) / 2;          // profile dwords a step reads per stream
    // profile planes per residue: rows 0..7 (NA dwords per lane, lane stride
    // SA dwords), then rows 8..R-1 (NB dwords, stride SB); strides of 1, 2 or 4
    // dwords keep the lanes of one read on distinct banks
    constexpr int NA = NW < 4 ? NW : 4, NB = NW - NA;
    constexpr int SA = NA == 3 ? 4 : NA, SB = NB == 3 ? 4 : NB;
    constexpr int PRW = LS * (SA + SB);      // profile dwords per residue
    constexpr int WQ = (R + 3) / 4;          // code words per step (both halves)
    constexpr int NS = 64 / LS;              // lane groups per wavefront
    constexpr int SPAN = LS * R;             // rows per pass
    constexpr int LG = LS == 32 ? 5 : 4;
    // profile int16 per residue r (PRW dwords): plane A [lane][SA dwords] holds
    // lane l's rows 0..7 (two rows per dword), plane B [lane][SB dwords] its
    // rows 8..R-1, so the lanes of a read touch consecutive slots whatever
    // residue each one reads; then the code staging [8 waves][4 steps][WQ][64 lanes]
    extern __shared__ int prof[];
    const int nprow = a.alpha + 1;
    const int prof_words = nprow * PRW;
    uint32_t *stage = reinterpret_cast<uint32_t *>(prof + prof_words) + (threadIdx.x >> 6) * 256 * WQ +
                      (threadIdx.x & 63);
    const uint32_t *profA = reinterpret_cast<const uint32_t *>(prof) + (threadIdx.x & (LS - 1)) * SA;
    const uint32_t *profB = reinterpret_cast<const uint32_t *>(prof) + LS * SA + (threadIdx.x & (LS - 1)) * SB;
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
    // residues of the stream columns k0 + ll (A, B), for the first 8 lanes
    // of each stream (the heads of steps k0 .. k0 + 7); padding outside.
    // They are combined (A | B << 16) only where used, a block later, so the
    // loads are not waited for here.
    auto residues = [&](int k0) __attribute__((always_inline)) {
        const int kk = k0 + ll;
        int ra = padc, rb = padc;
        if (ll < 8) {
            if (kk < CA) ra = (int)srA[kk];
            if (kk < CB) rb = (int)srB[kk];
        }
        return make_int2(ra, rb);
    };
    auto pair_code = [](int2 r) __attribute__((always_inline)) { return r.x | (r.y << 16); };
    for (int pass = 0; pass < a.passes; ++pass) {
        const int row0 = pass * SPAN;
        __syncthreads();
        {
            int16_t *p16 = reinterpret_cast<int16_t *>(prof);
            for (int x = tid; x < nprow * PRW * 2; x += nthreads) {
                // int16 x of residue r: plane A (lane l, row tt < 8) or plane B
                const int r = x / (PRW * 2), y = x - r * (PRW * 2);
                int l, tt;
                if (y < LS * SA * 2) { l = y / (SA * 2); tt = y - l * (SA * 2); }
                else { const int z = y - LS * SA * 2; l = z / (SB * 2); tt = 8 + z - l * (SB * 2); }
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
            // boundary rows of the previous pass (Hg, F*) of the stream columns
            // k0 + ll for the first 8 lanes of each stream
            auto bounds = [&](int k0) __attribute__((always_inline)) {
                const int kk = k0 + ll;
                int2 v = make_int2((int)init2u, (int)init2u);
                if (HB && bin && ll < 8 && kk < C) v = bin[kk];
                return v;
            };
            pk16 hg[R], e[R];
#pragma unroll
            for (int t = 0; t < R; ++t) { hg[t] = init2; e[t] = init2; }
            uint32_t botg = init2u, botf = init2u;
            uint32_t diag0 = init2u;
            // residues and boundary values of the current 8-step block and of
            // the next one (loaded a block ahead, so no step waits on memory)
            int rbuf = pair_code(residues(0));
            int2 rnext = residues(8);
            int2 bbuf = bounds(0), bnext = bounds(8);
            // the residue pair of this lane's column at the current step, and
            // the profile words it selects (read one step ahead)
            int rcur = stream_shift<LS>(padrc, rbuf);
            uint32_t wa[NW], wb[NW];
            auto prof_read = [&](int rc, uint32_t (&da)[NW], uint32_t (&db)[NW]) __attribute__((always_inline)) {
                const uint32_t ra = __builtin_amdgcn_ubfe((uint32_t)rc, 0, 7);
                const uint32_t rb = __builtin_amdgcn_ubfe((uint32_t)rc, 16, 7);
                lds_words<NA>(profA + ra * PRW, da);
                lds_words<NA>(profA + rb * PRW, db);
                if constexpr (NB > 0) {
                    lds_words<NB>(profB + ra * PRW, da + NA);
                    lds_words<NB>(profB + rb * PRW, db + NA);
                }
            };
            prof_read(rcur, wa, wb);
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
            auto step = [&](auto u_tag, int k8) __attribute__((always_inline)) {
                constexpr int u = decltype(u_tag)::value;
                const int k = k8 + u;
                // the next step's residues and profile words, issued first
                const int rnx = stream_shift<LS>(rcur, u < 7 ? row_take<(u + 1) & 7>(rbuf) : pair_code(rnext));
                uint32_t na[NW], nb[NW];
                prof_read(rnx, na, nb);
                uint32_t upgu, upfu;
                if (HB) {
                    upgu = (uint32_t)stream_shift<LS>((int)botg, row_take<u>(bbuf.x));
                    upfu = (uint32_t)stream_shift<LS>((int)botf, row_take<u>(bbuf.y));
                } else {
                    upgu = (uint32_t)stream_shift<LS>((int)botg, (int)init2u);
                    upfu = (uint32_t)stream_shift<LS>((int)botf, (int)init2u);
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
                rcur = rnx;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    wa[w] = na[w];
                    wb[w] = nb[w];
                }
            };
            for (int k8 = 0; k8 < steps8; k8 += 8) {
                step(std::integral_constant<int, 0>{}, k8);
                step(std::integral_constant<int, 1>{}, k8);
                step(std::integral_constant<int, 2>{}, k8);
                step(std::integral_constant<int, 3>{}, k8);
                step(std::integral_constant<int, 4>{}, k8);
                step(std::integral_constant<int, 5>{}, k8);
                step(std::integral_constant<int, 6>{}, k8);
                step(std::integral_constant<int, 7>{}, k8);
                rbuf = pair_code(rnext);
                bbuf = bnext;
                rnext = residues(k8 + 16);
                bnext = bounds(k8 + 16);
            }
            publishA();
            publishB();
        };
        if (pass > 0 || pass + 1 < a.passes) run(std::true_type{});
        else run(std::false_type{});
    }
}

}  // namespace hk
