// Strip kernel (one pair per lane) for gfx950: the score and traceback
// forward pass of many pairs against per-group centers.  Shares the
// recurrence, register form, traceback code and end-cell rule of the
// wavefront kernel (sw_kernels.hpp).
#pragma once
#include "sw_kernels.hpp"
#include "pk16.hpp"
#include "tiling.hpp"

namespace hk {

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
constexpr int kB = 4;        // columns per prefetch block (the 4 columns of a code chunk)
constexpr int kFMask = (1 << 27) - 1;  // F* bits of a strip boundary cell (residue code above)

struct InterArgs {
    const int8_t *mat;
    int alpha;
    const uint8_t *center;    // batch center (mode 0)
    int m;
    const uint8_t *res;
    const int64_t *off;
    int mode;                 // 0 batch, 1 all pairs (a < b), 2 anchored groups
    const int32_t *order;     // mode 0: 64 * ngroups pair ids (-1 = empty lane); NULL: pair 64g + lane
    const int32_t *gnmax;     // mode 0: per group longest sequence (code layout); NULL: from the lanes
    const int32_t *gcen;      // mode 2: center seq id per group
    const int32_t *gb0;       // mode 2: first partner position in perm per group
    const int32_t *perm;      // modes 1/2: sequence ids (mode 1: sorted by length)
    int nseq;
    const int32_t *gslot;     // mode 2: sums slot of the group's center
    int64_t *sums;            // modes 1/2: integer score sums (atomic adds)
    int64_t ngroups;          // groups of this launch
    int64_t gfirst, gtotal;   // mode 1: this launch runs groups gfirst .. gfirst + ngroups - 1 of the
                              // gtotal = tri_groups(nseq, partners per group), largest first
    int ge, goe;
    unsigned long long *counter;   // next group (zeroed before the launch)
    int32_t *score;           // mode 0: per pair id; mode 2: per lane slot (optional)
    int32_t *endcell;         // mode 0: (i1, j1) per pair id (optional)
    int4 *cells4;             // mode 0 score-only: (0, 0, i1, j1) per pair id (optional)
    uint32_t *codes;
    const int64_t *gcode_base;// per group (u32 words)
    int2 *bound;              // per workgroup slot: bstride int2
    int64_t bstride;          // >= 64 * (max nmax rounded up to kB)
};

// a wave-uniform 64-bit value (read from LDS by every lane) in SGPRs
__device__ __forceinline__ int64_t uniform64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

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
    __shared__ unsigned long long s_next;
    for (;;) {
        // fetch the next group: one atomic by lane 0, broadcast through LDS
        __syncthreads();
        if (lane == 0) s_next = atomicAdd(a.counter, 1ull);
        __syncthreads();
        const int64_t g = uniform64(s_next);
        if (g >= a.ngroups) break;
        int pid = -1;       // output slot (mode 0: pair id)
        int sid = -1;       // sequence of this lane
        const uint8_t *cen = a.center;
        int m = a.m;
        int cid = -1;
        if (a.mode == 0) {
            pid = a.order ? a.order[g * 64 + lane] : (g * 64 + lane < a.nseq ? (int)(g * 64 + lane) : -1);
            sid = pid;
        } else {
            int64_t apos = -1, b0;
            if (a.mode == 1) {
                tri_group(a.gtotal - 1 - (a.gfirst + g), a.nseq, 64, &apos, &b0);
                cid = a.perm[apos];
            } else {
                b0 = a.gb0[g];
                cid = a.gcen[g];
            }
            const int64_t bpos = b0 + lane;
            if (bpos < a.nseq && bpos > apos) {
                sid = a.perm[bpos];
                pid = (int)(g * 64 + lane);   // output slot (mode 2); a self pair scores 0
                if (sid == cid) sid = -1;
            }
            cen = a.res + a.off[cid];
            m = (int)(a.off[cid + 1] - a.off[cid]);
        }
        const int64_t so = sid >= 0 ? a.off[sid] : 0;
        const int n = sid >= 0 ? (int)(a.off[sid + 1] - so) : 0;
        const uint8_t *s = a.res + so;
        // prefetch base: the set's first residue for an empty lane (a group
        // that runs any column holds at least one residue)
        const uint8_t *sq = n > 0 ? s : a.res;
        int nmax = n;
        if (a.mode == 0 && a.gnmax) {
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
            // The first strip reads residues from the lane's sequence and
            // leaves each column's code in its boundary cell (bits 27-31 of
            // F*, which stays below 2^23 for lengths < 65536 and |scores| <
            // 128); later strips get residue and boundary in one load.  A
            // block of kB columns is fetched one block ahead into the other of
            // two buffers, so the load latency overlaps a block of cells.  The
            // loads are unconditional (indexes clamped into the lane's
            // sequence and the group's boundary row) and so is the boundary
            // store, which keeps the wait counts exact across blocks.  Every
            // block is whole: columns past nmax (up to nmaxp, a multiple of kB)
            // are padding columns as for a lane's columns past n, whose cells
            // stay below an earlier cell of the lane and never win the end cell.
            const int nlast = max(n - 1, 0);
            const int nmaxp = (nmax + kB - 1) / kB * kB;
            auto strip = [&](auto first_tag) {
                constexpr bool FIRST = decltype(first_tag)::value;
                auto fetch = [&](int j0, int2 (&bq)[kB]) {
#pragma unroll
                    for (int b = 0; b < kB; ++b) {
                        const int j = min(j0 + b, nmaxp);
                        if (FIRST) bq[b].x = (int)sq[min(j - 1, nlast)];
                        else bq[b] = load_agent(bnd + (int64_t)(j - 1) * 64 + lane);
                    }
                };
                auto block = [&](int j0, const int2 (&bc)[kB]) {
#pragma unroll
                    for (int b = 0; b < kB; ++b) {
                        const int j = j0 + b;
                        int upg, upf, r;
                        if (FIRST) {
                            upg = -goe;
                            upf = 0;
                            r = (j <= n) ? (bc[b].x & 31) : kPad;
                        } else {
                            upg = bc[b].x;
                            upf = bc[b].y & kFMask;
                            r = (int)((uint32_t)bc[b].y >> 27);
                        }
                        int diag = diag0;
                        diag0 = upg;
                        const int *prow = prof + r * kPS;
                        int p[kT];
#pragma unroll
                        for (int t = 0; t < kT; ++t) p[t] = prow[t];
                        uint32_t w0 = 0, w1 = 0;
                        int colkey = 0;
#pragma unroll
                        for (int t = 0; t < kT; t += 2) {
                            const int h0 = sw_cell<TB>(hg[t], e[t], diag, upg, upf, p[t], ge, goe,
                                                       t < 8 ? w0 : w1);
                            const int h1 = sw_cell<TB>(hg[t + 1], e[t + 1], diag, upg, upf, p[t + 1], ge, goe,
                                                       t < 8 ? w0 : w1);
                            if (ENDC) colkey = vmax3(colkey, (h0 << 5) | (31 - t), (h1 << 5) | (30 - t));
                            else hmax = vmax3(hmax, h0, h1);
                        }
                        bnd[(int64_t)(j - 1) * 64 + lane] = make_int2(upg, upf | (r << 27));
                        if (TB) {
                            stage[2 * b] = w0;
                            stage[2 * b + 1] = w1;
                            if (b == kB - 1) {
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
                };
                int2 bA[kB], bB[kB];
                fetch(1, bA);
                for (int j0 = 1; j0 <= nmaxp; j0 += 2 * kB) {
                    fetch(j0 + kB, bB);
                    block(j0, bA);
                    if (j0 + kB > nmaxp) break;
                    fetch(j0 + 2 * kB, bA);
                    block(j0 + kB, bB);
                }
            };
            if (nmax > 0) {
                if (st == 0) strip(std::true_type{});
                else strip(std::false_type{});
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
                if (ENDC && a.cells4)
                    a.cells4[pid] = make_int4(0, 0, best.h > 0 ? best.i + 1 : 0, best.h > 0 ? best.j : 0);
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
// Packed 16-bit score-only strip kernel (center selection: modes 1 and 2).
// Each lane scores two pairs of the group at once, pair A (partner gb0+lane)
// in the low and pair B (partner gb0+64+lane) in the high half of every
// register, with v_pk_* 16-bit integer ops: a group holds 128 partners.
// E* and F* are clamped at 0 as in the 32-bit kernel, and all values are
// biased (below) so that each three-way maximum is one v_pk_maximum3_f16:
//   eext = e - ge; en = max(eext, Hg, 0); fext = F - ge; fn = max(fext, Hg_up, 0);
//   hd = Hg_diag + P; h = max(hd, en, fn); Hg = h - goe
// that is 8 packed ops per two cells plus half a maximum for the running
// maximum.  The host uses this kernel only when every H stays below 15000
// (max S * longest sequence + go + ge < 15000), so that no biased value
// leaves [0, 0x7c00) and a padding profile entry can never be a source.  The
// profile (int16 [r][16]) of the two lanes' residues is interleaved into
// (A, B) pairs with v_perm_b32.
// Strip boundaries per lane and column: packed Hg and packed F (int2) and the
// two residue codes (uint16), written by every strip and read by the next one
// with agent-scope loads (as in the 32-bit kernel).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
sw_inter16_kernel(InterArgs a) {
    __shared__ uint32_t prof[kAlphaMax * 8];   // int16 [r][16], 8 words per residue
    __shared__ int8_t smat[kAlphaMax * kAlphaMax];
    __shared__ unsigned long long s_next;
    const int lane = threadIdx.x;
    for (int x = lane; x < kAlphaMax * kAlphaMax; x += 64) {
        const int r = x >> 5, q = x & 31;
        smat[x] = (r < a.alpha && q < a.alpha) ? a.mat[r * a.alpha + q] : (int8_t)0;
    }
    // per workgroup: int2 (packed Hg, packed F) per lane and column, then the
    // lane's two residue codes (uint16) per column
    int2 *bnd = reinterpret_cast<int2 *>(reinterpret_cast<int4 *>(a.bound) + (int64_t)blockIdx.x * a.bstride);
    uint16_t *bres = reinterpret_cast<uint16_t *>(bnd + a.bstride);
    const pk16 ge2 = pk16{(short)a.ge, (short)a.ge};
    const pk16 goe2 = pk16{(short)a.goe, (short)a.goe};
    const pk16 bias2 = pk16{(short)kBias16, (short)kBias16};             // 0, biased
    const pk16 init2 = pk16{(short)(kBias16 - a.goe), (short)(kBias16 - a.goe)};   // -go - ge, biased
    for (;;) {
        __syncthreads();
        if (lane == 0) s_next = atomicAdd(a.counter, 1ull);
        __syncthreads();
        const int64_t g = uniform64(s_next);
        if (g >= a.ngroups) break;
        int64_t apos = -1, b0;
        int cid;
        if (a.mode == 1) {
            tri_group(a.gtotal - 1 - (a.gfirst + g), a.nseq, 128, &apos, &b0);
            cid = a.perm[apos];
        } else {
            b0 = a.gb0[g];
            cid = a.gcen[g];
        }
        const int64_t pa = b0 + lane, pbp = pa + 64;
        int sa = (pa < a.nseq && pa > apos) ? a.perm[pa] : -1;
        int sb = (pbp < a.nseq && pbp > apos) ? a.perm[pbp] : -1;
        sa = sa == cid ? -1 : sa;   // a self pair scores 0
        sb = sb == cid ? -1 : sb;
        const uint8_t *cen = a.res + a.off[cid];
        const int m = __builtin_amdgcn_readfirstlane((int)(a.off[cid + 1] - a.off[cid]));
        const int64_t soa = sa >= 0 ? a.off[sa] : 0, sob = sb >= 0 ? a.off[sb] : 0;
        const int na = sa >= 0 ? (int)(a.off[sa + 1] - soa) : 0;
        const int nb = sb >= 0 ? (int)(a.off[sb + 1] - sob) : 0;
        // prefetch bases: the set's first residue for an empty lane (a group
        // that runs any column holds at least one residue)
        const uint8_t *qa = na > 0 ? a.res + soa : a.res;
        const uint8_t *qb = nb > 0 ? a.res + sob : a.res;
        int nmax = max(na, nb);
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) nmax = max(nmax, __shfl_xor(nmax, sh));
        nmax = __builtin_amdgcn_readfirstlane(nmax);
        const int nstrips = (m + kT - 1) / kT;
        const int nmaxp = (nmax + kB - 1) / kB * kB;
        const int la = max(na - 1, 0), lb = max(nb - 1, 0);
        pk16 hmax = bias2;
        for (int st = 0; st < nstrips && nmax > 0; ++st) {
            const int i0 = st * kT;
            __syncthreads();
            for (int x = lane; x < kAlphaMax * 8; x += 64) {
                const int r = x >> 3, t = 2 * (x & 7);
                int v0 = kPadProf16, v1 = kPadProf16;
                if (r < a.alpha && i0 + t < m) v0 = (int)smat[(cen[i0 + t] & 31) * 32 + r] + a.goe;
                if (r < a.alpha && i0 + t + 1 < m) v1 = (int)smat[(cen[i0 + t + 1] & 31) * 32 + r] + a.goe;
                prof[x] = (uint32_t)(v0 & 0xffff) | ((uint32_t)v1 << 16);
            }
            __syncthreads();
            pk16 hg[kT], e[kT];
#pragma unroll
            for (int t = 0; t < kT; ++t) { hg[t] = init2; e[t] = init2; }
            pk16 diag0 = init2;
            auto strip = [&](auto first_tag) {
                constexpr bool FIRST = decltype(first_tag)::value;
                auto fetch = [&](int j0, int4 (&bq)[kB]) __attribute__((always_inline)) {
#pragma unroll
                    for (int b = 0; b < kB; ++b) {
                        const int j = min(j0 + b, nmaxp);
                        if (FIRST) {
                            bq[b].x = (int)qa[min(j - 1, la)];
                            bq[b].y = (int)qb[min(j - 1, lb)];
                        } else {
                            const int2 v = load_agent(bnd + (int64_t)(j - 1) * 64 + lane);
                            const uint32_t rw = __hip_atomic_load(
                                reinterpret_cast<const uint32_t *>(bres + (int64_t)(j - 1) * 64 + (lane & ~1)),
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            bq[b] = make_int4(v.x, v.y, (int)(rw >> (16 * (lane & 1))), 0);
                        }
                    }
                };
                auto block = [&](int j0, const int4 (&bc)[kB]) {
#pragma unroll
                    for (int b = 0; b < kB; ++b) {
                        const int j = j0 + b;
                        pk16 upg, upf;
                        int ra, rb;
                        if (FIRST) {
                            upg = init2;
                            upf = init2;
                            ra = (j <= na) ? (bc[b].x & 31) : kPad;
                            rb = (j <= nb) ? (bc[b].y & 31) : kPad;
                        } else {
                            upg = as_pk((uint32_t)bc[b].x);
                            upf = as_pk((uint32_t)bc[b].y);
                            ra = bc[b].z & 255;
                            rb = (bc[b].z >> 8) & 255;
                        }
                        pk16 diag = diag0;
                        diag0 = upg;
                        const uint4 *pa4 = reinterpret_cast<const uint4 *>(prof + ra * 8);
                        const uint4 *pb4 = reinterpret_cast<const uint4 *>(prof + rb * 8);
                        const uint4 a0 = pa4[0], a1 = pa4[1], b0 = pb4[0], b1 = pb4[1];
                        const uint32_t wa[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                        const uint32_t wb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
                        pk16 hh0 = bias2;
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int t = 2 * k + h;
                                const pk16 p = as_pk(__builtin_amdgcn_perm(wb[k], wa[k], h ? 0x07060302u : 0x05040100u));
                                const pk16 en = max3h(e[t] - ge2, hg[t], bias2);
                                const pk16 fn = max3h(upf - ge2, upg, bias2);
                                const pk16 hd = diag + p;
                                const pk16 hh = max3h(hd, en, fn);
                                if (h) hmax = max3h(hmax, hh0, hh);
                                else hh0 = hh;
                                diag = hg[t];
                                hg[t] = hh - goe2;
                                e[t] = en;
                                upg = hg[t];
                                upf = fn;
                            }
                        }
                        bnd[(int64_t)(j - 1) * 64 + lane] = make_int2((int)as_u(upg), (int)as_u(upf));
                        bres[(int64_t)(j - 1) * 64 + lane] = (uint16_t)(ra | (rb << 8));
                    }
                };
                int4 bA[kB], bB[kB];
                fetch(1, bA);
                for (int j0 = 1; j0 <= nmaxp; j0 += 2 * kB) {
                    fetch(j0 + kB, bB);
                    block(j0, bA);
                    if (j0 + kB > nmaxp) break;
                    fetch(j0 + 2 * kB, bA);
                    block(j0 + kB, bB);
                }
            };
            if (st == 0) strip(std::true_type{});
            else strip(std::false_type{});
        }
        const uint32_t hm = as_u(hmax);
        const int va = sa >= 0 ? (int)(hm & 0xffff) - kBias16 : 0;
        const int vb = sb >= 0 ? (int)(hm >> 16) - kBias16 : 0;
        if (a.mode == 1) {
            if (sa >= 0) atomicAdd(reinterpret_cast<unsigned long long *>(a.sums + sa), (unsigned long long)va);
            if (sb >= 0) atomicAdd(reinterpret_cast<unsigned long long *>(a.sums + sb), (unsigned long long)vb);
        }
        int tot = va + vb;
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) tot += __shfl_xor(tot, sh);
        if (lane == 0) {
            const int slot = a.mode == 1 ? cid : a.gslot[g];
            atomicAdd(reinterpret_cast<unsigned long long *>(a.sums + slot), (unsigned long long)(int64_t)tot);
        }
    }
}

}  // namespace hk
