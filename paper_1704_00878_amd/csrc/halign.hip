// Host runtime and C ABI of the center-star MSA library (gfx950).
//
// The runtime owns device scratch (traceback codes, boundary rows, plans) in
// a halign_ctx, plans each batch on the host (length sort, grouping, chunking
// under a workspace cap), and launches the kernels of sw_kernels.hpp and
// msa_kernels.hpp on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <sstream>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <chrono>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/halign.h"
#include "launch.hpp"
#include "msa_kernels.hpp"
#include "plan_kernels.hpp"
#include "strip_kernels.hpp"
#include "walk_kernels.hpp"
#include "nuc_kernels.hpp"
#include "nj_kernels.hpp"
#include "mlp_kernels.hpp"

namespace {

// message of the last failure on this thread (a fixed buffer: reporting an
// error allocates nothing)
thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HCHK(expr)                                                                   \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(HALIGN_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

using hk::launch_stream;
using hk::launch_stream16;
using hk::stream16_supported;
using hk::stream_supported;

#define RCHK(expr)                 \
    do {                           \
        int r_ = (expr);           \
        if (r_ != HALIGN_OK) return r_; \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct HostBuf {
    void *p = nullptr;
    size_t cap = 0;
};

}  // namespace

struct halign_ctx {
    int device = 0;
    size_t cap = 0;          // workspace cap for codes + boundary rows (0 = none)
    int num_cu = 256;
    size_t lds_max = 65536;
    size_t lds_cu = 65536;      // LDS of a CU: what one workgroup may take with the attribute set
    int last_pk = 0;          // the last batch ran the packed 16-bit wavefront kernel
    // device scratch
    DevBuf codes, bound, plan, counter, pairbuf, msabuf, spbuf, sbuf;
    DevBuf mlp[10];          // learned-center scratch (features, activations, gradients, moments)
    // pinned host staging for plans: regions are taken in order within a
    // call (stage_off, plan_off) and never reused before the call ends, so the
    // copies of a captured graph each read their own region
    HostBuf stage;
    size_t stage_off = 0, plan_off = 0;
    hipEvent_t ev_stage = nullptr;
    bool stage_pending = false;
    // timing of the last call: one (start, forward end, walk end) event
    // triple per forward launch (chunk, route or graph replay)
    std::vector<std::array<hipEvent_t, 3>> tev;
    int ntev = 0;
    int64_t last_stats[4] = {0, 0, 0, 0};
    int fault_chunk = -1;    // test hook: chunk index whose first launch reports failure
    bool capturing = false;   // a hipGraph capture of halign_sw_batch is in progress
    int use_graph = 0;        // halign_msa passes HALIGN_GRAPH to its batch
    hipStream_t cap_stream = nullptr;
    hipStream_t aux_stream = nullptr;   // the tree's small joins beside the chip-wide ones
    struct GraphEntry {
        uint64_t key = 0;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        DevBuf plan, codes, sbuf, bound, counter, pairbuf, spbuf;
        HostBuf stage;
    } gent;
    int64_t graph_launches = 0;
    int autotune = 0;         // 1: tune route / rows per lane / stream count per bucket
    int progress = 0;         // 1: a line on stderr after each chunk of a chunked batch
    std::array<int, 5> last_tune = {-1, 0, 1, 64, 0};
    std::map<std::string, std::array<int, 5>> tuned;   // bucket -> {route, R, stream multiplier, lanes per stream, packed}
    std::string tune_file;    // optional cache file (HALIGN_TUNE_CACHE)
    int *flag_host = nullptr; // pinned: (tag << 8 | largest residue code) of the last validated call
    int64_t *mail_host = nullptr, *mail_dev = nullptr;   // coherent pinned mailbox: width, sequence number
    DevBuf nuctab, nucscr, nucdp;   // nucleotide path: segment table, matches and chains, stretch scratch
    DevBuf rowck;                   // chunked rows: residues before each chunk of blocks, per row
    DevBuf njrows, njD, njS, njacc, njB; // phylogeny: row lists and group tables, distance matrices, join scratch, slice counts, chip-wide join scratch
    int64_t mail_seq = 0;
    uint32_t vtag = 0;        // tag of the last eager code check
    uint32_t *vflag = nullptr;   // the flag word those tags were raised in (cleared when it changes)
    uint32_t check_tag = 0;   // tag validate_check expects (0 after a graph replay)
    int flag_alpha = 0;       // alphabet that value is checked against (0 = nothing pending)
    // HALIGN_HOST_TIMING=1: host time between labelled points of each
    // halign_msa call, one line on stderr per call
    int host_timing = 0;
    std::vector<std::pair<const char *, double>> hmarks;
    // learned center: pre-judge of the top prejudge_cand candidates by u
    // against prejudge_part common partners (0: off)
    int prejudge_cand = 0, prejudge_part = 0;
    // host planning scratch, kept between calls (no allocation per call)
    std::vector<int32_t> h_pids, h_plen, h_cnt, h_sof, h_head, h_nxt, h_scount, h_cur, h_split;
    std::vector<int64_t> h_scols;
    // the last tuned-plan lookup, by its integer key
    int64_t tkey[4] = {-1, -1, -1, -1};
    std::array<int, 5> tval = {-1, 0, 1, 64, 0};
};

namespace {

void hmark(halign_ctx *ctx, const char *label) {
    if (!ctx->host_timing) return;
    const double us =
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
    ctx->hmarks.push_back({label, us});
}

void hmark_print(halign_ctx *ctx) {
    if (!ctx->host_timing || ctx->hmarks.size() < 2) return;
    fprintf(stderr, "halign host us:");
    for (size_t q = 1; q < ctx->hmarks.size(); ++q)
        fprintf(stderr, " %s %.1f", ctx->hmarks[q].first, ctx->hmarks[q].second - ctx->hmarks[q - 1].second);
    fprintf(stderr, " (total %.1f)\n", ctx->hmarks.back().second - ctx->hmarks.front().second);
    ctx->hmarks.clear();
}

int grow(halign_ctx *ctx, DevBuf &b, size_t bytes) {
    if (bytes <= b.cap) return HALIGN_OK;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 4095) & ~size_t(4095);
    if (b.p) HCHK(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(HALIGN_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        }
        want = bytes;
    }
    b.cap = want;
    (void)ctx;
    return HALIGN_OK;
}

// Event records are skipped while a graph is being captured (timing of a
// replay comes from events around the graph launch).
int record(halign_ctx *ctx, hipEvent_t e, hipStream_t st) {
    if (ctx->capturing) return HALIGN_OK;
    HCHK(hipEventRecord(e, st));
    return HALIGN_OK;
}

void free_buf(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b = DevBuf();
}

void graph_drop(halign_ctx *ctx) {
    auto &g = ctx->gent;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    for (DevBuf *b : {&g.plan, &g.codes, &g.sbuf, &g.bound, &g.counter, &g.pairbuf, &g.spbuf}) free_buf(*b);
    if (g.stage.p) (void)hipHostFree(g.stage.p);
    g = halign_ctx::GraphEntry();
}

int stage_wait(halign_ctx *ctx) {
    if (ctx->capturing) return HALIGN_OK;
    if (ctx->stage_pending) {
        HCHK(hipEventSynchronize(ctx->ev_stage));
        ctx->stage_pending = false;
    }
    return HALIGN_OK;
}

// Start of a call: the previous call's copies have left the pinned stage,
// whose regions are then taken from its start again; the timing triples
// restart too.
int stage_begin(halign_ctx *ctx) {
    RCHK(stage_wait(ctx));
    ctx->stage_off = 0;
    ctx->plan_off = 0;
    ctx->ntev = 0;
    return HALIGN_OK;
}

// `bytes` of the pinned stage, after the regions this call took already.
int stage_host(halign_ctx *ctx, size_t bytes, char **host) {
    const size_t o = (ctx->stage_off + 255) & ~size_t(255);
    if (o + bytes > ctx->stage.cap) {
        if (ctx->capturing) return fail(HALIGN_E_UNSUPPORTED, "plan staging outgrew its buffer under graph capture");
        RCHK(stage_wait(ctx));   // the regions taken so far have been copied
        if (ctx->stage.p) HCHK(hipHostFree(ctx->stage.p));
        ctx->stage.p = nullptr;
        ctx->stage.cap = 0;
        const size_t want = std::max<size_t>(2 * (o + bytes), 1 << 16);
        HCHK(hipHostMalloc(&ctx->stage.p, want, hipHostMallocDefault));
        ctx->stage.cap = want;
    }
    *host = (char *)ctx->stage.p + o;
    ctx->stage_off = o + bytes;
    return HALIGN_OK;
}

// `bytes` of the device plan buffer, after the regions this call took already
// (a larger buffer replaces it only once the stream has drained).
int plan_dev(halign_ctx *ctx, size_t bytes, hipStream_t st, char **dev) {
    const size_t o = (ctx->plan_off + 255) & ~size_t(255);
    if (o + bytes > ctx->plan.cap) {
        if (ctx->capturing) return fail(HALIGN_E_UNSUPPORTED, "plan outgrew its buffer under graph capture");
        if (ctx->plan.p) HCHK(hipStreamSynchronize(st));
        RCHK(grow(ctx, ctx->plan, 2 * (o + bytes)));
    }
    *dev = (char *)ctx->plan.p + o;
    ctx->plan_off = o + bytes;
    return HALIGN_OK;
}

// The next timing triple of this call (created on first use).
int tev_next(halign_ctx *ctx, std::array<hipEvent_t, 3> **out) {
    if (ctx->ntev == (int)ctx->tev.size()) {
        std::array<hipEvent_t, 3> t{};
        for (auto &e : t) HCHK(hipEventCreate(&e));
        ctx->tev.push_back(t);
    }
    *out = &ctx->tev[ctx->ntev++];
    return HALIGN_OK;
}

// Forward and walk time (ms) summed over the triples of the last call
// (synchronises on the last one).
int tev_sum(halign_ctx *ctx, float *fwd, float *walk) {
    *fwd = *walk = 0.f;
    if (ctx->ntev == 0) return HALIGN_OK;
    HCHK(hipEventSynchronize(ctx->tev[ctx->ntev - 1][2]));
    for (int q = 0; q < ctx->ntev; ++q) {
        float f = 0.f, w = 0.f;
        HCHK(hipEventElapsedTime(&f, ctx->tev[q][0], ctx->tev[q][1]));
        HCHK(hipEventElapsedTime(&w, ctx->tev[q][1], ctx->tev[q][2]));
        *fwd += f;
        *walk += w;
    }
    return HALIGN_OK;
}

// A packed plan: host arrays laid out in one staging buffer and copied with
// one H2D transfer into ctx->plan.
struct PlanBuilder {
    std::vector<std::pair<size_t, size_t>> parts;  // (offset, bytes)
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t o = (total + 255) & ~size_t(255);
        parts.push_back({o, bytes});
        total = o + bytes;
        return o;
    }
};

inline int grid_for(int64_t n, int block, int maxg = 65536) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, maxg));
}

int launch_fill(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return HALIGN_OK;
    hipLaunchKernelGGL(hk::fill_u32_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, v, n);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int check_scoring(const halign_scoring *sc) {
    if (!sc || !sc->matrix_host) return fail(HALIGN_E_INVALID, "scoring is NULL");
    if (sc->alphabet <= 0 || sc->alphabet > hk::kAlphaMax)
        return fail(HALIGN_E_UNSUPPORTED, "alphabet %d outside 1..32", sc->alphabet);
    if (sc->gap_open < 0 || sc->gap_extend < 1)
        return fail(HALIGN_E_UNSUPPORTED, "need gap_open >= 0 and gap_extend >= 1");
    if (sc->gap_open + sc->gap_extend > 1000000)
        return fail(HALIGN_E_UNSUPPORTED, "gap costs too large");
    return HALIGN_OK;
}

int check_seqs(const halign_seqs *sq) {
    if (!sq || sq->n < 0) return fail(HALIGN_E_INVALID, "seqs is NULL or n < 0");
    if (sq->n == 0) return HALIGN_OK;
    if (!sq->residues || !sq->offsets || !sq->offsets_host)
        return fail(HALIGN_E_INVALID, "seqs pointers are NULL");
    const int64_t *o = sq->offsets_host;
    if (o[0] != 0) return fail(HALIGN_E_INVALID, "offsets[0] must be 0");
    for (int k = 0; k < sq->n; ++k) {
        const int64_t L = o[k + 1] - o[k];
        if (L < 0) return fail(HALIGN_E_INVALID, "offsets decrease at %d", k);
        if (L >= 65536) return fail(HALIGN_E_UNSUPPORTED, "sequence %d has length %lld >= 65536", k, (long long)L);
    }
    return HALIGN_OK;
}

// Device matrix copy (alpha x alpha int8) kept in the plan buffer head.
struct Scoring {
    const int8_t *dmat;
    const int8_t *hmat;   // host copy (planning decisions)
    int alpha, ge, goe;
};

// ---------------------------------------------------------------------------
// Forward + walk for one set of pairs against one center.
// ---------------------------------------------------------------------------
enum Route { kRouteIntra = 0, kRouteInter = 1 };

// pairs longer than this (sequence residues) run on the wavefront kernel even
// in a batch that runs one pair per lane
constexpr int kLongPair = 1000;

// Rows per lane and passes of the wavefront kernel: passes = ceil(m / 512),
// R = ceil(m / (64 * passes)) <= 8, so a pass holds 64*R >= m/passes rows.
void pick_geom(int m, int *R, int *passes) {
    const int p = std::max(1, (m + 511) / 512);
    *passes = p;
    *R = std::max(1, std::min(8, (m + 64 * p - 1) / (64 * p)));
}

// Boundary-row columns per strip-kernel lane: the longest sequence rounded
// up to whole prefetch blocks.
int64_t strip_cols(int nmax_all) {
    return ((int64_t)std::max(1, nmax_all) + hk::kB - 1) / hk::kB * hk::kB;
}

void launch_inter(const hk::InterArgs &a, bool tb, bool endc, int grid, hipStream_t st) {
    if (tb)
        hipLaunchKernelGGL((hk::sw_inter_kernel<true, true>), dim3(grid), dim3(64), 0, st, a);
    else if (endc)
        hipLaunchKernelGGL((hk::sw_inter_kernel<false, true>), dim3(grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((hk::sw_inter_kernel<false, false>), dim3(grid), dim3(64), 0, st, a);
}

struct BatchOut {
    int32_t *score, *cells, *endcell;
    uint16_t *ins;
    uint32_t *aligned;
    int32_t *G = nullptr;   // optional: max-merge of ins into G during the walk
    int gskip = -1;         // pair left out of G (the center itself)
};

// Plans and runs the forward pass (+ walk when tb) for the pairs `pids_in`
// against center (device) of length m.
struct Tune {
    int route = -1;   // -1: from flags
    int R = 0;        // 0: fitted to m
    int smul = 1;     // streams per resident wave slot
    double scale = 1; // stream count scale (a sample keeps the batch's pairs per stream)
    int LS = 0;       // lanes per stream (0: 64)
    int pk = 0;       // 1: packed 16-bit wavefront kernel (two streams per lane group)
};

// pairs_in: the pair ids of the batch (NULL: 0 .. np-1).
int run_batch(halign_ctx *ctx, const Scoring &S, const uint8_t *center, int m, const halign_seqs *sq,
              const int32_t *pids_in, int np, bool tb, bool endc, int route, const BatchOut &out, hipStream_t st,
              const Tune &tune = Tune()) {
    const int64_t *oh = sq->offsets_host;
    const int N = sq->n;
    if (np == 0) return HALIGN_OK;
    auto pid_of = [&](int x) { return pids_in ? pids_in[x] : x; };
    // longest first (counting sort on length, stable); plen[x] = length of
    // pids[x], so that later passes read lengths in order
    if ((int)ctx->h_pids.size() < np) {
        ctx->h_pids.resize(np);
        ctx->h_plen.resize(np);
    }
    int32_t *pids = ctx->h_pids.data(), *plen = ctx->h_plen.data();
    int64_t sum_len = 0;
    {
        int maxlen = 0;
        for (int x = 0; x < np; ++x) {
            const int p = pid_of(x);
            maxlen = std::max(maxlen, (int)(oh[p + 1] - oh[p]));
        }
        std::vector<int32_t> &cnt = ctx->h_cnt;
        cnt.assign(maxlen + 2, 0);
        for (int x = 0; x < np; ++x) {
            const int p = pid_of(x);
            const int L = (int)(oh[p + 1] - oh[p]);
            cnt[maxlen - L]++;
            sum_len += L;
        }
        int acc = 0;
        for (auto &c : cnt) { const int v = c; c = acc; acc += v; }
        for (int x = 0; x < np; ++x) {
            const int p = pid_of(x);
            const int L = (int)(oh[p + 1] - oh[p]);
            const int q = cnt[maxlen - L]++;
            pids[q] = p;
            plen[q] = L;
        }
    }
    hmark(ctx, "sort");
    const int aw = (m + 31) / 32;
    // int16 profile when every score and profile entry fits in 16 bits:
    // max score <= max(S) * min(m, longest sequence)
    int smax = 1;
    for (int x = 0; x < S.alpha * S.alpha; ++x) smax = std::max(smax, (int)S.hmat[x]);
    const int nlong = plen[0];
    const bool p16 = (int64_t)smax * std::min(m, nlong) <= 32000 && S.goe + 128 <= 32000 &&
                     !getenv("HALIGN_PROFILE32");
    int R = 8, passes = 1, LS = 64;
    pick_geom(m, &R, &passes);
    if (tune.route >= 0) route = tune.route;
    if (tune.R > 0 && stream_supported(tune.R, tune.LS > 0 ? tune.LS : 64, p16)) {
        LS = tune.LS > 0 ? tune.LS : 64;
        R = tune.R;
        passes = std::max(1, (m + LS * R - 1) / (LS * R));
    } else if (const char *e = getenv("HALIGN_STREAM_LANES")) {   // test knob: narrower streams
        const int ls = atoi(e);
        const int ps = std::max(1, (m + ls * 16 - 1) / std::max(1, ls * 16));
        const int r = std::max(2, (m + ls * ps - 1) / std::max(1, ls * ps));
        if ((ls == 32 || ls == 16) && stream_supported(r, ls, p16)) {
            LS = ls;
            R = r;
            passes = ps;
        }
    }
    // packed 16-bit wavefront kernel: asked for by the tuner (or the test knob
    // HALIGN_STREAM_PACK=1 with the lanes knob), traceback with end cells only,
    // and only when every H stays below 15000 and the gap costs are small
    bool pk = false;
    {
        const char *e = getenv("HALIGN_STREAM_PACK");
        const bool want = tune.R > 0 ? tune.pk > 0 : (e && atoi(e) != 0);
        const bool fits = p16 && tb && endc && (int64_t)smax * std::min(m, nlong) < 15000 && S.goe <= 256 &&
                          S.ge <= 256;
        pk = want && fits && route == kRouteIntra && stream16_supported(R, LS);
    }
    const int W = (R + 7) / 8, NS = 64 / LS;
    const int WQ = pk ? (R + 3) / 4 : W;   // code words per step
    const size_t prof_bytes =
        p16 ? (size_t)(S.alpha + 1) * LS * 16 * W : (size_t)hk::kAlphaMax * LS * R * 4;
    const size_t lds_stream = prof_bytes + (tb ? (pk ? (size_t)8 * 256 * 4 * WQ : (size_t)8 * 512 * 4 * W) : 0);
    if (route == kRouteIntra && lds_stream > ctx->lds_max) route = kRouteInter;
    ctx->last_stats[2] = route;
    ctx->last_pk = pk ? 1 : 0;

    // chunk the pairs so that codes + boundary rows fit the cap
    const size_t cap = ctx->cap ? ctx->cap : (size_t)1 << 62;
    std::vector<std::pair<int, int>> chunks;  // [lo, hi) in pids
    const size_t intra_bytes =
        (tb ? (size_t)passes * LS * 4 * WQ * ((size_t)sum_len + (size_t)(LS + 8) * (size_t)np) : 0) +
        (size_t)(passes - 1) * 8 * (size_t)sum_len;
    if (route == kRouteIntra && intra_bytes <= cap) {
        chunks.push_back({0, np});
    } else {
        const int nst = (m + hk::kT - 1) / hk::kT;
        int lo = 0;
        size_t acc = 0;
        for (int x = 0; x < np; ++x) {
            const int n = plen[x];
            size_t b = 0;
            bool boundary = true;
            if (route == kRouteIntra) {
                b = (tb ? (size_t)passes * (n + LS + 8) * LS * 4 * WQ : 0) + (size_t)(passes - 1) * n * 8;
            } else {
                boundary = (x - lo) % 64 == 0;
                b = (boundary && tb) ? (size_t)nst * ((n + 3) / 4) * 512 * 4 : 0;  // group charged by its longest
            }
            if (boundary && x > lo && acc + b > cap) {
                chunks.push_back({lo, x});
                lo = x;
                acc = 0;
            }
            acc += b;
        }
        chunks.push_back({lo, np});
    }
    ctx->last_stats[3] += (int64_t)chunks.size();
    const int64_t cells_total = (int64_t)m * sum_len;
    ctx->last_stats[0] += cells_total;
    RCHK(grow(ctx, ctx->counter, 256));
    unsigned long long *counter = (unsigned long long *)ctx->counter.p;

    int64_t launches = 0;
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        const int lo = chunks[ci].first, hi = chunks[ci].second;
        const int cn = hi - lo;
        PlanBuilder pb;
        size_t code_words = 0, bound_elems = 0;
        int nmax_all = 0;
        nmax_all = plen[lo];
        // strip route: the walk list and its walk descriptors, both in walk
        // order (the wavefront route's walk reads the per-slot and per-stream
        // plan)
        const bool strip_plan = route != kRouteIntra;
        const size_t o_cbase = strip_plan ? pb.add(sizeof(int64_t) * cn) : 0,
                     o_cstr = strip_plan ? pb.add(sizeof(int32_t) * cn) : 0,
                     o_ccol = strip_plan ? pb.add(sizeof(int32_t) * cn) : 0,
                     o_walk = strip_plan ? pb.add(sizeof(int32_t) * cn) : 0;
        size_t o_sbeg = 0, o_slot0 = 0, o_scb = 0, o_sbb = 0, o_spid = 0, o_scol = 0, o_sstr = 0;
        size_t o_order = 0, o_gnmax = 0, o_gcb = 0;
        int nstreams = 0, nslots = 0, ngroups = 0;
        int64_t total_cols = 0;
        int nonempty = 0;   // pairs [0, nonempty) of the chunk are non-empty: empty pairs sort last
        for (int x = hi - 1; x >= lo && plen[x] == 0; --x) ++nonempty;
        nonempty = cn - nonempty;
        const char *deal_env = getenv("HALIGN_DEAL");   // test knob: snake dealing
        const bool deal_lpt = !(deal_env && !strcmp(deal_env, "snake"));
        if (route == kRouteIntra) {
            // streams: snake-deal the (longest first) non-empty pairs over the
            // resident waves so that every stream has about the same columns
            // resident workgroups per CU: by LDS, and by registers (the packed
            // kernel and the 32-bit one with R > 6 hold four waves per SIMD,
            // the 32-bit one with R <= 6 six)
            const int waves_simd = (pk || R > 6) ? 4 : 6;
            const int wg_per_cu = std::max(1, std::min({4, (int)(ctx->lds_max / lds_stream), waves_simd * 4 / 8}));
            const int resident = ctx->num_cu * wg_per_cu * 8 * NS * std::max(1, tune.smul) * (pk ? 2 : 1);
            nstreams = std::max(1, std::min(nonempty, (int)std::max(1.0, resident * tune.scale)));
            if (const char *e = getenv("HALIGN_MAX_STREAMS")) {   // test knob: many pairs per stream
                const int cap_s = atoi(e);
                if (cap_s > 0) nstreams = std::min(nstreams, cap_s);
            }
            nslots = cn;
            o_sbeg = pb.add(sizeof(int64_t) * (nstreams + 1));
            o_slot0 = pb.add(sizeof(int32_t) * nstreams);
            o_scb = pb.add(sizeof(int64_t) * nstreams);
            o_sbb = pb.add(sizeof(int64_t) * nstreams);
            o_spid = pb.add(sizeof(int32_t) * nslots);
            o_scol = pb.add(sizeof(int64_t) * nslots);
            o_sstr = pb.add(sizeof(int32_t) * nslots);
        } else {
            ngroups = (cn + 63) / 64;
            o_order = pb.add(sizeof(int32_t) * (size_t)ngroups * 64);
            o_gnmax = pb.add(sizeof(int32_t) * ngroups);
            o_gcb = pb.add(sizeof(int64_t) * ngroups);
        }
        char *hs = nullptr;
        RCHK(stage_host(ctx, pb.total, &hs));
        int32_t *h_walk = (int32_t *)(hs + o_walk);
        int64_t *h_cbase = (int64_t *)(hs + o_cbase);
        int32_t *h_cstr = (int32_t *)(hs + o_cstr);
        int32_t *h_ccol = (int32_t *)(hs + o_ccol);
        if (strip_plan)
            for (int x = 0; x < cn; ++x) h_walk[x] = pids[lo + x];
        if (route == kRouteIntra) {
            int64_t *h_sbeg = (int64_t *)(hs + o_sbeg);
            int32_t *h_slot0 = (int32_t *)(hs + o_slot0);
            int64_t *h_scb = (int64_t *)(hs + o_scb);
            int64_t *h_sbb = (int64_t *)(hs + o_sbb);
            int32_t *h_spid = (int32_t *)(hs + o_spid);
            int64_t *h_scol = (int64_t *)(hs + o_scol);
            int32_t *h_sstr = (int32_t *)(hs + o_sstr);   // stream of each slot (for the walk)
            // pairs and columns of each stream, then slots grouped by stream.
            // Snake dealing: the k-th non-empty pair, k = r * nstreams + q, goes
            // to stream q in even rounds r and nstreams - 1 - q in odd ones.
            // Least-loaded dealing: each pair (longest first) goes to the stream
            // with the fewest columns so far (a bucket queue on the column
            // count, whose minimum only grows), so streams end within one pair
            // length of each other.
            std::vector<int32_t> &scount = ctx->h_scount;
            std::vector<int64_t> &scols = ctx->h_scols;
            scount.assign(nstreams, 0);
            scols.assign(nstreams, 0);
            std::vector<int32_t> &sof = ctx->h_sof;   // least-loaded dealing: stream of each non-empty pair
            int64_t sum_ne = 0;
            for (int x = 0; x < nonempty; ++x) sum_ne += plen[lo + x];
            const int64_t maxload = (nonempty > 0 ? sum_ne / nstreams + plen[lo] : 0) + 1;
            const bool lpt = deal_lpt && maxload <= ((int64_t)1 << 22);
            hmark(ctx, "p_setup");
            if (lpt) {
                if ((int)sof.size() < nonempty) sof.resize(nonempty);
                std::vector<int32_t> &head = ctx->h_head, &nxt = ctx->h_nxt;
                head.assign(maxload + 1, -1);
                if ((int)nxt.size() < nstreams) nxt.resize(nstreams);
                for (int s2 = 0; s2 < nstreams; ++s2) nxt[s2] = s2 + 1 < nstreams ? s2 + 1 : -1;
                head[0] = 0;
                int64_t minp = 0;
                for (int x = 0; x < nonempty; ++x) {
                    while (head[minp] < 0) ++minp;
                    const int s2 = head[minp];
                    head[minp] = nxt[s2];
                    sof[x] = s2;
                    scount[s2]++;
                    scols[s2] += plen[lo + x];
                    const int64_t l2 = minp + plen[lo + x];
                    nxt[s2] = head[l2];
                    head[l2] = s2;
                }
            } else {
                int r = 0, q = 0;   // round and position of the next non-empty pair
                for (int x = 0; x < nonempty; ++x) {
                    const int s2 = (r & 1) ? nstreams - 1 - q : q;
                    scount[s2]++;
                    scols[s2] += plen[lo + x];
                    if (++q == nstreams) { q = 0; ++r; }
                }
            }
            hmark(ctx, "p_deal");
            int slot = 0;
            int64_t col = 0;
            for (int s = 0; s < nstreams; ++s) {
                h_slot0[s] = slot;
                h_sbeg[s] = col;
                slot += scount[s];
                col += scols[s];
                h_scb[s] = (int64_t)code_words;
                h_sbb[s] = (int64_t)bound_elems;
                if (pk) {
                    // stream pair (s, s+1) shares the tiles and boundary rows of a
                    // lane group, sized by the longer stream
                    if (s & 1) {
                        h_scb[s] = h_scb[s - 1];
                        h_sbb[s] = h_sbb[s - 1];
                        continue;
                    }
                    const int64_t cq = std::max(scols[s], s + 1 < nstreams ? scols[s + 1] : (int64_t)0);
                    if (tb) code_words += (size_t)passes * ((cq + LS - 1 + 7) / 8) * LS * 8 * WQ;
                    if (passes > 1) bound_elems += (size_t)(passes - 1) * cq;
                    continue;
                }
                if (tb) code_words += (size_t)passes * ((scols[s] + LS - 1 + 7) / 8) * LS * 8 * W;
                if (passes > 1) bound_elems += (size_t)(passes - 1) * scols[s];
            }
            h_sbeg[nstreams] = col;
            total_cols = col;
            hmark(ctx, "p_streams");
            if (lpt) {
                // slots of each stream in dealing order (longest first): the
                // pairs are sorted by stream in host memory first, so that the
                // pinned plan is written sequentially
                std::vector<int32_t> &cur = ctx->h_cur, &ord = ctx->h_nxt;
                cur.assign(h_slot0, h_slot0 + nstreams);
                if ((int)ord.size() < nonempty) ord.resize(nonempty);
                for (int x = 0; x < nonempty; ++x) ord[cur[sof[x]]++] = x;
                for (int s2 = 0, qs = 0; s2 < nstreams; ++s2) {
                    int64_t c = h_sbeg[s2];
                    for (int pl = 0; pl < scount[s2]; ++pl, ++qs) {
                        const int x = ord[qs];
                        h_spid[qs] = pids[lo + x];
                        h_scol[qs] = c;
                        h_sstr[qs] = s2;
                        c += plen[lo + x];
                    }
                }
            } else {
                // slots stream by stream (sequential writes): the pl-th pair of
                // stream s is non-empty pair pl * nstreams + (pl odd ? nstreams - 1 - s : s)
                for (int s = 0; s < nstreams; ++s) {
                    int64_t c = h_sbeg[s];
                    for (int pl = 0, qs = h_slot0[s]; pl < scount[s]; ++pl, ++qs) {
                        const int x = pl * nstreams + ((pl & 1) ? nstreams - 1 - s : s);
                        h_spid[qs] = pids[lo + x];
                        h_scol[qs] = c;
                        h_sstr[qs] = s;
                        c += plen[lo + x];
                    }
                }
            }
            for (int x = nonempty; x < cn; ++x) {   // empty pairs after the streamed ones
                h_spid[x] = pids[lo + x];
                h_scol[x] = 0;
                h_sstr[x] = 0;
            }
        } else {
            int32_t *h_order = (int32_t *)(hs + o_order);
            int32_t *h_gnmax = (int32_t *)(hs + o_gnmax);
            int64_t *h_gcb = (int64_t *)(hs + o_gcb);
            const int nst = (m + hk::kT - 1) / hk::kT;
            for (int g = 0; g < ngroups; ++g) {
                int nmax = 0;
                for (int l = 0; l < 64; ++l) {
                    const int x = lo + g * 64 + l;
                    h_order[g * 64 + l] = x < hi ? pids[x] : -1;
                    if (x < hi) nmax = std::max(nmax, plen[x]);
                }
                h_gnmax[g] = nmax;
                h_gcb[g] = (int64_t)code_words;
                // walk entry q = g * 64 + l is the pair in lane l of group g
                for (int l = 0; l < 64 && lo + g * 64 + l < hi; ++l) {
                    const int q = g * 64 + l;
                    h_cbase[q] = (int64_t)code_words;
                    h_ccol[q] = l;
                    h_cstr[q] = nmax;
                }
                if (tb) code_words += (size_t)nst * ((nmax + 3) / 4) * 512;
            }
        }
        hmark(ctx, "plan");
        char *dplan = nullptr;
        RCHK(plan_dev(ctx, pb.total, st, &dplan));
        HCHK(hipMemcpyAsync(dplan, hs, pb.total, hipMemcpyHostToDevice, st));
        RCHK(record(ctx, ctx->ev_stage, st));
        ctx->stage_pending = true;
        std::array<hipEvent_t, 3> *tv = nullptr;
        RCHK(tev_next(ctx, &tv));

        if (tb) RCHK(grow(ctx, ctx->codes, std::max<size_t>(4, code_words * 4)));
        if (ctx->fault_chunk == (int)ci) {
            ctx->fault_chunk = -1;
            return fail(HALIGN_E_DEVICE, "injected failure in chunk %d", (int)ci);
        }
        if (route == kRouteIntra) {
            // staged stream residues and per-slot keys share one scratch buffer
            const size_t keys_b = ((size_t)nslots * 8 + 255) & ~size_t(255);
            RCHK(grow(ctx, ctx->sbuf, keys_b + (size_t)total_cols + 64));
            unsigned long long *keys = (unsigned long long *)ctx->sbuf.p;
            uint8_t *sres = (uint8_t *)ctx->sbuf.p + keys_b;
            if (passes > 1) RCHK(grow(ctx, ctx->bound, std::max<size_t>(8, bound_elems * 8)));
            hipLaunchKernelGGL(hk::stage_stream_kernel, dim3(nslots), dim3(128), 0, st, sq->residues, sq->offsets,
                               (const int32_t *)(dplan + o_spid), (const int64_t *)(dplan + o_scol), nslots,
                               p16 ? S.alpha : 31, sres, keys);
            HCHK(hipGetLastError());
            RCHK(record(ctx, (*tv)[0], st));
            hk::StreamArgs a{};
            a.mat = S.dmat;
            a.alpha = S.alpha;
            a.center = center;
            a.m = m;
            a.passes = passes;
            a.sres = sres;
            a.sbeg = (const int64_t *)(dplan + o_sbeg);
            a.nstreams = nstreams;
            a.ge = S.ge;
            a.goe = S.goe;
            a.keys = keys;
            a.sslot0 = (const int32_t *)(dplan + o_slot0);
            a.codes = tb ? (uint32_t *)ctx->codes.p : nullptr;
            a.scbase = (const int64_t *)(dplan + o_scb);
            a.bound = (int2 *)ctx->bound.p;
            a.sbbase = (const int64_t *)(dplan + o_sbb);
            if (pk) launch_stream16(R, LS, a, (((nstreams + 1) / 2 + NS - 1) / NS + 7) / 8, lds_stream, st);
            else launch_stream(R, LS, a, tb, endc, p16, ((nstreams + NS - 1) / NS + 7) / 8, lds_stream, st);
            HCHK(hipGetLastError());
            RCHK(record(ctx, (*tv)[1], st));
            hipLaunchKernelGGL(hk::decode_keys_kernel, dim3(grid_for(nslots, 256, 1 << 30)), dim3(256), 0, st,
                               (const unsigned long long *)keys, (const int32_t *)(dplan + o_spid), nslots, out.score,
                               endc ? out.endcell : (int32_t *)nullptr);
            HCHK(hipGetLastError());
        } else {
            const int slots = ctx->num_cu * 16;
            const int grid = std::max(1, std::min(ngroups, slots));
            RCHK(grow(ctx, ctx->bound, (size_t)grid * 64 * strip_cols(nmax_all) * 8));
            RCHK(launch_fill((uint32_t *)counter, 0u, 2, st));
            RCHK(record(ctx, (*tv)[0], st));
            hk::InterArgs a{};
            a.mat = S.dmat;
            a.alpha = S.alpha;
            a.center = center;
            a.m = m;
            a.res = sq->residues;
            a.off = sq->offsets;
            a.mode = 0;
            a.order = (const int32_t *)(dplan + o_order);
            a.gnmax = (const int32_t *)(dplan + o_gnmax);
            a.ngroups = ngroups;
            a.ge = S.ge;
            a.goe = S.goe;
            a.counter = counter;
            a.score = out.score;
            a.endcell = out.endcell;
            a.codes = tb ? (uint32_t *)ctx->codes.p : nullptr;
            a.gcode_base = (const int64_t *)(dplan + o_gcb);
            a.bound = (int2 *)ctx->bound.p;
            a.bstride = (int64_t)64 * strip_cols(nmax_all);
            launch_inter(a, tb, endc, grid, st);
            HCHK(hipGetLastError());
            RCHK(record(ctx, (*tv)[1], st));
        }
        ++launches;
        if (tb) {
            hk::WalkArgs w{};
            w.mat = S.dmat;
            w.alpha = S.alpha;
            w.center = center;
            w.m = m;
            w.res = sq->residues;
            w.off = sq->offsets;
            w.pids = strip_plan ? (const int32_t *)(dplan + o_walk) : nullptr;
            w.npairs = cn;
            if (!strip_plan) {
                w.slot_pid = (const int32_t *)(dplan + o_spid);
                w.slot_col = (const int64_t *)(dplan + o_scol);
                w.sbeg = (const int64_t *)(dplan + o_sbeg);
                w.slot0 = (const int32_t *)(dplan + o_slot0);
                w.slot_stream = (const int32_t *)(dplan + o_sstr);
                w.scb = (const int64_t *)(dplan + o_scb);
                w.nstreams = nstreams;
            }
            w.ge = S.ge;
            w.goe = S.goe;
            w.score = out.score;
            w.endcell = out.endcell;
            w.codes = (const uint32_t *)ctx->codes.p;
            w.cbase = strip_plan ? (const int64_t *)(dplan + o_cbase) : nullptr;
            w.cstride = strip_plan ? (const int32_t *)(dplan + o_cstr) : nullptr;
            w.ccol = strip_plan ? (const int32_t *)(dplan + o_ccol) : nullptr;
            w.R = R;
            w.lg_ls = LS == 64 ? 6 : (LS == 32 ? 5 : 4);
            w.W = WQ;
            w.kind = route == kRouteIntra ? 0 : 1;
            w.cells = out.cells;
            w.ins = out.ins;
            w.aligned = out.aligned;
            w.aw = aw;
            w.G = out.G;
            w.gskip = out.gskip;
            // cached chunk shape: about as many rows (NB blocks of R rows) as
            // columns (NG chunk columns of 8 or 4), NB * NG = 16
            const int wR = route == kRouteIntra ? R : 16;
            w.rmagic = wR >= 2 ? (uint32_t)((((uint64_t)1 << 32) + wR - 1) / wR) : 0u;
            w.lg_nb = route == kRouteIntra ? (wR >= 4 ? 2 : (wR >= 2 ? 3 : 4)) : 1;
            const dim3 wg(grid_for(cn, hk::kWalkPairs, 1 << 30));
            const bool cl = m <= hk::kWalkCenterLds;
            w.glds = (out.G && m < hk::kWalkGLds) ? 1 : 0;
            const size_t wlds = hk::walk_lds_bytes(route == kRouteIntra ? WQ : 1, m, cl, w.glds != 0);
            if (route == kRouteIntra) {
                if (pk) {
                    if (cl) hipLaunchKernelGGL((hk::walk_kernel<false, true, true>), wg, dim3(256), wlds, st, w);
                    else hipLaunchKernelGGL((hk::walk_kernel<false, false, true>), wg, dim3(256), wlds, st, w);
                } else {
                    if (cl) hipLaunchKernelGGL((hk::walk_kernel<false, true, false>), wg, dim3(256), wlds, st, w);
                    else hipLaunchKernelGGL((hk::walk_kernel<false, false, false>), wg, dim3(256), wlds, st, w);
                }
            } else {
                if (cl) hipLaunchKernelGGL((hk::walk_kernel<true, true, false>), wg, dim3(256), wlds, st, w);
                else hipLaunchKernelGGL((hk::walk_kernel<true, false, false>), wg, dim3(256), wlds, st, w);
            }
            HCHK(hipGetLastError());
        }
        RCHK(record(ctx, (*tv)[2], st));
        hmark(ctx, "launch");
        if (ctx->progress && chunks.size() > 1 && !ctx->capturing) {
            // progress lines wait for each chunk; otherwise the host plans the
            // next chunk while this one runs
            HCHK(hipEventSynchronize((*tv)[2]));
            float f = 0, w2 = 0;
            HCHK(hipEventElapsedTime(&f, (*tv)[0], (*tv)[1]));
            HCHK(hipEventElapsedTime(&w2, (*tv)[1], (*tv)[2]));
            fprintf(stderr, "halign: chunk %d/%d done (%d pairs, forward %.1f ms, walk %.1f ms)\n", (int)ci + 1,
                    (int)chunks.size(), cn, f, w2);
            fflush(stderr);
        }
    }
    ctx->last_stats[1] += launches;
    return HALIGN_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for a bucket of (center length, batch size, median sequence
// length, traceback) it times the candidate plans on a strided sample of the
// batch (every plan gives bit-identical results) and keeps the fastest.
// ---------------------------------------------------------------------------
std::string tune_key(int m, int N, int mean_len, bool tb) {
    int lg = 0;
    while ((1 << (lg + 1)) <= N) ++lg;
    std::ostringstream o;
    o << "m" << (m + 31) / 32 << "_n" << lg << "_l" << (mean_len + 63) / 64 << "_t" << (tb ? 1 : 0);
    return o.str();
}

void tune_load(halign_ctx *ctx) {
    if (ctx->tune_file.empty()) return;
    std::ifstream f(ctx->tune_file);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream s(line);
        std::string key;
        int r = -1, R = -1, sm = -1, ls = 64, pk = 0;
        if (!(s >> key >> r >> R >> sm)) continue;              // malformed: ignored
        if (!(s >> ls)) ls = 64;                                // lines without the lane count
        if (!(s >> pk)) pk = 0;                                 // lines without the packed flag
        if (r < 0 || r > 1 || R < 0 || R > 16 || sm < 1 || sm > 4 || (ls != 64 && ls != 32 && ls != 16) || pk < 0 ||
            pk > 1)
            continue;
        ctx->tuned[key] = {r, R, sm, ls, pk};
    }
}

void tune_save(halign_ctx *ctx, const std::string &key, const std::array<int, 5> &v) {
    if (ctx->tune_file.empty()) return;
    std::ofstream f(ctx->tune_file, std::ios::app);
    if (f) f << key << " " << v[0] << " " << v[1] << " " << v[2] << " " << v[3] << " " << v[4] << "\n";
}

// *ran: whether candidate plans were run (the stage is then drained).
int autotune(halign_ctx *ctx, const Scoring &S, const uint8_t *center, int m, const halign_seqs *sq, bool tb,
             bool endc, const BatchOut &out, hipStream_t st, Tune *best, bool *ran) {
    *ran = false;
    const int N = sq->n;
    const int mean = N > 0 ? (int)((sq->offsets_host[N] - sq->offsets_host[0]) / N) : 0;
    auto apply = [&](const std::array<int, 5> &v) {
        best->route = v[0];
        best->R = v[1];
        best->smul = v[2];
        best->LS = v[3];
        best->pk = v[4];
    };
    const int64_t ik[4] = {m, N, mean, tb ? 1 : 0};
    if (std::equal(ik, ik + 4, ctx->tkey)) {   // same bucket as the last call: no string key
        apply(ctx->tval);
        return HALIGN_OK;
    }
    const std::string key = tune_key(m, N, mean, tb);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) {
        apply(it->second);
        std::copy(ik, ik + 4, ctx->tkey);
        ctx->tval = it->second;
        return HALIGN_OK;
    }
    *ran = true;
    // the batch itself (up to 4e10 cells: a few tens of ms per candidate), or a
    // strided sample of 65,536 pairs that keeps the length mix and, through the
    // stream count, the number of pairs per stream
    const double bcells = (double)m * (double)(sq->offsets_host[N] - sq->offsets_host[0]);
    const int ns = bcells <= 4e10 ? N : std::min(N, 65536);
    std::vector<int32_t> sample(ns);
    for (int q = 0; q < ns; ++q) sample[q] = (int32_t)((int64_t)q * N / ns);
    int R0 = 8, p0 = 1;
    pick_geom(m, &R0, &p0);
    const double scale = (double)ns / N;
    std::vector<Tune> cands;
    cands.push_back({kRouteIntra, R0, 1, scale, 64});
    cands.push_back({kRouteIntra, R0, 2, scale, 64});
    if (R0 < 8) cands.push_back({kRouteIntra, R0 + 1, 1, scale, 64});
    // narrower streams: fewer fill/drain steps, more rows per lane (int16 profile only;
    // run_batch falls back to 64 lanes otherwise)
    for (int ls : {32, 16}) {
        const int ps = std::max(1, (m + ls * 16 - 1) / (ls * 16));
        const int r = std::max(2, (m + ls * ps - 1) / (ls * ps));
        cands.push_back({kRouteIntra, r, 1, scale, ls});
        // the packed 16-bit kernel on the same geometry (run_batch falls back to
        // the 32-bit one where it does not apply)
        if (tb && endc) cands.push_back({kRouteIntra, r, 1, scale, ls, 1});
    }
    cands.push_back({kRouteInter, 0, 1, scale, 64});
    // the forward kernels are timed in the same traceback mode as the call
    float best_ms = 1e30f;
    *best = cands[0];
    for (const Tune &c : cands) {
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            // every candidate run starts the stage and the timing triples anew
            // (the previous run has synchronised)
            ctx->stage_off = ctx->plan_off = 0;
            ctx->ntev = 0;
            RCHK(run_batch(ctx, S, center, m, sq, sample.data(), (int)sample.size(), tb, endc, c.route, out, st, c));
            float wk = 0.f;
            RCHK(tev_sum(ctx, &ms, &wk));
            RCHK(stage_wait(ctx));
        }
        if (ms < best_ms) {
            best_ms = ms;
            *best = c;
        }
    }
    best->scale = 1;
    const std::array<int, 5> v = {best->route, best->R, best->smul, best->LS > 0 ? best->LS : 64, best->pk};
    ctx->tuned[key] = v;
    tune_save(ctx, key, v);
    std::copy(ik, ik + 4, ctx->tkey);
    ctx->tval = v;
    return HALIGN_OK;
}

// The first staging step of every call: starts the call's stage regions.
int upload_matrix(halign_ctx *ctx, const halign_scoring *sc, hipStream_t st, Scoring *S) {
    const size_t bytes = (size_t)sc->alphabet * sc->alphabet;
    RCHK(stage_begin(ctx));
    if (ctx->capturing) {   // the device copy from the uncaptured run is kept by the graph
        S->dmat = (const int8_t *)ctx->spbuf.p;
        S->hmat = sc->matrix_host;
        S->alpha = sc->alphabet;
        S->ge = sc->gap_extend;
        S->goe = sc->gap_open + sc->gap_extend;
        return HALIGN_OK;
    }
    RCHK(grow(ctx, ctx->spbuf, 4096));
    char *hs = nullptr;
    RCHK(stage_host(ctx, bytes, &hs));
    memcpy(hs, sc->matrix_host, bytes);
    HCHK(hipMemcpyAsync(ctx->spbuf.p, hs, bytes, hipMemcpyHostToDevice, st));
    RCHK(record(ctx, ctx->ev_stage, st));
    ctx->stage_pending = true;
    S->dmat = (const int8_t *)ctx->spbuf.p;
    S->hmat = sc->matrix_host;
    S->alpha = sc->alphabet;
    S->ge = sc->gap_extend;
    S->goe = sc->gap_open + sc->gap_extend;
    return HALIGN_OK;
}

// Every residue code must be below the alphabet size (HALIGN_E_INVALID).
// The check is enqueued without waiting: the kernels are memory-safe for any
// code (they mask codes to 5 bits), and the result lands in pinned host memory
// that validate_check() reads after the call's synchronisation point.
int validate_codes(halign_ctx *ctx, int alpha, const uint8_t *res, int64_t nres, const uint8_t *center, int m,
                   hipStream_t st) {
    RCHK(grow(ctx, ctx->counter, 256));
    uint32_t *flag = (uint32_t *)ctx->counter.p + 8;
    // the flag holds (call tag << 8 | largest code) and is raised with
    // atomicMax: a larger tag per call replaces the last call's value without
    // a clearing launch (cleared once when the 24-bit tag wraps).  A captured
    // graph clears the flag itself and uses tag 0 on every replay.
    uint32_t tag = 0;
    if (ctx->capturing) {
        RCHK(launch_fill(flag, 0u, 1, st));
    } else {
        // a buffer not yet cleared here (new, or swapped in) holds stale
        // bytes that would outrank or mimic a tag: clear it first
        if (ctx->vflag != flag || ctx->vtag + 1 >= (1u << 24)) {
            RCHK(launch_fill(flag, 0u, 1, st));
            ctx->vflag = flag;
            ctx->vtag = 0;
        }
        tag = ++ctx->vtag;
    }
    ctx->check_tag = tag;
    const int64_t n1 = nres > 0 ? nres : 0, n2 = (center && m > 0) ? m : 0;
    if (n1 + n2 > 0) {
        hipLaunchKernelGGL(hk::maxcode_kernel, dim3(grid_for((n1 + 15) / 16 + 1, 256, 1024)), dim3(256), 0, st, res, n1,
                           center, n2, tag << 8, flag);
        HCHK(hipGetLastError());
    }
    HCHK(hipMemcpyAsync(ctx->flag_host, flag, 4, hipMemcpyDeviceToHost, st));
    ctx->flag_alpha = alpha;
    return HALIGN_OK;
}

// Call after the stream has synchronised past validate_codes().
int validate_check(halign_ctx *ctx) {
    if (!ctx->flag_alpha) return HALIGN_OK;
    const uint32_t v = (uint32_t)*ctx->flag_host;
    const int h = (v >> 8) == ctx->check_tag ? (int)(v & 0xffu) : 0, alpha = ctx->flag_alpha;
    ctx->flag_alpha = 0;
    if (h >= alpha) return fail(HALIGN_E_INVALID, "residue code %d >= alphabet %d", h, alpha);
    return HALIGN_OK;
}

int validate_now(halign_ctx *ctx, int alpha, const uint8_t *res, int64_t nres, const uint8_t *center, int m,
                 hipStream_t st) {
    RCHK(validate_codes(ctx, alpha, res, nres, center, m, st));
    HCHK(hipStreamSynchronize(st));
    return validate_check(ctx);
}

int route_of(uint32_t flags, int m, int N) {
    const uint32_t r = flags & (3u << 4);
    if (r == HALIGN_ROUTE_INTER) return kRouteInter;
    if (r == HALIGN_ROUTE_INTRA) return kRouteIntra;
    (void)m;
    if (const char *e = getenv("HALIGN_ROUTE")) {
        if (!strcmp(e, "intra")) return kRouteIntra;
        if (!strcmp(e, "inter")) return kRouteInter;
    }
    // enough independent lanes for the chip: 4 waves per SIMD in inter form
    return (N >= 64 * 4 * 1024) ? kRouteInter : kRouteIntra;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *halign_last_error(void) { return g_err; }

int halign_ctx_create(int device, size_t workspace_cap_bytes, halign_ctx **out) {
    if (!out) return fail(HALIGN_E_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(HALIGN_E_INVALID, "device %d of %d", device, ndev);
    HCHK(hipSetDevice(device));
    halign_ctx *ctx = new (std::nothrow) halign_ctx();
    if (!ctx) return fail(HALIGN_E_NOMEM, "host allocation failed");
    ctx->device = device;
    ctx->cap = workspace_cap_bytes;
    if (ctx->cap == 0) {   // default: a quarter of the memory free at creation
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr > 0) ctx->cap = fr / 4;
    }
    if (const char *e = getenv("HALIGN_AUTOTUNE")) ctx->autotune = atoi(e) != 0;
    if (const char *e = getenv("HALIGN_PROGRESS")) ctx->progress = atoi(e) != 0;
    if (const char *e = getenv("HALIGN_HOST_TIMING")) ctx->host_timing = atoi(e) != 0;
    if (const char *e = getenv("HALIGN_TUNE_CACHE")) ctx->tune_file = e;
    tune_load(ctx);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->num_cu = prop.multiProcessorCount;
        ctx->lds_max = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                             : prop.sharedMemPerBlock;
        if (prop.sharedMemPerBlock && prop.sharedMemPerBlock < ctx->lds_max) ctx->lds_max = prop.sharedMemPerBlock;
        // row emission of long centers takes up to the CU's LDS in one workgroup
        const size_t cu = prop.maxSharedMemoryPerMultiProcessor;
        if (cu > ctx->lds_max &&
            hipFuncSetAttribute((const void *)hk::rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cu) ==
                hipSuccess)
            ctx->lds_cu = cu;
        else
            ctx->lds_cu = ctx->lds_max;
        (void)hipGetLastError();
    }
    if (hipHostMalloc((void **)&ctx->flag_host, 64, hipHostMallocDefault) != hipSuccess) {
        halign_ctx_destroy(ctx);
        return fail(HALIGN_E_DEVICE, "pinned allocation");
    }
    // the width mailbox; without it the width comes back by a copy and a
    // stream synchronisation
    if (hipHostMalloc((void **)&ctx->mail_host, 64, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
        ctx->mail_host[0] = ctx->mail_host[1] = 0;
        if (hipHostGetDevicePointer((void **)&ctx->mail_dev, ctx->mail_host, 0) != hipSuccess) ctx->mail_dev = nullptr;
    } else {
        ctx->mail_host = nullptr;
        (void)hipGetLastError();
    }
    if (hipEventCreateWithFlags(&ctx->ev_stage, hipEventDisableTiming) != hipSuccess) {
        halign_ctx_destroy(ctx);
        return fail(HALIGN_E_DEVICE, "event create");
    }
    *out = ctx;
    return HALIGN_OK;
}

void halign_ctx_destroy(halign_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    graph_drop(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
    for (DevBuf *b : {&ctx->codes, &ctx->bound, &ctx->plan, &ctx->counter, &ctx->pairbuf, &ctx->msabuf, &ctx->spbuf,
                      &ctx->sbuf, &ctx->nuctab, &ctx->nucscr, &ctx->nucdp, &ctx->rowck,
                      &ctx->njrows, &ctx->njD, &ctx->njS, &ctx->njacc, &ctx->njB})
        if (b->p) (void)hipFree(b->p);
    for (DevBuf &b : ctx->mlp)
        if (b.p) (void)hipFree(b.p);
    if (ctx->stage.p) (void)hipHostFree(ctx->stage.p);
    if (ctx->flag_host) (void)hipHostFree(ctx->flag_host);
    if (ctx->mail_host) (void)hipHostFree(ctx->mail_host);
    for (auto &t : ctx->tev)
        for (auto &e : t) (void)hipEventDestroy(e);
    if (ctx->ev_stage) (void)hipEventDestroy(ctx->ev_stage);
    delete ctx;
}

int halign_ctx_workspace_bytes(const halign_ctx *ctx, size_t *bytes_host) {
    if (!ctx || !bytes_host) return fail(HALIGN_E_INVALID, "NULL argument");
    *bytes_host = ctx->codes.cap + ctx->bound.cap + ctx->plan.cap + ctx->pairbuf.cap + ctx->msabuf.cap;
    return HALIGN_OK;
}

int halign_ctx_last_timings(halign_ctx *ctx, float *ms_host) {
    if (!ctx || !ms_host) return fail(HALIGN_E_INVALID, "NULL argument");
    RCHK(tev_sum(ctx, &ms_host[0], &ms_host[1]));
    ms_host[2] = ms_host[0] + ms_host[1];
    return HALIGN_OK;
}

int halign_ctx_last_stats(const halign_ctx *ctx, int64_t *stats_host) {
    if (!ctx || !stats_host) return fail(HALIGN_E_INVALID, "NULL argument");
    for (int i = 0; i < 4; ++i) stats_host[i] = ctx->last_stats[i];
    return HALIGN_OK;
}

int halign_ctx_set_graph(halign_ctx *ctx, int enable) {
    if (!ctx) return fail(HALIGN_E_INVALID, "NULL ctx");
    ctx->use_graph = enable != 0;
    if (!enable) graph_drop(ctx);
    return HALIGN_OK;
}

int halign_ctx_graph_launches(const halign_ctx *ctx, int64_t *n_host) {
    if (!ctx || !n_host) return fail(HALIGN_E_INVALID, "NULL argument");
    *n_host = ctx->graph_launches;
    return HALIGN_OK;
}

int halign_ctx_set_prejudge(halign_ctx *ctx, int candidates, int partners) {
    if (!ctx || candidates < 0 || candidates > 256 || partners < 0) return fail(HALIGN_E_INVALID, "bad arguments");
    ctx->prejudge_cand = candidates;
    ctx->prejudge_part = partners;
    return HALIGN_OK;
}

int halign_ctx_set_autotune(halign_ctx *ctx, int enable) {
    if (!ctx) return fail(HALIGN_E_INVALID, "NULL ctx");
    ctx->autotune = enable != 0;
    return HALIGN_OK;
}

int halign_ctx_last_plan(const halign_ctx *ctx, int32_t *plan_host) {
    if (!ctx || !plan_host) return fail(HALIGN_E_INVALID, "NULL argument");
    for (int i = 0; i < 5; ++i) plan_host[i] = ctx->last_tune[i];
    return HALIGN_OK;
}

// Failure injection (declared in halign.h): chunk `c` of the next
// halign_sw_batch fails before its launch.
int halign_debug_fail_chunk(halign_ctx *ctx, int c) {
    if (!ctx) return fail(HALIGN_E_INVALID, "NULL ctx");
    ctx->fault_chunk = c;
    return HALIGN_OK;
}

int halign_encode(const uint8_t *ascii, int64_t len, uint8_t *codes, void *stream) {
    static const char kAlpha[] = "ARNDCQEGHILKMFPSTWYVBZX*";
    if (len < 0 || (len > 0 && (!ascii || !codes))) return fail(HALIGN_E_INVALID, "bad arguments");
    if (len == 0) return HALIGN_OK;
    static uint8_t *dtab = nullptr;
    static int dtab_dev = -1;
    int dev = 0;
    HCHK(hipGetDevice(&dev));
    if (!dtab || dtab_dev != dev) {
        uint8_t tab[256];
        for (int x = 0; x < 256; ++x) tab[x] = 22;  // X
        for (int x = 0; x < 24; ++x) {
            tab[(uint8_t)kAlpha[x]] = (uint8_t)x;
            if (kAlpha[x] >= 'A' && kAlpha[x] <= 'Z') tab[(uint8_t)(kAlpha[x] - 'A' + 'a')] = (uint8_t)x;
        }
        tab['U'] = tab['u'] = 4;   // C
        tab['O'] = tab['o'] = 11;  // K
        uint8_t *p = nullptr;
        HCHK(hipMalloc(&p, 256));
        HCHK(hipMemcpy(p, tab, 256, hipMemcpyHostToDevice));
        dtab = p;
        dtab_dev = dev;
    }
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(hk::encode_kernel, dim3(grid_for(len, 256, 8192)), dim3(256), 0, st, ascii, len, codes,
                       (const uint8_t *)dtab);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

}  // extern "C"

// The launch sequence of halign_sw_batch (validation, plan, forward, walk).
static int sw_batch_body(halign_ctx *ctx, const halign_scoring *sc, const uint8_t *center, int32_t m,
                          const halign_seqs *seqs, uint32_t flags, int32_t *score, int32_t *cells, uint16_t *ins,
                          uint32_t *aligned, void *stream, int32_t *G = nullptr, int gskip = -1,
                          bool checked = false) {
    if (!ctx) return fail(HALIGN_E_INVALID, "ctx is NULL");
    if (!checked) {   // halign_msa has checked both already
        RCHK(check_scoring(sc));
        RCHK(check_seqs(seqs));
    }
    if (m <= 0 || !center) return fail(HALIGN_E_INVALID, "empty center");
    if (m >= 65536) return fail(HALIGN_E_UNSUPPORTED, "center length %d >= 65536", m);
    if (!score && seqs->n > 0) return fail(HALIGN_E_INVALID, "score is NULL");
    const bool tb = (flags & HALIGN_TRACEBACK) != 0;
    if (tb && (!cells || !ins || !aligned)) return fail(HALIGN_E_INVALID, "traceback needs cells, ins, aligned");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int N = seqs->n;
    if (N == 0) return HALIGN_OK;
    Scoring S;
    RCHK(upload_matrix(ctx, sc, st, &S));
    // endcells: needed by the walk, or to fill cells in score-only mode
    const bool endc = tb || cells != nullptr;
    RCHK(grow(ctx, ctx->pairbuf, (size_t)N * 8 + 256));
    int32_t *endcell = (int32_t *)ctx->pairbuf.p;
    hmark(ctx, "upload");
    Tune tune;
    const bool want_tune = ctx->autotune && (flags & (3u << 4)) == HALIGN_ROUTE_AUTO;
    if (want_tune) {
        BatchOut tout{score, cells, endcell, ins, aligned};
        bool ran = false;
        RCHK(autotune(ctx, S, center, m, seqs, tb, endc, tout, st, &tune, &ran));
        if (ran) RCHK(stage_begin(ctx));   // the tuner's runs have synchronised
    }
    for (auto &v : ctx->last_stats) v = 0;
    hmark(ctx, "tune");
    // the code check and the zeroing of the outputs go in before the host
    // plans the batch, so these small kernels run while the host works (the
    // forward kernels read codes masked to 5 bits, the check is read after the
    // batch, and the outputs are first written by the walk)
    auto prep = [&]() -> int {
        if (tb) {
            // ins (as 32-bit words; an odd trailing uint16 on its own), aligned
            // and G zeroed in one launch
            hk::ZeroArgs z{};
            const int64_t nins = (int64_t)N * (m + 1);
            z.p[0] = reinterpret_cast<uint32_t *>(ins);
            z.n[0] = nins / 2;
            z.p[1] = aligned;
            z.n[1] = (int64_t)N * ((m + 31) / 32);
            z.p[2] = reinterpret_cast<uint32_t *>(G);
            z.n[2] = G ? (int64_t)m + 1 : 0;
            z.tail16 = (nins & 1) ? ins + (nins - 1) : nullptr;
            hipLaunchKernelGGL(hk::zero_kernel, dim3(grid_for(z.n[0] + z.n[1], 256, 4096)), dim3(256), 0, st, z);
            HCHK(hipGetLastError());
        }
        RCHK(validate_codes(ctx, sc->alphabet, seqs->residues, seqs->offsets_host[N], center, m, st));
        return HALIGN_OK;
    };
    BatchOut out{score, cells, endcell, ins, aligned};
    if (tb && G) {
        out.G = G;
        out.gskip = gskip;
    }
    RCHK(prep());
    hmark(ctx, "prep");
    // Routing by pair length: when the batch as a whole runs one pair per lane
    // (the route the caller did not force), pairs longer than kLongPair
    // residues run on the wavefront kernel, one pair per stream, in a launch
    // of their own; the rest keep the strip kernel.  Both write the same
    // outputs, each at its own pair ids.
    const int route = tune.route >= 0 ? tune.route : route_of(flags, m, N);
    const int64_t *oh = seqs->offsets_host;
    const bool split = route == kRouteInter && (flags & (3u << 4)) == HALIGN_ROUTE_AUTO;
    int nlong = 0;
    if (split)
        for (int k = 0; k < N; ++k) nlong += oh[k + 1] - oh[k] > kLongPair;
    if (nlong == 0) {
        RCHK(run_batch(ctx, S, center, m, seqs, nullptr, N, tb, endc, route, out, st, tune));
    } else {
        // long pairs first in the id list, then the rest
        std::vector<int32_t> &ids = ctx->h_split;
        ids.resize(N);
        int a = 0, b = nlong;
        for (int k = 0; k < N; ++k) ids[oh[k + 1] - oh[k] > kLongPair ? a++ : b++] = k;
        RCHK(run_batch(ctx, S, center, m, seqs, ids.data(), nlong, tb, endc, kRouteIntra, out, st));
        RCHK(run_batch(ctx, S, center, m, seqs, ids.data() + nlong, N - nlong, tb, endc, route, out, st, tune));
    }
    ctx->last_tune = {tune.route, tune.R, tune.smul, tune.LS > 0 ? tune.LS : 64, ctx->last_pk};
    if (!tb && cells) {
        // score-only with cells: report the end cell as (0, 0, i1, j1)
        hipLaunchKernelGGL(hk::endcell_to_cells_kernel, dim3(grid_for(N, 256)), dim3(256), 0, st,
                           (const int32_t *)endcell, N, cells);
        HCHK(hipGetLastError());
    }
    return HALIGN_OK;
}

namespace {

// FNV-1a over 8-byte words (then the tail bytes)
uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const uint8_t *b = (const uint8_t *)p;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        memcpy(&w, b + i, 8);
        h ^= w;
        h *= 0x100000001b3ull;
        h ^= h >> 29;
    }
    for (; i < n; ++i) { h ^= b[i]; h *= 0x100000001b3ull; }
    return h;
}

}  // namespace

// halign_sw_batch without the final synchronisation: the code check is left
// pending for the caller's next synchronisation point (validate_check).
// With HALIGN_GRAPH the launch sequence is captured once into a hipGraph that
// owns its scratch and plan buffers, and replayed while the call's arguments
// (pointers, sizes, offsets, scoring) stay the same.
static int sw_batch_async(halign_ctx *ctx, const halign_scoring *sc, const uint8_t *center, int32_t m,
                          const halign_seqs *seqs, uint32_t flags, int32_t *score, int32_t *cells, uint16_t *ins,
                          uint32_t *aligned, void *stream, int32_t *G = nullptr, int gskip = -1,
                          bool checked = false) {
    if (!(flags & HALIGN_GRAPH))
        return sw_batch_body(ctx, sc, center, m, seqs, flags, score, cells, ins, aligned, stream, G, gskip, checked);
    if (!ctx || !sc || !seqs || !sc->matrix_host || !seqs->offsets_host)
        return sw_batch_body(ctx, sc, center, m, seqs, flags, score, cells, ins, aligned, stream, G, gskip);
    hipStream_t st = (hipStream_t)stream;
    uint64_t key = 0xcbf29ce484222325ull;
    const void *ptrs[8] = {center, seqs->residues, seqs->offsets, score, cells, ins, aligned, G};
    key = fnv(key, ptrs, sizeof ptrs);
    const int32_t ints[8] = {m, seqs->n, (int32_t)flags, sc->alphabet, sc->gap_open, sc->gap_extend, ctx->autotune,
                             gskip};
    key = fnv(key, ints, sizeof ints);
    if (sc->alphabet > 0 && sc->alphabet <= 32)
        key = fnv(key, sc->matrix_host, (size_t)sc->alphabet * sc->alphabet);
    if (seqs->n >= 0) key = fnv(key, seqs->offsets_host, sizeof(int64_t) * ((size_t)seqs->n + 1));
    if (ctx->gent.exec && ctx->gent.key == key) {
        HCHK(hipSetDevice(ctx->device));
        RCHK(stage_begin(ctx));
        std::array<hipEvent_t, 3> *tv = nullptr;
        RCHK(tev_next(ctx, &tv));
        RCHK(record(ctx, (*tv)[0], st));
        HCHK(hipGraphLaunch(ctx->gent.exec, st));
        RCHK(record(ctx, (*tv)[1], st));
        RCHK(record(ctx, (*tv)[2], st));
        ctx->flag_alpha = sc->alphabet;   // the graph copies the code check into flag_host
        ctx->check_tag = 0;               // with tag 0
        ctx->graph_launches++;
        return HALIGN_OK;
    }
    // first call: run it, then capture the same sequence for later calls
    RCHK(sw_batch_body(ctx, sc, center, m, seqs, flags, score, cells, ins, aligned, stream, G, gskip));
    // the captured run writes its plans into the stage from its start again:
    // the copies of the run above must have read it first
    RCHK(stage_wait(ctx));
    const int pending = ctx->flag_alpha;
    const uint32_t pending_tag = ctx->check_tag;
    graph_drop(ctx);
    if (!ctx->cap_stream) HCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
    ctx->capturing = true;
    const int rc = sw_batch_body(ctx, sc, center, m, seqs, flags, score, cells, ins, aligned, ctx->cap_stream, G,
                                 gskip);
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
    ctx->flag_alpha = pending;
    ctx->check_tag = pending_tag;
    if (rc != HALIGN_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ec != hipSuccess) return fail(HALIGN_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(HALIGN_E_DEVICE, "graph instantiation failed");
    }
    // the graph keeps the buffers it references; the ctx gets fresh ones later
    auto &e = ctx->gent;
    e.key = key;
    e.graph = g;
    e.exec = ex;
    std::swap(e.plan, ctx->plan);
    std::swap(e.codes, ctx->codes);
    std::swap(e.sbuf, ctx->sbuf);
    std::swap(e.bound, ctx->bound);
    std::swap(e.counter, ctx->counter);
    std::swap(e.pairbuf, ctx->pairbuf);
    std::swap(e.spbuf, ctx->spbuf);
    std::swap(e.stage, ctx->stage);
    ctx->stage_pending = false;
    return HALIGN_OK;
}

extern "C" {

int halign_sw_batch(halign_ctx *ctx, const halign_scoring *sc, const uint8_t *center, int32_t m,
                    const halign_seqs *seqs, uint32_t flags, int32_t *score, int32_t *cells, uint16_t *ins,
                    uint32_t *aligned, void *stream) {
    RCHK(sw_batch_async(ctx, sc, center, m, seqs, flags, score, cells, ins, aligned, stream));
    if (ctx->flag_alpha) {
        HCHK(hipStreamSynchronize((hipStream_t)stream));
        RCHK(validate_check(ctx));
    }
    return HALIGN_OK;
}

}  // extern "C"

// col[p] = sum_{q<p} (G[q] + 1) and the MSA width (copied to the host and
// synchronised when width_host is given).
static int merge_offsets(halign_ctx *ctx, const int32_t *G, int m1, int64_t *col, int64_t *width_host,
                         hipStream_t st) {
    RCHK(grow(ctx, ctx->spbuf, 4096));
    int64_t *dwidth = (int64_t *)((char *)ctx->spbuf.p + 2048);
    const bool mail = width_host && ctx->mail_dev && !ctx->capturing;
    const int64_t seq = mail ? ++ctx->mail_seq : 0;
    hipLaunchKernelGGL(hk::merge_scan_kernel, dim3(1), dim3(1024), 0, st, G, m1, col, dwidth,
                       mail ? ctx->mail_dev : nullptr, seq);
    HCHK(hipGetLastError());
    if (mail) {
        // spin on the mailbox (the kernel's release store of seq follows the
        // width); now and then ask the stream whether it failed or finished
        volatile int64_t *mb = ctx->mail_host;
        for (uint64_t it = 1;; ++it) {
            if (mb[1] == seq) break;
            if ((it & 4095) == 0) {
                const hipError_t q = hipStreamQuery(st);
                if (q == hipSuccess) {
                    if (mb[1] == seq) break;
                    return fail(HALIGN_E_DEVICE, "merge scan finished without its width");
                }
                if (q != hipErrorNotReady) return fail(HALIGN_E_DEVICE, "%s", hipGetErrorString(q));
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        *width_host = mb[0];
    } else if (width_host) {
        HCHK(hipMemcpyAsync(width_host, dwidth, 8, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
    }
    return HALIGN_OK;
}

extern "C" {

int halign_merge(halign_ctx *ctx, const uint16_t *ins, int32_t n, int32_t m, int32_t *G, int64_t *col,
                 int64_t *width_host, void *stream) {
    if (!ctx || !G || !col || m < 0 || n < 0 || (n > 0 && !ins)) return fail(HALIGN_E_INVALID, "bad arguments");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int m1 = m + 1;
    RCHK(launch_fill((uint32_t *)G, 0u, m1, st));
    if (n > 0) {
        dim3 grid((m1 + 255) / 256, (n + hk::kMergeRows - 1) / hk::kMergeRows);
        if (grid.y > 65535) {
            // fold rows: launch in slices of 65535 * kMergeRows rows
            for (int64_t r0 = 0; r0 < n; r0 += (int64_t)65535 * hk::kMergeRows) {
                const int rn = (int)std::min<int64_t>(n - r0, (int64_t)65535 * hk::kMergeRows);
                dim3 g2((m1 + 255) / 256, (rn + hk::kMergeRows - 1) / hk::kMergeRows);
                hipLaunchKernelGGL(hk::merge_max_kernel, g2, dim3(256), 0, st, ins + r0 * m1, rn, m1, G);
            }
        } else {
            hipLaunchKernelGGL(hk::merge_max_kernel, grid, dim3(256), 0, st, ins, n, m1, G);
        }
        HCHK(hipGetLastError());
    }
    return merge_offsets(ctx, G, m1, col, width_host, st);
}

int halign_emit_rows(halign_ctx *ctx, const halign_seqs *seqs, int32_t m, const uint16_t *ins,
                     const uint32_t *aligned, const int32_t *G, const int64_t *col, int64_t width, uint8_t *msa,
                     void *stream) {
    if (!ctx || !seqs || m < 0 || width < m || (seqs->n > 0 && (!ins || !aligned || !G || !col || !msa)))
        return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_seqs(seqs));
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int N = seqs->n;
    if (N == 0 || width == 0) return HALIGN_OK;
    const int m1 = m + 1, aw = (m + 31) / 32;
    // long centers: tasks of (row, 256 blocks) after a per-row count pass
    // (HALIGN_ROWS=chunk|lds picks a kernel for any center)
    bool chunk_rows = m1 > hk::kRowsChunkMinBlocks;
    if (const char *e = getenv("HALIGN_ROWS")) {
        if (!strcmp(e, "chunk")) chunk_rows = true;
        if (!strcmp(e, "lds")) chunk_rows = false;
    }
    if (chunk_rows) {
        const int nck = (m1 + hk::kRowChunk - 1) / hk::kRowChunk;
        RCHK(grow(ctx, ctx->rowck, 4 * (size_t)N * nck));
        int32_t *ck = (int32_t *)ctx->rowck.p;
        hk::RowsArgs ra{seqs->residues, seqs->offsets, N, m, ins, aligned, aw, G, col, width, 0, 0, 0, msa};
        const int cgrid = std::max(1, std::min((N + 3) / 4, ctx->num_cu * 8));
        hipLaunchKernelGGL(hk::rows_count_kernel, dim3(cgrid), dim3(256), 0, st, ra, ck, nck);
        HCHK(hipGetLastError());
        const int64_t ntask = (int64_t)N * nck;
        const int egrid = (int)std::max<int64_t>(1, std::min<int64_t>((ntask + 3) / 4, (int64_t)ctx->num_cu * 8));
        hipLaunchKernelGGL(hk::rows_chunk_kernel, dim3(egrid), dim3(256), 4 * hk::kRowWave, st, ra,
                           (const int32_t *)ck, nck);
        HCHK(hipGetLastError());
        return HALIGN_OK;
    }
    // LDS per wavefront: (m+1) block starts and counts, the aligned bits and
    // a chunk of ch columns
    size_t lim = std::min<size_t>(ctx->lds_max, 64 * 1024);
    auto wave_bytes = [&](int ch) {
        const size_t h2 = ((size_t)m1 * 2 + 3) & ~(size_t)3;
        const size_t head = (2 * h2 + 4 * (size_t)aw + 15) & ~(size_t)15;
        return head + (size_t)ch + 32;
    };
    int ch = (int)std::min<int64_t>(8192, (width + 15) & ~(int64_t)15), wpb = hk::kWaveRows;
    while (ch > 1024 && (size_t)wpb * wave_bytes(ch) > lim) ch = ((ch / 2) + 15) & ~15;
    while (wpb > 1 && (size_t)wpb * wave_bytes(ch) > lim) --wpb;
    if ((size_t)wpb * wave_bytes(ch) > lim && wave_bytes(ch) <= ctx->lds_cu) lim = ctx->lds_cu;   // long centers
    if ((size_t)wpb * wave_bytes(ch) > lim) return fail(HALIGN_E_UNSUPPORTED, "center length %d too long for row emission", m);
    if (width >= ((int64_t)1 << 31)) return fail(HALIGN_E_UNSUPPORTED, "MSA width %lld", (long long)width);
    const size_t gcb = 4 * (size_t)(m1 + 1);
    if ((size_t)wpb * wave_bytes(ch) + gcb > lim && (size_t)wpb * wave_bytes(ch) + gcb <= ctx->lds_cu)
        lim = ctx->lds_cu;   // the column table in LDS too
    const int gc_lds = (size_t)wpb * wave_bytes(ch) + gcb <= lim ? 1 : 0;
    hk::RowsArgs ra{seqs->residues, seqs->offsets, N, m, ins, aligned, aw, G, col, width, ch, (int)wave_bytes(ch),
                    gc_lds, msa};
    const size_t lds = (size_t)wpb * wave_bytes(ch) + (gc_lds ? gcb : 0);
    const int per_cu = std::max(1, std::min(8, (int)(ctx->lds_max / lds)));
    const int grid = std::max(1, std::min((N + wpb - 1) / wpb, ctx->num_cu * per_cu));
    hipLaunchKernelGGL(hk::rows_kernel, dim3(grid), dim3(64 * wpb), lds, st, ra);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

// Center selection -----------------------------------------------------------
// The packed 16-bit score-only strip kernel applies when every H stays below
// 15000: max S times the longest sequence (plus go + ge) stays below 15000,
// and go + ge <= 256.
// HALIGN_STRIP32=1 keeps the 32-bit kernel (tests of both paths).
static bool strip16_ok(const Scoring &S, const halign_seqs *sq) {
    const char *e = getenv("HALIGN_STRIP32");
    if (e && atoi(e) != 0) return false;
    int smax = 0;
    for (int x = 0; x < S.alpha * S.alpha; ++x) smax = std::max(smax, (int)S.hmat[x]);
    int64_t lmax = 0;
    for (int k = 0; k < sq->n; ++k) lmax = std::max(lmax, sq->offsets_host[k + 1] - sq->offsets_host[k]);
    return S.goe <= 256 && S.ge <= 256 && (int64_t)smax * lmax + S.goe < 15000;
}

// Groups: one center, 64 partners (32-bit kernel) or 128 (16-bit kernel).
// Mode 1 (all pairs a < b of `perm`, in length order): the groups follow the
// closed-form triangular tiling of tiling.hpp, ngroups = tri_groups(N, step),
// with no per-group arrays.  Mode 2 (anchored groups): gcen, gb0 and gslot
// list the groups.
constexpr int64_t kGroupSlice = (int64_t)1 << 21;   // all-pairs groups per launch

static int run_groups(halign_ctx *ctx, const Scoring &S, const halign_seqs *sq, int mode, int64_t ngroups,
                      const std::vector<int32_t> &gcen, const std::vector<int32_t> &gb0,
                      const std::vector<int32_t> &perm, const std::vector<int32_t> &gslot, int64_t *sums,
                      int32_t *score, hipStream_t st, int nperm = -1, bool p16 = false) {
    if (p16 && (score || mode == 0)) return fail(HALIGN_E_INVALID, "16-bit strip kernel: score-only center selection");
    if (ngroups <= 0) return HALIGN_OK;
    const size_t ng2 = mode == 2 ? (size_t)ngroups : 1;
    PlanBuilder pb;
    const size_t o_gcen = pb.add(4 * ng2), o_gb0 = pb.add(4 * ng2), o_perm = pb.add(4 * perm.size()),
                 o_gslot = pb.add(4 * ng2);
    char *hs = nullptr;
    RCHK(stage_host(ctx, pb.total, &hs));
    if (mode == 2) {
        memcpy(hs + o_gcen, gcen.data(), 4 * ng2);
        memcpy(hs + o_gb0, gb0.data(), 4 * ng2);
        memcpy(hs + o_gslot, gslot.data(), 4 * ng2);
    }
    memcpy(hs + o_perm, perm.data(), 4 * perm.size());
    char *dplan = nullptr;
    RCHK(plan_dev(ctx, pb.total, st, &dplan));
    HCHK(hipMemcpyAsync(dplan, hs, pb.total, hipMemcpyHostToDevice, st));
    RCHK(record(ctx, ctx->ev_stage, st));
    ctx->stage_pending = true;
    int nmax_all = 0;
    const int64_t *oh = sq->offsets_host;
    for (int k = 0; k < sq->n; ++k) nmax_all = std::max(nmax_all, (int)(oh[k + 1] - oh[k]));
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ngroups, (int64_t)ctx->num_cu * 16));
    RCHK(grow(ctx, ctx->bound, (size_t)grid * 64 * strip_cols(nmax_all) * (p16 ? 16 : 8)));
    RCHK(grow(ctx, ctx->counter, 256));
    RCHK(launch_fill((uint32_t *)ctx->counter.p, 0u, 2, st));
    hk::InterArgs a{};
    a.mat = S.dmat;
    a.alpha = S.alpha;
    a.res = sq->residues;
    a.off = sq->offsets;
    a.mode = mode;
    a.gcen = (const int32_t *)(dplan + o_gcen);
    a.gb0 = (const int32_t *)(dplan + o_gb0);
    a.perm = (const int32_t *)(dplan + o_perm);
    a.nseq = nperm >= 0 ? nperm : sq->n;
    a.gslot = (const int32_t *)(dplan + o_gslot);
    a.sums = sums;
    a.ngroups = ngroups;
    a.ge = S.ge;
    a.goe = S.goe;
    a.counter = (unsigned long long *)ctx->counter.p;
    a.score = score;
    a.bound = (int2 *)ctx->bound.p;
    a.bstride = (int64_t)64 * strip_cols(nmax_all);
    ctx->last_stats[0] = 0;
    std::array<hipEvent_t, 3> *tv = nullptr;
    RCHK(tev_next(ctx, &tv));
    RCHK(record(ctx, (*tv)[0], st));
    // all pairs run in launches of at most kGroupSlice groups (a few seconds
    // each at the largest sets), so that no single kernel runs for minutes
    int64_t slice = mode == 1 ? kGroupSlice : ngroups;
    if (const char *e = getenv("HALIGN_GROUP_SLICE"))   // test knob: many small launches
        if (mode == 1 && atoll(e) > 0) slice = atoll(e);
    a.gtotal = ngroups;
    for (int64_t g0 = 0; g0 < ngroups; g0 += slice) {
        a.gfirst = g0;
        a.ngroups = std::min(slice, ngroups - g0);
        if (g0 > 0) RCHK(launch_fill((uint32_t *)ctx->counter.p, 0u, 2, st));
        if (p16) hipLaunchKernelGGL(hk::sw_inter16_kernel, dim3(grid), dim3(64), 0, st, a);
        else launch_inter(a, false, false, grid, st);
        HCHK(hipGetLastError());
        if (ctx->progress && ngroups > slice && !ctx->capturing) {
            HCHK(hipStreamSynchronize(st));
            fprintf(stderr, "halign: all-pairs groups %lld / %lld\n", (long long)(g0 + a.ngroups), (long long)ngroups);
        }
    }
    RCHK(record(ctx, (*tv)[1], st));
    RCHK(record(ctx, (*tv)[2], st));
    return HALIGN_OK;
}

static std::vector<int32_t> length_perm(const halign_seqs *sq) {
    std::vector<int32_t> perm(sq->n);
    std::iota(perm.begin(), perm.end(), 0);
    const int64_t *oh = sq->offsets_host;
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int32_t x, int32_t y) { return (oh[x + 1] - oh[x]) < (oh[y + 1] - oh[y]); });
    return perm;
}

static int argmax_sums(halign_ctx *ctx, const int64_t *sums, const int32_t *cand_host, int ncand, int32_t *center_host,
                       hipStream_t st) {
    std::vector<int64_t> h(ncand);
    HCHK(hipMemcpyAsync(h.data(), sums, 8 * (size_t)ncand, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    int best = 0;
    for (int q = 1; q < ncand; ++q) {
        const int cq = cand_host ? cand_host[q] : q, cb = cand_host ? cand_host[best] : best;
        if (h[q] > h[best] || (h[q] == h[best] && cq < cb)) best = q;
    }
    *center_host = cand_host ? cand_host[best] : best;
    (void)ctx;
    return HALIGN_OK;
}

int halign_exact_tiling(int64_t n, int32_t step, int64_t g, int64_t *ngroups_host, int64_t *center_pos_host,
                        int64_t *partner0_host) {
    if (n < 0 || step < 1 || !ngroups_host) return fail(HALIGN_E_INVALID, "bad arguments");
    const int64_t ng = hk::tri_groups(n, step);
    *ngroups_host = ng;
    if (g < 0) return HALIGN_OK;
    if (g >= ng || !center_pos_host || !partner0_host) return fail(HALIGN_E_INVALID, "group %lld of %lld", (long long)g, (long long)ng);
    hk::tri_group(g, n, step, center_pos_host, partner0_host);
    return HALIGN_OK;
}

int halign_center_exact(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, int64_t *sums,
                        int32_t *center_host, void *stream) {
    if (!ctx || !sums) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    const int N = seqs->n;
    if (N <= 0) return fail(HALIGN_E_INVALID, "empty set");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    Scoring S;
    RCHK(upload_matrix(ctx, sc, st, &S));
    RCHK(validate_now(ctx, sc->alphabet, seqs->residues, seqs->offsets_host[N], nullptr, 0, st));
    RCHK(launch_fill((uint32_t *)sums, 0u, 2 * (int64_t)N, st));
    // all pairs a' < b' in length order: the longer sequence is the lane's,
    // the shorter one the group's center; the groups are numbered in closed
    // form (tiling.hpp), so the host holds O(N) plan data
    std::vector<int32_t> perm = length_perm(seqs), none;
    const bool p16 = strip16_ok(S, seqs);
    const int step = p16 ? 128 : 64;
    RCHK(run_groups(ctx, S, seqs, 1, hk::tri_groups(N, step), none, none, perm, none, sums, nullptr, st, -1, p16));
    if (center_host) RCHK(argmax_sums(ctx, sums, nullptr, N, center_host, st));
    return HALIGN_OK;
}

}  // extern "C"

// Sums of scores of candidates hc[q] against a partner list (NULL: every
// sequence), center = the candidate with the largest sum, ties to the lower
// sequence index.
static int judge_impl(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                      const std::vector<int32_t> &hc, const int32_t *partners_host, int32_t npart, int64_t *sums,
                      int32_t *center_host, hipStream_t st) {
    const int N = seqs->n;
    const int ncand = (int)hc.size();
    for (int q = 0; q < ncand; ++q)
        if (hc[q] < 0 || hc[q] >= N) return fail(HALIGN_E_INVALID, "candidate %d out of range", hc[q]);
    Scoring S;
    RCHK(upload_matrix(ctx, sc, st, &S));
    RCHK(validate_now(ctx, sc->alphabet, seqs->residues, seqs->offsets_host[N], nullptr, 0, st));
    RCHK(launch_fill((uint32_t *)sums, 0u, 2 * (int64_t)ncand, st));
    std::vector<int32_t> perm, gcen, gb0, gslot;
    if (partners_host) {   // partners in length order, as for all sequences
        perm.assign(partners_host, partners_host + npart);
        const int64_t *oh = seqs->offsets_host;
        std::stable_sort(perm.begin(), perm.end(),
                         [&](int32_t x, int32_t y) { return (oh[x + 1] - oh[x]) < (oh[y + 1] - oh[y]); });
    } else {
        perm = length_perm(seqs);
    }
    const int np = (int)perm.size();
    const bool p16 = strip16_ok(S, seqs);
    const int step = p16 ? 128 : 64;
    for (int q = 0; q < ncand; ++q)
        for (int b = 0; b < np; b += step) {
            gcen.push_back(hc[q]);
            gb0.push_back(b);
            gslot.push_back(q);
        }
    RCHK(run_groups(ctx, S, seqs, 2, (int64_t)gcen.size(), gcen, gb0, perm, gslot, sums, nullptr, st, np, p16));
    if (center_host) RCHK(argmax_sums(ctx, sums, hc.data(), ncand, center_host, st));
    return HALIGN_OK;
}

extern "C" {

int halign_center_judge(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, const int32_t *cand,
                        int32_t ncand, int64_t *sums, int32_t *center_host, void *stream) {
    if (!ctx || !sums || !cand || ncand <= 0) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> hc(ncand);
    HCHK(hipMemcpyAsync(hc.data(), cand, 4 * (size_t)ncand, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    return judge_impl(ctx, sc, seqs, hc, nullptr, 0, sums, center_host, st);
}

int halign_center_judge_sample(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                               const int32_t *cand, int32_t ncand, const int32_t *partners_host, int32_t npartners,
                               int64_t *sums, int32_t *center_host, void *stream) {
    if (!ctx || !sums || !cand || ncand <= 0 || npartners < 0 || (npartners > 0 && !partners_host))
        return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    const int N = seqs->n;
    for (int q = 0; q < npartners; ++q)
        if (partners_host[q] < 0 || partners_host[q] >= N) return fail(HALIGN_E_INVALID, "partner out of range");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> hc(ncand);
    HCHK(hipMemcpyAsync(hc.data(), cand, 4 * (size_t)ncand, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    return judge_impl(ctx, sc, seqs, hc, partners_host, npartners, sums, center_host, st);
}

int halign_sw_pairs(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, const int32_t *anchors_host,
                    int32_t nanchors, const int32_t *partners_host, int32_t *score, void *stream) {
    if (!ctx || nanchors < 0 || (nanchors > 0 && (!anchors_host || !partners_host || !score)))
        return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    const int N = seqs->n;
    const int64_t np = (int64_t)nanchors * 64;
    for (int q = 0; q < nanchors; ++q)
        if (anchors_host[q] < 0 || anchors_host[q] >= N) return fail(HALIGN_E_INVALID, "anchor out of range");
    for (int64_t q = 0; q < np; ++q)
        if (partners_host[q] < 0 || partners_host[q] >= N) return fail(HALIGN_E_INVALID, "partner out of range");
    if (nanchors == 0) return HALIGN_OK;
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    Scoring S;
    RCHK(upload_matrix(ctx, sc, st, &S));
    RCHK(validate_now(ctx, sc->alphabet, seqs->residues, seqs->offsets_host[N], nullptr, 0, st));
    // group q: anchor q as the center, lanes = partners[64q .. 64q+63] (the
    // "perm" of the anchored mode), scores land at slot 64q + lane
    std::vector<int32_t> perm(partners_host, partners_host + np), gcen(anchors_host, anchors_host + nanchors),
        gb0(nanchors), gslot(nanchors);
    for (int q = 0; q < nanchors; ++q) {
        gb0[q] = q * 64;
        gslot[q] = q;
    }
    RCHK(grow(ctx, ctx->pairbuf, 16 * (size_t)nanchors + 256));
    int64_t *sums = (int64_t *)ctx->pairbuf.p;
    RCHK(launch_fill((uint32_t *)sums, 0u, 2 * (int64_t)nanchors, st));
    halign_seqs sq2 = *seqs;
    sq2.n = N;
    RCHK(run_groups(ctx, S, &sq2, 2, (int64_t)gcen.size(), gcen, gb0, perm, gslot, sums, score, st, (int)np));
    return HALIGN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free score-only batch: its scratch (matrix copy, work counter,
// strip boundary rows) is one static device array per GPU.  In host code the
// array's name only stands for the symbol; its device address on the current
// GPU comes from hipGetSymbolAddress, taken once per device and kept.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = HALIGN_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchHead = 4096;   // matrix copy at 0, work counter at 2048, boundary rows after
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct ScratchSlot {
    void *ptr = nullptr;
    int num_cu = 0;
};
constexpr int kMaxDevices = 64;
ScratchSlot g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// the current device's copy of `scratch` (address and compute-unit count)
int scratch_of_device(int dev, ScratchSlot *out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HALIGN_E_UNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchSlot &s = g_scratch[dev];
    if (!s.ptr) {
        void *p = nullptr;
        HCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        int cu = 0;
        HCHK(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
        s.num_cu = std::max(1, cu);
        s.ptr = p;
    }
    *out = s;
    return HALIGN_OK;
}

}  // namespace

extern "C" {

int halign_sw_score_noalloc(const halign_scoring *sc, const uint8_t *center, int32_t m, const halign_seqs *seqs,
                            int32_t *score, int32_t *cells, void *stream) {
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    if (m <= 0 || !center) return fail(HALIGN_E_INVALID, "empty center");
    if (m >= 65536) return fail(HALIGN_E_UNSUPPORTED, "center length %d >= 65536", m);
    const int N = seqs->n;
    if (N == 0) return HALIGN_OK;
    if (!score) return fail(HALIGN_E_INVALID, "score is NULL");
    int dev = 0;
    HCHK(hipGetDevice(&dev));
    ScratchSlot sl;
    RCHK(scratch_of_device(dev, &sl));
    const int64_t *oh = seqs->offsets_host;
    int nmax_all = 0;
    for (int k = 0; k < N; ++k) nmax_all = std::max(nmax_all, (int)(oh[k + 1] - oh[k]));
    // boundary rows: 64 lanes x the longest sequence (whole prefetch blocks) per workgroup
    const int64_t bstride = (int64_t)64 * strip_cols(nmax_all);
    const size_t per_wg = (size_t)bstride * sizeof(int2);
    const size_t avail = kScratchBytes - kScratchHead;
    if (per_wg > avail)
        return fail(HALIGN_E_UNSUPPORTED,
                    "longest sequence %d needs %zu bytes of scratch per workgroup; the static scratch holds %zu",
                    nmax_all, per_wg, avail);
    const int64_t ngroups = ((int64_t)N + 63) / 64;
    const int grid = (int)std::max<int64_t>(
        1, std::min<int64_t>({ngroups, (int64_t)sl.num_cu * 16, (int64_t)(avail / per_wg)}));
    hipStream_t st = (hipStream_t)stream;
    unsigned char *base = (unsigned char *)sl.ptr;
    hk::MatrixArg mat{};
    memcpy(mat.v, sc->matrix_host, (size_t)sc->alphabet * sc->alphabet);
    hipLaunchKernelGGL(hk::matrix_copy_kernel, dim3(1), dim3(256), 0, st, mat, sc->alphabet * sc->alphabet,
                       (int8_t *)base);
    HCHK(hipGetLastError());
    // the work counter starts at zero on every call (the array keeps the last call's contents)
    RCHK(launch_fill((uint32_t *)(base + 2048), 0u, 2, st));
    hk::InterArgs a{};
    a.mat = (const int8_t *)base;
    a.alpha = sc->alphabet;
    a.center = center;
    a.m = m;
    a.res = seqs->residues;
    a.off = seqs->offsets;
    a.mode = 0;
    a.order = nullptr;
    a.gnmax = nullptr;
    a.nseq = N;
    a.ngroups = ngroups;
    a.ge = sc->gap_extend;
    a.goe = sc->gap_open + sc->gap_extend;
    a.counter = (unsigned long long *)(base + 2048);
    a.score = score;
    a.endcell = nullptr;
    a.cells4 = reinterpret_cast<int4 *>(cells);
    a.bound = (int2 *)(base + kScratchHead);
    a.bstride = bstride;
    launch_inter(a, false, cells != nullptr, grid, st);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

}  // extern "C"

// Column profile into prof, *dbad raised on a byte that is neither a residue
// code below alpha nor the gap.  Rows are split into slabs (at most
// kProfMaxSlab rows, for 16-bit partial counts) so that the grid has a few
// thousand workgroups; the slabs' counts meet in a second pass, not in
// atomics (many workgroups adding into the same profile line serialise).
// part: at least column_profile_part_bytes() bytes of device scratch.
static void column_profile_shape(int32_t n, int64_t width, int64_t *ncb, int64_t *nslab, int *slab) {
    if (n <= 0 || width <= 0) {   // nothing to count
        *ncb = *nslab = 0;
        *slab = 1;
        return;
    }
    *ncb = (width + hk::kProfCols - 1) / hk::kProfCols;
    int64_t ns = std::max<int64_t>((n + hk::kProfMaxSlab - 1) / hk::kProfMaxSlab,
                                   std::min<int64_t>((3072 + *ncb - 1) / *ncb, (n + 255) / 256));
    int sl = (int)((n + ns - 1) / std::max<int64_t>(ns, 1));
    if (const char *e = getenv("HALIGN_PROFILE_SLAB"))   // test knob: rows per slab
        if (atoi(e) > 0) sl = std::min(atoi(e), hk::kProfMaxSlab);
    *slab = std::max(sl, 1);
    *nslab = (n + *slab - 1) / *slab;
}

static size_t column_profile_part_bytes(int32_t n, int64_t width, int32_t alpha) {
    int64_t ncb, nslab;
    int slab;
    column_profile_shape(n, width, &ncb, &nslab, &slab);
    return (size_t)nslab * (size_t)width * (size_t)(alpha + 1) * 2;
}

static int column_profile_launch(const uint8_t *msa, int32_t n, int64_t width, int32_t alpha, int32_t *prof,
                                 uint16_t *part, int *dbad, hipStream_t st) {
    const int nsym = alpha + 1;
    if (n <= 0 || width <= 0) return launch_fill((uint32_t *)prof, 0u, width * nsym, st);
    int64_t ncb, nslab;
    int slab;
    column_profile_shape(n, width, &ncb, &nslab, &slab);
    if (ncb > 0x7fffffff || nslab > 65535) return fail(HALIGN_E_UNSUPPORTED, "%d x %lld MSA", n, (long long)width);
    hipLaunchKernelGGL(hk::colprof_kernel, dim3((unsigned)ncb, (unsigned)nslab), dim3(256),
                       (size_t)(alpha + 3) * 256 * 4, st, msa, n, width, alpha, slab, part, dbad);
    HCHK(hipGetLastError());
    const int64_t nelem = width * nsym;
    hipLaunchKernelGGL(hk::colprof_sum_kernel, dim3((unsigned)((nelem + 255) / 256)), dim3(256), 0, st,
                       (const uint16_t *)part, (int)nslab, nelem, prof);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

extern "C" {

int halign_column_profile(const uint8_t *msa, int32_t n, int64_t width, int32_t alphabet, int32_t *profile,
                          void *stream) {
    if (n < 0 || width < 0 || alphabet < 1 || alphabet > 32 || (width > 0 && !profile) ||
        (n > 0 && width > 0 && !msa))
        return fail(HALIGN_E_INVALID, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    int *dbad = nullptr;
    HCHK(hipMalloc(&dbad, 256 + column_profile_part_bytes(n, width, alphabet)));
    int rc = launch_fill((uint32_t *)dbad, 0u, 1, st);
    if (rc == HALIGN_OK)
        rc = column_profile_launch(msa, n, width, alphabet, profile, (uint16_t *)((char *)dbad + 256), dbad, st);
    int hbad = 0;
    if (rc == HALIGN_OK && hipMemcpyAsync(&hbad, dbad, 4, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = fail(HALIGN_E_DEVICE, "profile flag copy");
    if (rc == HALIGN_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(HALIGN_E_DEVICE, "profile sync");
    (void)hipFree(dbad);
    if (rc != HALIGN_OK) return rc;
    if (hbad) return fail(HALIGN_E_INVALID, "MSA byte neither a residue code below %d nor the gap", alphabet);
    return HALIGN_OK;
}

int halign_sp_score(const halign_scoring *sc, const uint8_t *msa, int32_t n, int64_t width, int64_t *out_host,
                    void *stream) {
    RCHK(check_scoring(sc));
    if (!out_host || n < 0 || width < 0 || (n > 0 && width > 0 && !msa)) return fail(HALIGN_E_INVALID, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int alpha = sc->alphabet;
    // one allocation: matrix (1 KiB), sums (16 B), flag, profile
    const size_t prof_b = ((size_t)std::max<int64_t>(width, 1) * (alpha + 1) * 4 + 255) & ~(size_t)255;
    char *buf = nullptr;
    HCHK(hipMalloc(&buf, 2048 + prof_b + column_profile_part_bytes(n, width, alpha)));
    int8_t *dmat = (int8_t *)buf;
    unsigned long long *dout = (unsigned long long *)(buf + 1024);
    int *dbad = (int *)(buf + 1040);
    int32_t *prof = (int32_t *)(buf + 2048);
    int rc = HALIGN_OK;
    unsigned long long h[2] = {0, 0};
    int hbad = 0;
    if (hipMemcpyAsync(dmat, sc->matrix_host, (size_t)alpha * alpha, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(HALIGN_E_DEVICE, "matrix copy");
    if (rc == HALIGN_OK) rc = launch_fill((uint32_t *)dout, 0u, 5, st);   // sums and flag
    if (rc == HALIGN_OK)
        rc = column_profile_launch(msa, n, width, alpha, prof, (uint16_t *)(buf + 2048 + prof_b), dbad, st);
    if (rc == HALIGN_OK && n > 0 && width > 0) {
        hipLaunchKernelGGL(hk::sp_profile_kernel, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, st, prof,
                           width, alpha, (const int8_t *)dmat, sc->gap_extend, dout);
        if (hipGetLastError() != hipSuccess) rc = fail(HALIGN_E_DEVICE, "sp_profile_kernel launch");
    }
    if (rc == HALIGN_OK && (hipMemcpyAsync(h, dout, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
                            hipMemcpyAsync(&hbad, dbad, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                            hipStreamSynchronize(st) != hipSuccess))
        rc = fail(HALIGN_E_DEVICE, "sp result copy");
    (void)hipFree(buf);
    if (rc != HALIGN_OK) return rc;
    if (hbad) return fail(HALIGN_E_INVALID, "MSA byte neither a residue code below %d nor the gap", alpha);
    out_host[0] = (int64_t)h[0];
    out_host[1] = (int64_t)h[1];
    return HALIGN_OK;
}

int halign_msa(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, int32_t center,
               const halign_model *model, halign_alloc_fn alloc, void *user, uint8_t **msa, int64_t *width_host,
               int32_t *center_out_host, void *stream) {
    if (!ctx || !alloc || !msa || !width_host) return fail(HALIGN_E_INVALID, "bad arguments");
    ctx->hmarks.clear();
    hmark(ctx, "start");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    hmark(ctx, "checks");
    const int N = seqs->n;
    if (N <= 0) return fail(HALIGN_E_INVALID, "empty set");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int32_t c = center;
    if (center == HALIGN_CENTER_EXACT) {
        RCHK(grow(ctx, ctx->msabuf, 16 * (size_t)N + 256));
        RCHK(halign_center_exact(ctx, sc, seqs, (int64_t *)ctx->msabuf.p, &c, stream));
    } else if (center == HALIGN_CENTER_LEARNED) {
        if (!model) return fail(HALIGN_E_INVALID, "learned center needs a model");
        RCHK(halign_center_learned(ctx, sc, seqs, model, 16, nullptr, &c, stream));
    } else if (center < 0 || center >= N) {
        return fail(HALIGN_E_INVALID, "center %d out of range", center);
    }
    const int64_t *oh = seqs->offsets_host;
    const int m = (int)(oh[c + 1] - oh[c]);
    if (m <= 0) return fail(HALIGN_E_INVALID, "center sequence is empty");
    const int aw = (m + 31) / 32;
    // per-pair outputs in one workspace
    const size_t b_score = 4 * (size_t)N, b_cells = 16 * (size_t)N, b_ins = 2 * (size_t)N * (m + 1) + 4,
                 b_al = 4 * (size_t)N * aw, b_G = 4 * (size_t)(m + 1), b_col = 8 * (size_t)(m + 1);
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 255) & ~size_t(255); return r; };
    const size_t o_score = take(b_score), o_cells = take(b_cells), o_ins = take(b_ins), o_al = take(b_al),
                 o_G = take(b_G), o_col = take(b_col);
    DevBuf &W = ctx->msabuf;
    RCHK(grow(ctx, W, o));
    char *wb = (char *)W.p;
    int32_t *score = (int32_t *)(wb + o_score);
    int32_t *cells = (int32_t *)(wb + o_cells);
    uint16_t *ins = (uint16_t *)(wb + o_ins);
    uint32_t *al = (uint32_t *)(wb + o_al);
    int32_t *G = (int32_t *)(wb + o_G);
    int64_t *col = (int64_t *)(wb + o_col);
    const uint8_t *cen = seqs->residues + oh[c];
    // the walk max-merges every pair's insertion counts into G (the center's own are all zero)
    RCHK(sw_batch_async(ctx, sc, cen, m, seqs, HALIGN_TRACEBACK | (ctx->use_graph ? HALIGN_GRAPH : 0u), score, cells,
                        ins, al, stream, G, c, true));
    hipLaunchKernelGGL(hk::center_row_kernel, dim3(1), dim3(256), 0, st, ins, al, c, m, aw);
    HCHK(hipGetLastError());
    int64_t width = 0;
    hmark(ctx, "batch");
    RCHK(merge_offsets(ctx, G, m + 1, col, &width, st));   // synchronises
    hmark(ctx, "sync");
    RCHK(validate_check(ctx));
    uint8_t *out = (uint8_t *)alloc((size_t)N * (size_t)width, user);
    if (!out && width > 0) return fail(HALIGN_E_NOMEM, "allocator returned NULL for %lld bytes", (long long)(N * width));
    hmark(ctx, "alloc");
    RCHK(halign_emit_rows(ctx, seqs, m, ins, al, G, col, width, out, stream));
    hmark(ctx, "rows");
    hmark_print(ctx);
    *msa = out;
    *width_host = width;
    if (center_out_host) *center_out_host = c;
    return HALIGN_OK;
}

}  // extern "C"

// ===========================================================================
// Learned center proposer
// ===========================================================================
namespace {

template <bool TA, bool TB, int EPI>
int gemm(const hk::GemmArgs &g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0) return HALIGN_OK;
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
    if (grid.y > 65535) return fail(HALIGN_E_UNSUPPORTED, "GEMM with %d rows", g.M);
    hipLaunchKernelGGL((hk::gemm_bf16_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, g);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

// fixed-order column sums of a rows x cols fp32 matrix into out[cols]
int colsum(halign_ctx *ctx, DevBuf &scratch, const float *A, int rows, int cols, int lda, float *out, hipStream_t st) {
    const int nblk = std::max(1, (rows + 1023) / 1024);
    RCHK(grow(ctx, scratch, (size_t)nblk * cols * 4 + 256));
    float *part = (float *)scratch.p;
    if (rows > 0) {
        hipLaunchKernelGGL(hk::colsum_partial_kernel, dim3((cols + 255) / 256, nblk), dim3(256), 0, st, A, rows, cols,
                           lda, part);
    } else {
        RCHK(launch_fill((uint32_t *)part, 0u, cols, st));
    }
    hipLaunchKernelGGL(hk::colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, (const float *)part,
                       rows > 0 ? nblk : 1, cols, out);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int check_model(const halign_model *md) {
    if (!md || !md->W1 || !md->b1 || !md->W2 || !md->b2) return fail(HALIGN_E_INVALID, "model pointers are NULL");
    return HALIGN_OK;
}

}  // namespace

extern "C" {

int halign_featurize(const halign_seqs *seqs, const int32_t *rows, int32_t nrows, uint16_t *X, void *stream) {
    if (!seqs || nrows < 0 || (nrows > 0 && !X)) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_seqs(seqs));
    if (!rows && nrows > seqs->n) return fail(HALIGN_E_INVALID, "nrows > N");
    if (nrows == 0) return HALIGN_OK;
    hipLaunchKernelGGL(hk::featurize_kernel, dim3(nrows), dim3(256), 0, (hipStream_t)stream, seqs->residues,
                       seqs->offsets, rows, nrows, X);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int halign_mlp_forward(halign_ctx *ctx, const halign_model *model, const uint16_t *X, int32_t nrows, float *Z,
                       uint16_t *Hb, float *E, void *stream) {
    if (!ctx || nrows < 0 || (nrows > 0 && (!X || !Hb || !E))) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_model(model));
    hipStream_t st = (hipStream_t)stream;
    hk::GemmArgs g1{};
    g1.A = X; g1.B = model->W1; g1.M = nrows; g1.N = hk::kHid; g1.K = hk::kFeat; g1.lda = hk::kFeat; g1.ldb = hk::kHid;
    g1.C = Z; g1.ldc = hk::kHid; g1.bias = model->b1; g1.Cb = Hb; g1.ldcb = hk::kHid;
    RCHK((gemm<false, false, 1>(g1, st)));
    hk::GemmArgs g2{};
    g2.A = Hb; g2.B = model->W2; g2.M = nrows; g2.N = hk::kEmb; g2.K = hk::kHid; g2.lda = hk::kHid; g2.ldb = hk::kEmb;
    g2.C = E; g2.ldc = hk::kEmb; g2.bias = model->b2;
    RCHK((gemm<false, false, 0>(g2, st)));
    return HALIGN_OK;
}

int halign_pair_loss(halign_ctx *ctx, const float *E, const float *target, int32_t npairs, float *dE,
                     float *loss_out, void *stream) {
    if (!ctx || npairs < 0 || (npairs > 0 && (!E || !target || !dE || !loss_out)))
        return fail(HALIGN_E_INVALID, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    RCHK(grow(ctx, ctx->mlp[0], (size_t)npairs * 4 + (size_t)2 * npairs * hk::kEmb * 2 + 512));
    float *sq = (float *)ctx->mlp[0].p;
    uint16_t *dEb = (uint16_t *)((char *)ctx->mlp[0].p + (((size_t)npairs * 4 + 255) & ~size_t(255)));
    if (npairs > 0) {
        hipLaunchKernelGGL(hk::pair_loss_kernel, dim3((npairs + 255) / 256), dim3(256), 0, st, E, target, npairs, dE,
                           dEb, sq);
        HCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(hk::mean_kernel, dim3(1), dim3(256), 0, st, (const float *)sq, npairs, loss_out);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int halign_pair_loss_grouped(halign_ctx *ctx, const float *E, const float *target, int32_t npairs, int32_t group,
                             float lam, float *dE, float *loss_out, void *stream) {
    if (group <= 0) return halign_pair_loss(ctx, E, target, npairs, dE, loss_out, stream);
    if (!ctx || npairs < 0 || group > 64 || npairs % group != 0 ||
        (npairs > 0 && (!E || !target || !dE || !loss_out)))
        return fail(HALIGN_E_INVALID, "bad arguments (1 <= group <= 64 dividing npairs)");
    hipStream_t st = (hipStream_t)stream;
    const int G = npairs / group;
    const size_t b_sq = ((size_t)npairs * 4 + 255) & ~size_t(255), b_g = ((size_t)G * 4 + 255) & ~size_t(255);
    RCHK(grow(ctx, ctx->mlp[0], b_sq + b_g + (size_t)2 * npairs * hk::kEmb * 2 + 512));
    float *sq = (float *)ctx->mlp[0].p;
    float *gsq = (float *)((char *)ctx->mlp[0].p + b_sq);
    uint16_t *dEb = (uint16_t *)((char *)ctx->mlp[0].p + b_sq + b_g);
    if (G > 0) {
        hipLaunchKernelGGL(hk::pair_group_loss_kernel, dim3(G), dim3(64), 0, st, E, target, npairs, group, lam, dE,
                           dEb, sq, gsq);
        HCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(hk::mean2_kernel, dim3(1), dim3(256), 0, st, (const float *)sq, npairs, (const float *)gsq, G,
                       lam, loss_out);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int halign_mlp_backward(halign_ctx *ctx, const halign_model *model, const uint16_t *X, int32_t nrows, const float *Z,
                        const uint16_t *Hb, const float *dE, float *dW1, float *db1, float *dW2, float *db2,
                        void *stream) {
    if (!ctx || nrows < 0 || !dW1 || !db1 || !dW2 || !db2 || (nrows > 0 && (!X || !Z || !Hb || !dE)))
        return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_model(model));
    hipStream_t st = (hipStream_t)stream;
    const size_t b_dEb = ((size_t)nrows * hk::kEmb * 2 + 255) & ~size_t(255);
    const size_t b_dZ = ((size_t)nrows * hk::kHid * 4 + 255) & ~size_t(255);
    const size_t b_dZb = ((size_t)nrows * hk::kHid * 2 + 255) & ~size_t(255);
    RCHK(grow(ctx, ctx->mlp[1], b_dEb + b_dZ + b_dZb + 256));
    uint16_t *dEb = (uint16_t *)ctx->mlp[1].p;
    float *dZ = (float *)((char *)ctx->mlp[1].p + b_dEb);
    uint16_t *dZb = (uint16_t *)((char *)ctx->mlp[1].p + b_dEb + b_dZ);
    if (nrows > 0) {
        hipLaunchKernelGGL(hk::f32_to_bf16_kernel, dim3(grid_for((int64_t)nrows * hk::kEmb, 256, 4096)), dim3(256), 0,
                           st, dE, dEb, (int64_t)nrows * hk::kEmb);
        HCHK(hipGetLastError());
    }
    hk::GemmArgs a{};
    // dW2 = Hb^T dEb
    a.A = Hb; a.B = dEb; a.M = hk::kHid; a.N = hk::kEmb; a.K = nrows; a.lda = hk::kHid; a.ldb = hk::kEmb;
    a.C = dW2; a.ldc = hk::kEmb;
    if (nrows > 0) RCHK((gemm<true, false, 0>(a, st)));
    else RCHK(launch_fill((uint32_t *)dW2, 0u, (int64_t)hk::kHid * hk::kEmb, st));
    RCHK(colsum(ctx, ctx->mlp[2], dE, nrows, hk::kEmb, hk::kEmb, db2, st));
    // dZ = (dEb W2^T) * (Z > 0)
    hk::GemmArgs b{};
    b.A = dEb; b.B = model->W2; b.M = nrows; b.N = hk::kHid; b.K = hk::kEmb; b.lda = hk::kEmb; b.ldb = hk::kEmb;
    b.C = dZ; b.ldc = hk::kHid; b.Cb = dZb; b.ldcb = hk::kHid; b.Hpre = Z; b.ldh = hk::kHid;
    RCHK((gemm<false, true, 2>(b, st)));
    RCHK(colsum(ctx, ctx->mlp[2], dZ, nrows, hk::kHid, hk::kHid, db1, st));
    // dW1 = X^T dZb
    hk::GemmArgs c{};
    c.A = X; c.B = dZb; c.M = hk::kFeat; c.N = hk::kHid; c.K = nrows; c.lda = hk::kFeat; c.ldb = hk::kHid;
    c.C = dW1; c.ldc = hk::kHid;
    if (nrows > 0) RCHK((gemm<true, false, 0>(c, st)));
    else RCHK(launch_fill((uint32_t *)dW1, 0u, (int64_t)hk::kFeat * hk::kHid, st));
    return HALIGN_OK;
}

int halign_f32_to_bf16(const float *src, uint16_t *dst, int64_t n, void *stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) return fail(HALIGN_E_INVALID, "bad arguments");
    if (n == 0) return HALIGN_OK;
    hipLaunchKernelGGL(hk::f32_to_bf16_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, (hipStream_t)stream, src,
                       dst, n);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int halign_adam_step(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr, float beta1,
                     float beta2, float eps, int32_t t, void *stream) {
    if (n < 0 || t < 1 || (n > 0 && (!p || !g || !m || !v))) return fail(HALIGN_E_INVALID, "bad arguments");
    if (n == 0) return HALIGN_OK;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(hk::adam_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, pb,
                       n, lr, beta1, beta2, eps, c1, c2);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int halign_topk_center(halign_ctx *ctx, const float *E, int32_t nrows, int32_t k, float *u, int32_t *top,
                       void *stream) {
    if (!ctx || !E || !u || !top || nrows <= 0 || k <= 0 || k > nrows || k > 256)
        return fail(HALIGN_E_INVALID, "bad arguments (1 <= k <= min(N, 256))");
    hipStream_t st = (hipStream_t)stream;
    RCHK(grow(ctx, ctx->mlp[3], 4096));
    float *S = (float *)ctx->mlp[3].p;
    RCHK(colsum(ctx, ctx->mlp[2], E, nrows, hk::kEmb, hk::kEmb, S, st));
    hipLaunchKernelGGL(hk::center_score_kernel, dim3((nrows + 255) / 256), dim3(256), 0, st, E, (const float *)S, nrows,
                       u);
    HCHK(hipGetLastError());
    // rounds of block top-k until one block holds everything
    int n = nrows;
    const float *val = u;
    const int32_t *idx = nullptr;
    int round = 0;
    for (;;) {
        const int nblk = (n + hk::kTopkChunk - 1) / hk::kTopkChunk;
        const size_t need = (size_t)nblk * k * 8 + 512;
        DevBuf &buf = ctx->mlp[4 + (round & 1)];
        RCHK(grow(ctx, buf, need));
        float *ov = (float *)buf.p;
        int32_t *oi = (int32_t *)((char *)buf.p + (((size_t)nblk * k * 4 + 255) & ~size_t(255)));
        hipLaunchKernelGGL(hk::topk_kernel, dim3(nblk), dim3(256), 0, st, val, idx, n, k, ov, oi);
        HCHK(hipGetLastError());
        if (nblk == 1) {
            HCHK(hipMemcpyAsync(top, oi, 4 * (size_t)k, hipMemcpyDeviceToDevice, st));
            break;
        }
        val = ov;
        idx = oi;
        n = nblk * k;
        ++round;
    }
    return HALIGN_OK;
}

int halign_train_proposer(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                          const halign_train_opts *opts, const halign_params *pr, float *loss_host, void *stream) {
    if (!ctx || !opts || !pr || !pr->W1 || !pr->b1 || !pr->W2 || !pr->b2 || !pr->W1b || !pr->W2b)
        return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    const int N = seqs->n;
    if (N < 2 || opts->anchors <= 0 || opts->batch <= 0 || opts->epochs <= 0)
        return fail(HALIGN_E_INVALID, "need N >= 2 and positive anchors, batch, epochs");
    hipStream_t st = (hipStream_t)stream;
    HCHK(hipSetDevice(ctx->device));
    // training pairs: anchors with `partners` partners each (never the anchor
    // itself); the score kernel takes 64 partners per anchor, of which the
    // first `partners` are used
    uint64_t rs = opts->seed;
    const int A = opts->anchors;
    const int PA = (opts->partners > 0 && opts->partners < 64) ? opts->partners : 64;
    const int P = A * PA;
    std::vector<int32_t> anc(A), par((size_t)A * 64);
    for (int q = 0; q < A; ++q) anc[q] = (int32_t)(splitmix(rs) % (uint64_t)N);
    for (size_t q = 0; q < (size_t)A * 64; ++q) {
        int32_t b;
        do { b = (int32_t)(splitmix(rs) % (uint64_t)N); } while (b == anc[q / 64]);
        par[q] = b;
    }
    // with a group weight, a batch holds whole anchors (all PA partners of
    // each), and the loss adds the squared mean error of each anchor's pairs
    const bool grouped = opts->group_weight > 0.f;
    // scratch layout in mlp[6]: scores, targets, batch index lists, X_all
    const int B = grouped ? std::max(1, std::min(opts->batch, P) / PA) * PA : std::min(opts->batch, P);
    const int steps_per_epoch = P / B;
    const int nsteps = steps_per_epoch * opts->epochs;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = (off + bytes + 255) & ~size_t(255); return r; };
    const size_t o_score = take(4 * (size_t)A * 64), o_tgt = take(4 * (size_t)A * 64),
                 o_idx = take(4 * (size_t)nsteps * 2 * B),
                 o_tix = take(4 * (size_t)nsteps * B), o_tb = take(4 * (size_t)B), o_loss = take(4 * (size_t)nsteps),
                 o_X = take(2 * (size_t)N * hk::kFeat), o_Xb = take(2 * (size_t)2 * B * hk::kFeat),
                 o_Z = take(4 * (size_t)2 * B * hk::kHid), o_Hb = take(2 * (size_t)2 * B * hk::kHid),
                 o_E = take(4 * (size_t)2 * B * hk::kEmb), o_dE = take(4 * (size_t)2 * B * hk::kEmb),
                 o_g = take(4 * (size_t)(hk::kFeat * hk::kHid + hk::kHid + hk::kHid * hk::kEmb + hk::kEmb)),
                 o_m = take(4 * (size_t)(hk::kFeat * hk::kHid + hk::kHid + hk::kHid * hk::kEmb + hk::kEmb)),
                 o_v = take(4 * (size_t)(hk::kFeat * hk::kHid + hk::kHid + hk::kHid * hk::kEmb + hk::kEmb)),
                 o_e = take(4 * (size_t)(hk::kFeat * hk::kHid + hk::kHid + hk::kHid * hk::kEmb + hk::kEmb));
    RCHK(grow(ctx, ctx->mlp[6], off));
    char *w = (char *)ctx->mlp[6].p;
    int32_t *score = (int32_t *)(w + o_score);
    float *tgt = (float *)(w + o_tgt);
    RCHK(halign_sw_pairs(ctx, sc, seqs, anc.data(), A, par.data(), score, stream));
    hipLaunchKernelGGL(hk::scale_targets_kernel, dim3((A * 64 + 255) / 256), dim3(256), 0, st, (const int32_t *)score,
                       A * 64, tgt);
    HCHK(hipGetLastError());
    // batch index lists for every step (rows of X_all for a then b, and target slots)
    {
        std::vector<int32_t> order(P), hidx((size_t)nsteps * 2 * B), htix((size_t)nsteps * B);
        for (int q = 0; q < P; ++q) order[q] = q;
        std::vector<int32_t> aord(A);
        for (int q = 0; q < A; ++q) aord[q] = q;
        for (int e = 0; e < opts->epochs; ++e) {
            if (grouped) {   // shuffled anchors, each with its partners in order
                for (int q = A - 1; q > 0; --q) std::swap(aord[q], aord[(int)(splitmix(rs) % (uint64_t)(q + 1))]);
                for (int q = 0; q < P; ++q) order[q] = aord[q / PA] * PA + q % PA;
            } else {
                for (int q = P - 1; q > 0; --q) std::swap(order[q], order[(int)(splitmix(rs) % (uint64_t)(q + 1))]);
            }
            for (int s = 0; s < steps_per_epoch; ++s) {
                const int step = e * steps_per_epoch + s;
                for (int r = 0; r < B; ++r) {
                    const int q = order[s * B + r];
                    const int slot = (q / PA) * 64 + q % PA;
                    hidx[(size_t)step * 2 * B + r] = anc[q / PA];
                    hidx[(size_t)step * 2 * B + B + r] = par[slot];
                    htix[(size_t)step * B + r] = slot;
                }
            }
        }
        HCHK(hipMemcpyAsync(w + o_idx, hidx.data(), 4 * hidx.size(), hipMemcpyHostToDevice, st));
        HCHK(hipMemcpyAsync(w + o_tix, htix.data(), 4 * htix.size(), hipMemcpyHostToDevice, st));
        HCHK(hipStreamSynchronize(st));   // host vectors go out of scope
    }
    uint16_t *X = (uint16_t *)(w + o_X);
    RCHK(halign_featurize(seqs, nullptr, N, X, stream));
    const int64_t nW1 = (int64_t)hk::kFeat * hk::kHid, nW2 = (int64_t)hk::kHid * hk::kEmb;
    float *g = (float *)(w + o_g), *mo = (float *)(w + o_m), *vo = (float *)(w + o_v);
    const int64_t ntot = nW1 + hk::kHid + nW2 + hk::kEmb;
    RCHK(launch_fill((uint32_t *)mo, 0u, ntot, st));
    RCHK(launch_fill((uint32_t *)vo, 0u, ntot, st));
    float *gW1 = g, *gb1 = g + nW1, *gW2 = gb1 + hk::kHid, *gb2 = gW2 + nW2;
    float *mW1 = mo, *mb1 = mo + nW1, *mW2 = mb1 + hk::kHid, *mb2 = mW2 + nW2;
    float *vW1 = vo, *vb1 = vo + nW1, *vW2 = vb1 + hk::kHid, *vb2 = vW2 + nW2;
    uint16_t *Xb = (uint16_t *)(w + o_Xb), *Hb = (uint16_t *)(w + o_Hb);
    float *Z = (float *)(w + o_Z), *E = (float *)(w + o_E), *dE = (float *)(w + o_dE), *tb = (float *)(w + o_tb);
    float *loss = (float *)(w + o_loss);
    halign_model md{pr->W1b, pr->b1, pr->W2b, pr->b2};
    // parameter average (starts from the initial parameters)
    const bool use_ema = opts->ema > 0.f && opts->ema < 1.f;
    float *ema = (float *)(w + o_e);
    float *eW1 = ema, *eb1 = ema + nW1, *eW2 = eb1 + hk::kHid, *eb2 = eW2 + nW2;
    if (use_ema) {
        HCHK(hipMemcpyAsync(eW1, pr->W1, 4 * (size_t)nW1, hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpyAsync(eb1, pr->b1, 4 * (size_t)hk::kHid, hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpyAsync(eW2, pr->W2, 4 * (size_t)nW2, hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpyAsync(eb2, pr->b2, 4 * (size_t)hk::kEmb, hipMemcpyDeviceToDevice, st));
    }
    auto ema_step = [&](const float *p, float *e, int64_t n) -> int {
        hipLaunchKernelGGL(hk::ema_kernel, dim3(grid_for(n, 256, 2048)), dim3(256), 0, st, p, e, n, opts->ema);
        HCHK(hipGetLastError());
        return HALIGN_OK;
    };
    for (int step = 0; step < nsteps; ++step) {
        const int32_t *ix = (const int32_t *)(w + o_idx) + (size_t)step * 2 * B;
        const int32_t *tx = (const int32_t *)(w + o_tix) + (size_t)step * B;
        hipLaunchKernelGGL(hk::gather_rows_kernel, dim3(2 * B), dim3(256), 0, st, (const uint16_t *)X, ix, 2 * B,
                           hk::kFeat, Xb);
        hipLaunchKernelGGL(hk::gather_f32_kernel, dim3((B + 255) / 256), dim3(256), 0, st, (const float *)tgt, tx, B, tb);
        HCHK(hipGetLastError());
        RCHK(halign_mlp_forward(ctx, &md, Xb, 2 * B, Z, Hb, E, stream));
        RCHK(halign_pair_loss_grouped(ctx, E, tb, B, grouped ? PA : 0, opts->group_weight, dE, loss + step, stream));
        RCHK(halign_mlp_backward(ctx, &md, Xb, 2 * B, Z, Hb, dE, gW1, gb1, gW2, gb2, stream));
        const float lr = opts->lr;
        RCHK(halign_adam_step(pr->W1, gW1, mW1, vW1, pr->W1b, nW1, lr, 0.9f, 0.999f, 1e-8f, step + 1, stream));
        RCHK(halign_adam_step(pr->b1, gb1, mb1, vb1, nullptr, hk::kHid, lr, 0.9f, 0.999f, 1e-8f, step + 1, stream));
        RCHK(halign_adam_step(pr->W2, gW2, mW2, vW2, pr->W2b, nW2, lr, 0.9f, 0.999f, 1e-8f, step + 1, stream));
        RCHK(halign_adam_step(pr->b2, gb2, mb2, vb2, nullptr, hk::kEmb, lr, 0.9f, 0.999f, 1e-8f, step + 1, stream));
        if (use_ema) {
            RCHK(ema_step(pr->W1, eW1, nW1));
            RCHK(ema_step(pr->b1, eb1, hk::kHid));
            RCHK(ema_step(pr->W2, eW2, nW2));
            RCHK(ema_step(pr->b2, eb2, hk::kEmb));
        }
    }
    if (use_ema) {   // the averaged parameters become the model
        HCHK(hipMemcpyAsync(pr->W1, eW1, 4 * (size_t)nW1, hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpyAsync(pr->b1, eb1, 4 * (size_t)hk::kHid, hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpyAsync(pr->W2, eW2, 4 * (size_t)nW2, hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpyAsync(pr->b2, eb2, 4 * (size_t)hk::kEmb, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(hk::f32_to_bf16_kernel, dim3(grid_for(nW1, 256, 2048)), dim3(256), 0, st,
                           (const float *)pr->W1, pr->W1b, nW1);
        hipLaunchKernelGGL(hk::f32_to_bf16_kernel, dim3(grid_for(nW2, 256, 2048)), dim3(256), 0, st,
                           (const float *)pr->W2, pr->W2b, nW2);
        HCHK(hipGetLastError());
    }
    if (loss_host) {
        std::vector<float> hl(nsteps);
        HCHK(hipMemcpyAsync(hl.data(), loss, 4 * (size_t)nsteps, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        for (int e = 0; e < opts->epochs; ++e) {
            double s = 0;
            for (int q = 0; q < steps_per_epoch; ++q) s += hl[(size_t)e * steps_per_epoch + q];
            loss_host[e] = (float)(s / std::max(1, steps_per_epoch));
        }
    }
    return HALIGN_OK;
}

int halign_center_learned(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, const halign_model *model,
                          int32_t k, int32_t *cand_host, int32_t *center_host, void *stream) {
    if (!ctx || !center_host || k <= 0) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    RCHK(check_model(model));
    const int N = seqs->n;
    if (N <= 0) return fail(HALIGN_E_INVALID, "empty set");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int kk = std::min<int>(k, N);
    const int CH = 16384;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = (off + bytes + 255) & ~size_t(255); return r; };
    const size_t o_E = take(4 * (size_t)N * hk::kEmb), o_X = take(2 * (size_t)CH * hk::kFeat),
                 o_Hb = take(2 * (size_t)CH * hk::kHid), o_rows = take(4 * (size_t)N), o_u = take(4 * (size_t)N),
                 o_top = take(4 * (size_t)kk), o_sums = take(8 * (size_t)kk);
    RCHK(grow(ctx, ctx->mlp[7], off));
    char *w = (char *)ctx->mlp[7].p;
    float *E = (float *)(w + o_E);
    uint16_t *X = (uint16_t *)(w + o_X), *Hb = (uint16_t *)(w + o_Hb);
    int32_t *rows = (int32_t *)(w + o_rows);
    hipLaunchKernelGGL(hk::iota_kernel, dim3((N + 255) / 256), dim3(256), 0, st, rows, N);
    HCHK(hipGetLastError());
    for (int r0 = 0; r0 < N; r0 += CH) {
        const int nr = std::min(CH, N - r0);
        RCHK(halign_featurize(seqs, rows + r0, nr, X, stream));
        RCHK(halign_mlp_forward(ctx, model, X, nr, nullptr, Hb, E + (size_t)r0 * hk::kEmb, stream));
    }
    int32_t *top = (int32_t *)(w + o_top);
    const int kp = std::min(std::min(ctx->prejudge_cand, 256), N);
    const int np = std::min(ctx->prejudge_part, N);
    if (kp > kk && np > 0) {
        // pre-judge: the top kp by u, scored against a common sample of np
        // partners (evenly spaced indices); the kk best of that sample go on
        RCHK(grow(ctx, ctx->mlp[8], 12 * (size_t)kp + 512));
        int32_t *wide = (int32_t *)ctx->mlp[8].p;
        int64_t *wsum = (int64_t *)((char *)ctx->mlp[8].p + ((4 * (size_t)kp + 255) & ~size_t(255)));
        RCHK(halign_topk_center(ctx, E, N, kp, (float *)(w + o_u), wide, stream));
        std::vector<int32_t> part(np), hw(kp), order(kp);
        for (int q = 0; q < np; ++q) part[q] = (int32_t)((int64_t)q * N / np);
        RCHK(halign_center_judge_sample(ctx, sc, seqs, wide, kp, part.data(), np, wsum, nullptr, stream));
        std::vector<int64_t> hs(kp);
        HCHK(hipMemcpyAsync(hw.data(), wide, 4 * (size_t)kp, hipMemcpyDeviceToHost, st));
        HCHK(hipMemcpyAsync(hs.data(), wsum, 8 * (size_t)kp, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return hs[x] > hs[y] || (hs[x] == hs[y] && hw[x] < hw[y]);
        });
        std::vector<int32_t> sel(kk);
        for (int q = 0; q < kk; ++q) sel[q] = hw[order[q]];
        HCHK(hipMemcpyAsync(top, sel.data(), 4 * (size_t)kk, hipMemcpyHostToDevice, st));
        HCHK(hipStreamSynchronize(st));
    } else {
        RCHK(halign_topk_center(ctx, E, N, kk, (float *)(w + o_u), top, stream));
    }
    int32_t c = -1;
    RCHK(halign_center_judge(ctx, sc, seqs, top, kk, (int64_t *)(w + o_sums), &c, stream));
    if (cand_host) {
        HCHK(hipMemcpyAsync(cand_host, top, 4 * (size_t)kk, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
    }
    *center_host = c;
    return HALIGN_OK;
}

}  // extern "C"

// ===========================================================================
// Nucleotide center star (trie section)
// ===========================================================================
namespace {

// exclusive sums of n int64 values (+ add each) into out, the total into
// *total_dev (device, may be out + n) and *total_host
int scan_i64(halign_ctx *ctx, const int64_t *in, int64_t n, int64_t add, int64_t *out, int64_t *total_dev,
             int64_t *total_host, hipStream_t st) {
    if (n <= hk::kScanTile) {
        hipLaunchKernelGGL(hk::scan_i64_kernel, dim3(1), dim3(1024), 0, st, in, (int)n, add, out, total_dev);
        HCHK(hipGetLastError());
    } else {
        const int64_t nt = (n + hk::kScanTile - 1) / hk::kScanTile;
        if (nt > 0x7fffffff) return fail(HALIGN_E_UNSUPPORTED, "scan of %lld values", (long long)n);
        RCHK(grow(ctx, ctx->sbuf, 16 * (size_t)nt + 256));
        int64_t *part = (int64_t *)ctx->sbuf.p, *poff = part + nt;
        hipLaunchKernelGGL(hk::scan_tile_kernel, dim3((unsigned)nt), dim3(1024), 0, st, in, n, add, out, part);
        hipLaunchKernelGGL(hk::scan_i64_kernel, dim3(1), dim3(1024), 0, st, (const int64_t *)part, (int)nt,
                           (int64_t)0, poff, total_dev);
        hipLaunchKernelGGL(hk::scan_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n,
                           (const int64_t *)poff);
        HCHK(hipGetLastError());
    }
    if (total_host) {   // NULL: the caller reads total_dev itself
        HCHK(hipMemcpyAsync(total_host, total_dev, 8, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
    }
    return HALIGN_OK;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int halign_nuc_align(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, int32_t center, int32_t k,
                     int32_t *score, uint16_t *ins, uint32_t *aligned, int32_t *G, void *stream) {
    if (!ctx || !score || !ins || !aligned) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_scoring(sc));
    RCHK(check_seqs(seqs));
    if (sc->alphabet < 5) return fail(HALIGN_E_UNSUPPORTED, "nucleotide alphabet needs codes 0..4 (A C G T other)");
    if (k < 1 || k > 32) return fail(HALIGN_E_UNSUPPORTED, "segment length %d outside 1..32", k);
    const int N = seqs->n;
    if (center < 0 || center >= N) return fail(HALIGN_E_INVALID, "center %d of %d", center, N);
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t *oh = seqs->offsets_host;
    const int m = (int)(oh[center + 1] - oh[center]);
    const uint8_t *dc = seqs->residues + oh[center];
    Scoring S;
    RCHK(upload_matrix(ctx, sc, st, &S));
    // the code check and the center's copy to the host share one wait
    RCHK(validate_codes(ctx, sc->alphabet, seqs->residues, oh[N], nullptr, 0, st));
    std::vector<uint8_t> c(m);
    if (m > 0) HCHK(hipMemcpyAsync(c.data(), dc, m, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    RCHK(validate_check(ctx));
    // the center's segments, on the host: segment q (k codes 0..3) is indexed
    // when no other such segment has the same string
    const int nsg = m / k;
    std::vector<unsigned long long> key(nsg);
    std::vector<int32_t> segscore(std::max(nsg, 1), 0);
    std::vector<uint8_t> clean(nsg, 1);
    for (int q = 0; q < nsg; ++q) {
        unsigned long long kk = 0;
        for (int t = 0; t < k; ++t) {
            const int b = c[q * k + t];
            if (b > 3) clean[q] = 0;
            kk |= (unsigned long long)(b & 3) << (2 * t);   // base t at bits 2t, 2t + 1
            segscore[q] += sc->matrix_host[b * sc->alphabet + b];
        }
        key[q] = kk;
    }
    std::map<unsigned long long, int> seen;
    for (int q = 0; q < nsg; ++q)
        if (clean[q]) seen[key[q]]++;
    int nidx = 0;
    for (int q = 0; q < nsg; ++q)
        if (clean[q] && seen[key[q]] == 1) ++nidx;
    int lg_t = 6;
    while ((1 << lg_t) < 2 * nidx) ++lg_t;
    const int T = 1 << lg_t;
    std::vector<unsigned long long> tkey(T, 0);
    std::vector<int32_t> tseg(T, -1);
    for (int q = 0; q < nsg; ++q) {
        if (!clean[q] || seen[key[q]] != 1) continue;
        uint32_t h = hk::nuc_hash(key[q], lg_t);
        while (tseg[h] >= 0) h = (h + 1) & (T - 1);
        tkey[h] = key[q];
        tseg[h] = q;
    }
    // scan chunks: sequence x covers the match starts 0 .. n - k in chunks
    std::vector<int64_t> cbase(N + 1, 0);
    for (int x = 0; x < N; ++x) {
        const int64_t w = std::max<int64_t>(0, oh[x + 1] - oh[x] - k + 1);
        cbase[x + 1] = cbase[x] + (w + hk::kNucChunk - 1) / hk::kNucChunk;
    }
    const int64_t nchunk = cbase[N];
    // device tables: segment table, segment scores, chunk bases, two totals,
    // and per chunk: counts (int32), the same widened, offsets (nchunk + 1)
    const size_t o_tk = 0, o_ts = al256(8 * (size_t)T), o_ss = o_ts + al256(4 * (size_t)T),
                 o_cb = o_ss + al256(4 * segscore.size()), o_tot = o_cb + al256(8 * (size_t)(N + 1)),
                 o_lc = o_tot + 128, o_cc = o_tot + 256, o_cw = o_cc + al256(4 * (size_t)nchunk + 4),
                 o_co = o_cw + al256(8 * (size_t)nchunk + 8), tab_bytes = o_co + al256(8 * (size_t)(nchunk + 1));
    RCHK(grow(ctx, ctx->nuctab, tab_bytes));
    char *tb = (char *)ctx->nuctab.p;
    HCHK(hipMemcpyAsync(tb + o_tk, tkey.data(), 8 * (size_t)T, hipMemcpyHostToDevice, st));
    HCHK(hipMemcpyAsync(tb + o_ts, tseg.data(), 4 * (size_t)T, hipMemcpyHostToDevice, st));
    HCHK(hipMemcpyAsync(tb + o_ss, segscore.data(), 4 * segscore.size(), hipMemcpyHostToDevice, st));
    HCHK(hipMemcpyAsync(tb + o_cb, cbase.data(), 8 * (size_t)(N + 1), hipMemcpyHostToDevice, st));
    const int aw = (m + 31) / 32;
    {   // zero the vectors (ins as words plus an odd tail) and G
        const int64_t n16 = (int64_t)N * (m + 1);
        hk::ZeroArgs z{};
        z.p[0] = (uint32_t *)ins;
        z.n[0] = n16 / 2;
        z.p[1] = aligned;
        z.n[1] = (int64_t)N * aw;
        z.p[2] = (uint32_t *)G;
        z.n[2] = G ? m + 1 : 0;
        z.p[3] = (uint32_t *)(tb + o_lc);   // the stretch list counts
        z.n[3] = 3;
        z.tail16 = (n16 & 1) ? ins + (n16 - 1) : nullptr;
        hipLaunchKernelGGL(hk::zero_kernel, dim3(grid_for(z.n[0] + z.n[1], 256, 4096)), dim3(256), 0, st, z);
        HCHK(hipGetLastError());
    }
    hk::NucArgs a{};
    a.res = seqs->residues;
    a.off = seqs->offsets;
    a.nseq = N;
    a.center = dc;
    a.m = m;
    a.k = k;
    a.tkey = (const unsigned long long *)(tb + o_tk);
    a.tseg = (const int32_t *)(tb + o_ts);
    a.lg_t = lg_t;
    a.segscore = (const int32_t *)(tb + o_ss);
    a.mat = S.dmat;
    a.alpha = S.alpha;
    a.go = S.goe - S.ge;
    a.ge = S.ge;
    a.cbase = (const int64_t *)(tb + o_cb);
    a.nchunk = nchunk;
    a.ccount = (int32_t *)(tb + o_cc);
    a.cmoff = (const int64_t *)(tb + o_co);
    a.score = score;
    a.ins = ins;
    a.aligned = aligned;
    a.aw = aw;
    a.G = G;
    a.gskip = center;
    int64_t *dtot = (int64_t *)(tb + o_tot);
    const unsigned cgrid = (unsigned)std::max<int64_t>(1, (nchunk + 255) / 256);
    // wavefront scan: one chunk per wavefront, 16 per workgroup sharing the table
    const unsigned wgrid_scan = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nchunk + 15) / 16, (int64_t)ctx->num_cu * 3));
    if (nchunk > 0) {
        if (k <= hk::kNucWaveMaxK)
            hipLaunchKernelGGL(hk::nuc_count_wave_kernel, dim3(wgrid_scan), dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL(hk::nuc_count_kernel, dim3(cgrid), dim3(256), 0, st, a);
        HCHK(hipGetLastError());
        hipLaunchKernelGGL(hk::widen_kernel, dim3(cgrid), dim3(256), 0, st, (const int32_t *)a.ccount, (int)nchunk,
                           (int64_t *)(tb + o_cw));
        HCHK(hipGetLastError());
    }
    int64_t nmt = 0;
    int64_t *cm = (int64_t *)(tb + o_co);
    RCHK(scan_i64(ctx, (const int64_t *)(tb + o_cw), nchunk, 0, cm, cm + nchunk, &nmt, st));
    // per match (4 x int32) and per slot (matches + N): chain table, stretch
    // descriptor, sequence, sizes and their offsets (+ a total each)
    const int64_t nslot = nmt + N;
    if (nslot >= ((int64_t)1 << 31)) return fail(HALIGN_E_UNSUPPORTED, "%lld segment matches", (long long)nmt);
    const size_t m_q = 0, m_p = al256(4 * (size_t)nmt), m_b = m_p + al256(4 * (size_t)nmt),
                 m_r = m_b + al256(4 * (size_t)nmt), s_tl = m_r + al256(4 * (size_t)nmt),
                 s_d = s_tl + al256(4 * (size_t)nslot), s_x = s_d + al256(16 * (size_t)nslot),
                 s_r = s_x + al256(4 * (size_t)nslot), s_c = s_r + al256(8 * (size_t)nslot),
                 s_ro = s_c + al256(8 * (size_t)nslot), s_co = s_ro + al256(8 * (size_t)nslot + 8),
                 s_sl = s_co + al256(8 * (size_t)nslot + 8), s_bl = s_sl + al256(4 * (size_t)nslot),
                 scr_bytes = s_bl + al256(4 * (size_t)nslot);
    RCHK(grow(ctx, ctx->nucscr, scr_bytes));
    char *sb = (char *)ctx->nucscr.p;
    a.mq = (int32_t *)(sb + m_q);
    a.mp = (int32_t *)(sb + m_p);
    a.mbest = (int32_t *)(sb + m_b);
    a.mpred = (int32_t *)(sb + m_r);
    a.tails = (int32_t *)(sb + s_tl);
    a.sdesc = (int4 *)(sb + s_d);
    a.sseq = (int32_t *)(sb + s_x);
    a.srow = (int64_t *)(sb + s_r);
    a.scode = (int64_t *)(sb + s_c);
    a.nslot = nslot;
    a.slist = (int32_t *)(sb + s_sl);
    a.blist = (int32_t *)(sb + s_bl);
    a.lcount = (int32_t *)(tb + o_lc);
    if (nchunk > 0) {
        if (k <= hk::kNucWaveMaxK)
            hipLaunchKernelGGL(hk::nuc_store_wave_kernel, dim3(wgrid_scan), dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL(hk::nuc_store_kernel, dim3(cgrid), dim3(256), 0, st, a);
        HCHK(hipGetLastError());
    }
    // LDS sized for twice the mean match count (a power of two, 64 ..
    // kChainLdsMax), so several workgroups share a CU; a sequence with more
    // matches is chained in the global arrays
    int cap = 64;
    while (cap < hk::kChainLdsMax && (int64_t)cap * N < 2 * nmt) cap *= 2;
    a.chain_cap = cap;
    hipLaunchKernelGGL(hk::nuc_chain_kernel, dim3((unsigned)N), dim3(64), hk::nuc_chain_lds_bytes(cap, aw), st, a);
    HCHK(hipGetLastError());
    // stretch scratch: row buffers and codes, one region per stretch
    int64_t nrow = 0, ncode = 0;
    int64_t *ro = (int64_t *)(sb + s_ro), *co = (int64_t *)(sb + s_co);
    RCHK(scan_i64(ctx, a.srow, nslot, 0, ro, dtot, nullptr, st));
    RCHK(scan_i64(ctx, a.scode, nslot, 0, co, dtot + 1, nullptr, st));
    {   // both totals in one copy and one wait
        int64_t t2[2] = {0, 0};
        HCHK(hipMemcpyAsync(t2, dtot, 16, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        nrow = t2[0];
        ncode = t2[1];
    }
    const size_t d_co = al256(8 * (size_t)nrow), dp_bytes = d_co + al256(4 * (size_t)ncode);
    RCHK(grow(ctx, ctx->nucdp, dp_bytes));
    a.srowoff = ro;
    a.scodeoff = co;
    a.rows = (int2 *)ctx->nucdp.p;
    a.codes = (uint32_t *)((char *)ctx->nucdp.p + d_co);
    // the stretches: lists sized on the device, grids bounded by the slots
    const int sgrid = (int)std::max<int64_t>(1, std::min<int64_t>((nslot + 255) / 256, (int64_t)ctx->num_cu * 8));
    hipLaunchKernelGGL(hk::nuc_stretch_small_kernel, dim3(sgrid), dim3(256), 0, st, a);
    HCHK(hipGetLastError());
    const int wgrid = (int)std::max<int64_t>(1, std::min<int64_t>(nslot, (int64_t)ctx->num_cu * 16));
    hipLaunchKernelGGL(hk::nuc_stretch_wave_kernel, dim3(wgrid), dim3(64), 0, st, a);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

int halign_nuc_msa(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs, int32_t center, int32_t k,
                   int32_t *score, halign_alloc_fn alloc, void *user, uint8_t **msa, int64_t *width_host,
                   void *stream) {
    if (!ctx || !alloc || !msa || !width_host || !score) return fail(HALIGN_E_INVALID, "bad arguments");
    RCHK(check_seqs(seqs));
    const int N = seqs->n;
    if (center < 0 || center >= N) return fail(HALIGN_E_INVALID, "center %d of %d", center, N);
    hipStream_t st = (hipStream_t)stream;
    const int m = (int)(seqs->offsets_host[center + 1] - seqs->offsets_host[center]);
    const int aw = (m + 31) / 32;
    // vectors, G, col in the ctx's MSA scratch
    const size_t o_ins = 0, o_al = (2 * (size_t)N * (m + 1) + 255) & ~(size_t)255,
                 o_g = o_al + ((4 * (size_t)N * aw + 255) & ~(size_t)255), o_col = o_g + ((4 * (size_t)(m + 1) + 255) & ~(size_t)255),
                 bytes = o_col + 8 * (size_t)(m + 1);
    RCHK(grow(ctx, ctx->msabuf, bytes));
    char *mb = (char *)ctx->msabuf.p;
    uint16_t *ins = (uint16_t *)(mb + o_ins);
    uint32_t *al = (uint32_t *)(mb + o_al);
    int32_t *G = (int32_t *)(mb + o_g);
    int64_t *col = (int64_t *)(mb + o_col);
    RCHK(halign_nuc_align(ctx, sc, seqs, center, k, score, ins, al, G, stream));
    hipLaunchKernelGGL(hk::center_row_kernel, dim3(1), dim3(256), 0, st, ins, al, center, m, aw);
    HCHK(hipGetLastError());
    int64_t width = 0;
    RCHK(merge_offsets(ctx, G, m + 1, col, &width, st));
    uint8_t *out = (uint8_t *)alloc((size_t)N * (size_t)width, user);
    if (!out && width > 0) return fail(HALIGN_E_NOMEM, "allocator returned NULL for %lld bytes", (long long)(N * width));
    RCHK(halign_emit_rows(ctx, seqs, m, ins, al, G, col, width, out, stream));
    *msa = out;
    *width_host = width;
    return HALIGN_OK;
}

}  // extern "C"

// ===========================================================================
// Phylogeny (NJ section, Fig. 4): p-distances, neighbour joining, the sampled
// clustering and the merged tree
// ===========================================================================
namespace {

inline size_t al256z(size_t b) { return (b + 255) & ~(size_t)255; }

// The distance launch: whole width per tile, or, when the tiles are too few
// to fill the chip several times over (under 8,192) and the MSA is wide,
// column slices (256 or 1,024 columns and up) added atomically into zeroed
// counts and a finalize pass.  nout:
// outputs the groups address (for the counts).
int pdist_launch(halign_ctx *ctx, hk::PdArgs a, int64_t tiles, int64_t nout, hipStream_t st) {
    int64_t nslice = 1;
    // few tiles: slices of 256 columns, about 256 workgroups in all (each
    // slice's atomics cost more than a further slice hides); more tiles:
    // slices of 1,024 columns up to 8,192 workgroups
    if (tiles < 64 && a.width > 512)
        nslice = std::min<int64_t>((a.width + 255) / 256, (256 + tiles - 1) / tiles);
    else if (tiles < 8192 && a.width > 2048)
        nslice = std::min<int64_t>((a.width + 1023) / 1024, (8192 + tiles - 1) / tiles);
    a.nslice = 1;
    a.cslice = a.width;
    a.acc = nullptr;
    a.mode = 0;
    if (nslice > 1) {
        a.nslice = (int)nslice;
        a.cslice = (((a.width + nslice - 1) / nslice) + hk::kPdChunk - 1) / hk::kPdChunk * hk::kPdChunk;
        RCHK(grow(ctx, ctx->njacc, 8 * (size_t)nout));
        a.acc = (int32_t *)ctx->njacc.p;
        RCHK(launch_fill((uint32_t *)a.acc, 0u, 2 * nout, st));
        a.mode = 1;
        // under four workgroups per CU the next pass's loads go out early
        if (tiles * nslice < 1024)
            hipLaunchKernelGGL(hk::pdist_kernel<true>, dim3((unsigned)(tiles * nslice)), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(hk::pdist_kernel<false>, dim3((unsigned)(tiles * nslice)), dim3(256), 0, st, a);
        HCHK(hipGetLastError());
        a.mode = 2;
    }
    hipLaunchKernelGGL(hk::pdist_kernel<false>, dim3((unsigned)tiles), dim3(256), 0, st, a);
    HCHK(hipGetLastError());
    return HALIGN_OK;
}

// Upload rows and the group table, then one pdist launch over every group's
// tiles.  Synchronises the stream after the upload (the host vectors may go).
int pdist_groups(halign_ctx *ctx, const uint8_t *msa, int64_t width, const std::vector<int32_t> &rows,
                 std::vector<hk::PdGroup> &groups, double *D, int32_t *mism, int32_t *comp, hipStream_t st) {
    int64_t tiles = 0;
    for (auto &g : groups) {
        g.tiles_b = (g.nb + hk::kPdTile - 1) / hk::kPdTile;
        g.tile0 = tiles;
        tiles += (int64_t)((g.na + hk::kPdTile - 1) / hk::kPdTile) * g.tiles_b;
    }
    if (tiles == 0) return HALIGN_OK;
    if (tiles > 0x7fffffff) return fail(HALIGN_E_UNSUPPORTED, "%lld distance tiles", (long long)tiles);
    const size_t o_g = al256z(4 * rows.size());
    RCHK(grow(ctx, ctx->njrows, o_g + sizeof(hk::PdGroup) * groups.size()));
    char *b = (char *)ctx->njrows.p;
    if (!rows.empty()) HCHK(hipMemcpyAsync(b, rows.data(), 4 * rows.size(), hipMemcpyHostToDevice, st));
    HCHK(hipMemcpyAsync(b + o_g, groups.data(), sizeof(hk::PdGroup) * groups.size(), hipMemcpyHostToDevice, st));
    int64_t nout = 0;
    for (auto &g : groups)
        if (g.na > 0 && g.nb > 0) nout = std::max<int64_t>(nout, g.o + (int64_t)(g.na - 1) * g.ld + g.nb);
    hk::PdArgs a{msa, width, (const int32_t *)b, (const hk::PdGroup *)(b + o_g), (int)groups.size(), D, mism, comp};
    RCHK(pdist_launch(ctx, a, tiles, nout, st));
    HCHK(hipStreamSynchronize(st));
    return HALIGN_OK;
}

// Neighbour joining over groups (each D at its d0 in dbase, modified); the
// trees come back to the host: tree g at t0 = 2 * (sum of earlier n) + g.
// The one-workgroup joins of several problems (each group's offsets filled
// in), enqueued on st; nj_groups_finish copies the trees to the host.
struct NjLaunch {
    size_t o_p = 0, o_b = 0, o_nd = 0;
    int64_t nt = 0;
    size_t G = 0;
};

int nj_groups_launch(halign_ctx *ctx, std::vector<hk::NjGroup> &groups, double *dbase, NjLaunch &L, hipStream_t st) {
    int64_t ns = 0, nt = 0;
    int nmax = 0;
    for (auto &g : groups) {
        g.s0 = ns;
        g.t0 = nt;
        ns += g.n;
        nt += 2 * (int64_t)g.n + 1;
        nmax = std::max(nmax, g.n);
    }
    const size_t G = groups.size();
    const size_t o_r = 0, o_id = al256z(8 * ns), o_p = o_id + al256z(4 * ns), o_b = o_p + al256z(4 * nt),
                 o_nd = o_b + al256z(8 * nt), o_g = o_nd + al256z(4 * G), o_act = o_g + al256z(sizeof(hk::NjGroup) * G),
                 bytes = o_act + al256z(ns);
    RCHK(grow(ctx, ctx->njS, bytes));
    char *b = (char *)ctx->njS.p;
    HCHK(hipMemcpyAsync(b + o_g, groups.data(), sizeof(hk::NjGroup) * G, hipMemcpyHostToDevice, st));
    hk::NjArgs a{(const hk::NjGroup *)(b + o_g), dbase, (double *)(b + o_r), (uint8_t *)(b + o_act),
                 (int32_t *)(b + o_id), (int32_t *)(b + o_p), (double *)(b + o_b), (int32_t *)(b + o_nd)};
    const int bs = nmax > 128 ? 1024 : 256;
    const size_t lds = hk::nj_lds_bytes(nmax);   // at most 55 KiB
    hipLaunchKernelGGL(hk::nj_kernel, dim3((unsigned)G), dim3(bs), lds, st, a, lds > 0 ? 1 : 0);
    HCHK(hipGetLastError());
    L.o_p = o_p;
    L.o_b = o_b;
    L.o_nd = o_nd;
    L.nt = nt;
    L.G = G;
    return HALIGN_OK;
}

int nj_groups_finish(halign_ctx *ctx, const NjLaunch &L, std::vector<int32_t> &parent, std::vector<double> &blen,
                     std::vector<int32_t> &nodes, hipStream_t st) {
    char *b = (char *)ctx->njS.p;
    parent.resize(L.nt);
    blen.resize(L.nt);
    nodes.resize(L.G);
    HCHK(hipMemcpyAsync(parent.data(), b + L.o_p, 4 * L.nt, hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(blen.data(), b + L.o_b, 8 * L.nt, hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(nodes.data(), b + L.o_nd, 4 * L.G, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    return HALIGN_OK;
}

int nj_groups(halign_ctx *ctx, std::vector<hk::NjGroup> &groups, double *dbase, std::vector<int32_t> &parent,
              std::vector<double> &blen, std::vector<int32_t> &nodes, hipStream_t st) {
    NjLaunch L;
    RCHK(nj_groups_launch(ctx, groups, dbase, L, st));
    return nj_groups_finish(ctx, L, parent, blen, nodes, st);
}

// Problems above this many nodes are joined over the whole chip (three
// launches per join); smaller ones one workgroup each, all in one launch.
constexpr int kNjBigMin = 256;

// Neighbour joining of one problem over the chip: D (device, n x n, modified);
// the tree to the host (2n + 1 entries).
int nj_big(halign_ctx *ctx, double *D, int n, std::vector<int32_t> &parent, std::vector<double> &blen, int *nodes,
           hipStream_t st) {
    const int64_t nn = (int64_t)n * n;
    const int nparts = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (nn + 255) / 256));
    const size_t nt = 2 * (size_t)n + 1;
    const size_t o_r = 0, o_id = al256z(8 * (size_t)n), o_p = o_id + al256z(4 * (size_t)n), o_b = o_p + al256z(4 * nt),
                 o_part = o_b + al256z(8 * nt), o_pd = o_part + al256z(sizeof(hk::NjBest) * nparts),
                 o_ctrl = o_pd + al256z(8 * (size_t)nparts),
                 o_nodes = o_ctrl + 256, o_act = o_nodes + 256, bytes = o_act + al256z(n);
    RCHK(grow(ctx, ctx->njB, bytes));
    char *b = (char *)ctx->njB.p;
    hk::NjBigArgs a{n, D, (double *)(b + o_r), (uint8_t *)(b + o_act), (int32_t *)(b + o_id), (int32_t *)(b + o_p),
                    (double *)(b + o_b), (hk::NjBest *)(b + o_part), (double *)(b + o_pd), nparts, (hk::NjCtrl *)(b + o_ctrl)};
    const unsigned rg = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(hk::nj_big_init_kernel, dim3(rg), dim3(256), 0, st, a);
    HCHK(hipGetLastError());
    for (int t = 0; t < n - 3; ++t) {
        hipLaunchKernelGGL(hk::nj_big_rows_kernel, dim3((unsigned)((n + hk::kNjRowsCols - 1) / hk::kNjRowsCols)),
                           dim3(256), 0, st, a);
        hipLaunchKernelGGL(hk::nj_big_q_kernel, dim3((unsigned)nparts), dim3(256), 0, st, a);
        hipLaunchKernelGGL(hk::nj_big_join_kernel, dim3(1), dim3(256), 0, st, a);
    }
    HCHK(hipGetLastError());
    hipLaunchKernelGGL(hk::nj_big_finish_kernel, dim3(1), dim3(1), 0, st, a, (int32_t *)(b + o_nodes));
    HCHK(hipGetLastError());
    parent.resize(nt);
    blen.resize(nt);
    int32_t nd = 0;
    HCHK(hipMemcpyAsync(parent.data(), b + o_p, 4 * nt, hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(blen.data(), b + o_b, 8 * nt, hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(&nd, b + o_nodes, 4, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    *nodes = nd;
    return HALIGN_OK;
}

// labels[i] = nearest of the nb columns of D (na x nb, device), to the host
// labels[g][i] = nearest of the nb columns of group g's block (D + o, na x
// nb): every group's launch, then one copy to the host
int nearest_groups(halign_ctx *ctx, const double *D, const std::vector<hk::PdGroup> &gr,
                   std::vector<std::vector<int32_t>> &label, hipStream_t st) {
    size_t tot = 0;
    for (auto &g : gr) tot += (size_t)std::max(0, g.na);
    RCHK(grow(ctx, ctx->njS, al256z(4 * tot + 4)));
    int32_t *lab = (int32_t *)ctx->njS.p;
    size_t at = 0;
    for (auto &g : gr) {
        if (g.na > 0 && g.nb > 0)
            hipLaunchKernelGGL(hk::nearest_kernel, dim3((unsigned)((g.na + 255) / 256)), dim3(256), 0, st, D + g.o,
                               (int64_t)g.nb, g.na, g.nb, lab + at);
        at += (size_t)std::max(0, g.na);
    }
    HCHK(hipGetLastError());
    std::vector<int32_t> all(tot);
    if (tot > 0) HCHK(hipMemcpyAsync(all.data(), lab, 4 * tot, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    label.resize(gr.size());
    at = 0;
    for (size_t gi = 0; gi < gr.size(); ++gi) {
        const int na = std::max(0, gr[gi].na);
        label[gi].assign(all.begin() + at, all.begin() + at + na);
        at += na;
    }
    return HALIGN_OK;
}

int nearest_host(halign_ctx *ctx, const double *D, int na, int nb, std::vector<int32_t> &label, hipStream_t st) {
    RCHK(grow(ctx, ctx->njS, al256z(4 * (size_t)na)));
    int32_t *lab = (int32_t *)ctx->njS.p;
    hipLaunchKernelGGL(hk::nearest_kernel, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, st, D, (int64_t)nb, na,
                       nb, lab);
    HCHK(hipGetLastError());
    label.resize(na);
    HCHK(hipMemcpyAsync(label.data(), lab, 4 * (size_t)na, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    return HALIGN_OK;
}

}  // namespace

extern "C" {

int halign_pdist(halign_ctx *ctx, const uint8_t *msa, int32_t n, int64_t width, const int32_t *a_rows, int32_t na,
                 const int32_t *b_rows, int32_t nb, double *D, int32_t *mism, int32_t *comp, void *stream) {
    if (!ctx || n < 0 || width < 0 || na < 0 || nb < 0 || ((int64_t)na * nb > 0 && (!D || (!msa && width > 0))))
        return fail(HALIGN_E_INVALID, "bad arguments");
    if ((!a_rows && na > n) || (!b_rows && nb > n)) return fail(HALIGN_E_INVALID, "row count above n");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if ((int64_t)na * nb == 0) return HALIGN_OK;
    // the row lists: given ones copied into the ctx buffer behind an identity prefix
    std::vector<int32_t> rows;
    if (!a_rows || !b_rows) {
        rows.resize(std::max(a_rows ? 0 : na, b_rows ? 0 : nb));
        for (size_t x = 0; x < rows.size(); ++x) rows[x] = (int32_t)x;
    }
    const int64_t ida = (int64_t)rows.size();
    std::vector<hk::PdGroup> groups(1);
    hk::PdGroup &g = groups[0];
    g.a0 = a_rows ? ida : 0;
    g.b0 = b_rows ? ida + (a_rows ? na : 0) : 0;
    g.na = na;
    g.nb = nb;
    g.o = 0;
    g.ld = nb;
    g.diag0 = 0;
    rows.resize(ida + (a_rows ? na : 0) + (b_rows ? nb : 0));   // placeholders, filled on the device below
    // upload the identity part with the table, then the given lists device to device
    int64_t tiles = (int64_t)((na + hk::kPdTile - 1) / hk::kPdTile) * ((nb + hk::kPdTile - 1) / hk::kPdTile);
    if (tiles > 0x7fffffff) return fail(HALIGN_E_UNSUPPORTED, "%lld distance tiles", (long long)tiles);
    g.tiles_b = (nb + hk::kPdTile - 1) / hk::kPdTile;
    g.tile0 = 0;
    const size_t o_g = al256z(4 * rows.size());
    RCHK(grow(ctx, ctx->njrows, o_g + sizeof(hk::PdGroup)));
    char *b = (char *)ctx->njrows.p;
    if (ida > 0) HCHK(hipMemcpyAsync(b, rows.data(), 4 * (size_t)ida, hipMemcpyHostToDevice, st));
    if (a_rows) HCHK(hipMemcpyAsync(b + 4 * g.a0, a_rows, 4 * (size_t)na, hipMemcpyDeviceToDevice, st));
    if (b_rows) HCHK(hipMemcpyAsync(b + 4 * g.b0, b_rows, 4 * (size_t)nb, hipMemcpyDeviceToDevice, st));
    HCHK(hipMemcpyAsync(b + o_g, groups.data(), sizeof(hk::PdGroup), hipMemcpyHostToDevice, st));
    hk::PdArgs a{msa, width, (const int32_t *)b, (const hk::PdGroup *)(b + o_g), 1, D, mism, comp};
    RCHK(pdist_launch(ctx, a, tiles, (int64_t)na * nb, st));
    HCHK(hipStreamSynchronize(st));   // the host vectors above were copied from
    return HALIGN_OK;
}

int halign_nj(halign_ctx *ctx, const double *D, int32_t n, int32_t *parent_host, double *blen_host, int32_t *nodes,
              void *stream) {
    if (!ctx || n < 1 || !D || !parent_host || !blen_host || !nodes) return fail(HALIGN_E_INVALID, "bad arguments");
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = 8 * (size_t)n * n;
    RCHK(grow(ctx, ctx->njD, bytes));
    HCHK(hipMemcpyAsync(ctx->njD.p, D, bytes, hipMemcpyDeviceToDevice, st));
    std::vector<int32_t> parent, nd;
    std::vector<double> blen;
    if (n > kNjBigMin) {
        int nn = 0;
        RCHK(nj_big(ctx, (double *)ctx->njD.p, n, parent, blen, &nn, st));
        nd.assign(1, nn);
    } else {
        std::vector<hk::NjGroup> groups(1);
        groups[0].n = n;
        groups[0].d0 = 0;
        RCHK(nj_groups(ctx, groups, (double *)ctx->njD.p, parent, blen, nd, st));
    }
    memcpy(parent_host, parent.data(), 4 * (size_t)nd[0]);
    memcpy(blen_host, blen.data(), 8 * (size_t)nd[0]);
    *nodes = nd[0];
    return HALIGN_OK;
}

int halign_nj_tree(halign_ctx *ctx, const uint8_t *msa, int32_t n, int64_t width, const int32_t *perm_host,
                   int32_t *parent_host, double *blen_host, int32_t *nodes, void *stream) {
    if (!ctx || n < 1 || width < 0 || (!msa && width > 0) || !perm_host || !parent_host || !blen_host || !nodes)
        return fail(HALIGN_E_INVALID, "bad arguments");
    {   // a permutation of 0 .. n-1
        std::vector<char> seen(n, 0);
        for (int t = 0; t < n; ++t) {
            const int v = perm_host[t];
            if (v < 0 || v >= n || seen[v]) return fail(HALIGN_E_INVALID, "perm is not a permutation of 0..%d", n - 1);
            seen[v] = 1;
        }
    }
    HCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int N = n, S = (N + 9) / 10;
    std::vector<int32_t> seed(perm_host, perm_host + S);
    // every row against the sample: nearest seed
    std::vector<int32_t> label;
    {
        std::vector<int32_t> rows(N + S);
        for (int x = 0; x < N; ++x) rows[x] = x;
        for (int c = 0; c < S; ++c) rows[N + c] = seed[c];
        std::vector<hk::PdGroup> gr(1);
        gr[0] = hk::PdGroup{0, N, N, S, 0, S, 0, 0, 0};
        RCHK(grow(ctx, ctx->njD, 8 * (size_t)N * S));
        RCHK(pdist_groups(ctx, msa, width, rows, gr, (double *)ctx->njD.p, nullptr, nullptr, st));
        RCHK(nearest_host(ctx, (const double *)ctx->njD.p, N, S, label, st));
    }
    int K = S;
    std::vector<int> size(N + 1, 0);
    for (int x = 0; x < N; ++x) size[label[x]]++;
    if (ctx->progress) fprintf(stderr, "halign_nj_tree: %d rows labelled against %d seeds\n", N, S);
    // clusters of fewer than 3 rows join the cluster of the nearest seed
    bool small = false;
    for (int c = 0; c < K; ++c) small = small || (size[c] > 0 && size[c] < 3);
    if (small && K > 1) {
        std::vector<int32_t> rows(S);
        for (int c = 0; c < S; ++c) rows[c] = seed[c];
        std::vector<hk::PdGroup> gr(1);
        gr[0] = hk::PdGroup{0, 0, S, S, 0, S, 0, 0, 0};
        RCHK(grow(ctx, ctx->njD, 8 * (size_t)S * S));
        RCHK(pdist_groups(ctx, msa, width, rows, gr, (double *)ctx->njD.p, nullptr, nullptr, st));
        std::vector<int> to(K);   // cluster a small one moved to (itself when kept)
        for (int c = 0; c < K; ++c) to[c] = c;
        // the seeds' distances to the host in one copy
        std::vector<double> dss((size_t)S * S);
        HCHK(hipMemcpyAsync(dss.data(), ctx->njD.p, 8 * (size_t)S * S, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        for (int c = 0; c < K; ++c) {
            if (size[c] == 0 || size[c] >= 3) continue;
            const double *drow = dss.data() + (size_t)c * S;
            double best = 0.0;
            int bc = -1;
            for (int e = 0; e < K; ++e) {
                if (e == c || size[e] == 0) continue;
                if (bc < 0 || drow[e] < best) {
                    best = drow[e];
                    bc = e;
                }
            }
            if (bc < 0) continue;
            to[c] = bc;   // the rows follow at the end, along the chain of moves
            size[bc] += size[c];
            size[c] = 0;
        }
        for (int x = 0; x < N; ++x) {
            int c = label[x];
            while (to[c] != c) c = to[c];
            label[x] = c;
        }
    }
    {   // renumber the clusters left, in order
        std::vector<int> map(K);
        int K2 = 0;
        for (int c = 0; c < K; ++c) map[c] = size[c] > 0 ? K2++ : -1;
        for (int c = 0; c < K; ++c)
            if (map[c] >= 0) {
                seed[map[c]] = seed[c];
                size[map[c]] = size[c];
            }
        for (int x = 0; x < N; ++x) label[x] = map[label[x]];
        K = K2;
    }
    // clusters of more than ceil(N / 10) rows are divided until none is left:
    // among their first ceil(size / 10) rows in permutation order (nearest),
    // or in runs of ceil(N / 10) rows in permutation order when one seed
    // takes them all; empty clusters are dropped after each pass
    for (;;) {
        bool big = false;
        for (int c = 0; c < K; ++c) big = big || size[c] > S;
        if (!big) break;
        std::vector<int32_t> nseed, nlab(N);
        // the big clusters' rows and new seeds, one distance group each
        std::vector<int32_t> rows;
        std::vector<hk::PdGroup> gr;
        std::vector<int> gbase;                     // per group: its cluster's first new seed
        std::vector<std::vector<int32_t>> mem(K);
        for (int x = 0; x < N; ++x)
            if (size[label[x]] > S) mem[label[x]].push_back(x);
        int64_t dtot = 0;
        std::vector<int32_t> kpos(K, -1);   // a kept cluster's seed position in nseed
        for (int c = 0; c < K; ++c) {
            if (size[c] <= S) {
                kpos[c] = (int32_t)nseed.size();
                nseed.push_back(seed[c]);
                continue;
            }
            const int nsd = (size[c] + 9) / 10;
            const int base = (int)nseed.size();
            for (int t = 0; t < N && (int)nseed.size() - base < nsd; ++t)
                if (label[perm_host[t]] == c) nseed.push_back(perm_host[t]);
            const int64_t r0 = (int64_t)rows.size();
            rows.insert(rows.end(), mem[c].begin(), mem[c].end());
            rows.insert(rows.end(), nseed.begin() + base, nseed.end());
            const int nm = (int)mem[c].size();
            gr.push_back(hk::PdGroup{r0, r0 + nm, nm, nsd, dtot, nsd, 0, 0, 0});
            gbase.push_back(base);
            dtot += (int64_t)nm * nsd;
        }
        for (int x = 0; x < N; ++x)   // rows of kept clusters: their seed's position
            if (kpos[label[x]] >= 0) nlab[x] = kpos[label[x]];
        RCHK(grow(ctx, ctx->njD, 8 * (size_t)dtot));
        RCHK(pdist_groups(ctx, msa, width, rows, gr, (double *)ctx->njD.p, nullptr, nullptr, st));
        // the nearest new seed of every row of each divided cluster, on the GPU
        // (one launch per cluster, one copy back)
        std::vector<std::vector<int32_t>> glab(gr.size());
        RCHK(nearest_groups(ctx, (const double *)ctx->njD.p, gr, glab, st));
        // nearest new seed per row (ties to the earlier), or runs in permutation order
        std::vector<int> remap(nseed.size(), -1);
        {
            // rebuild nseed in order, replacing each divided cluster's seeds by
            // runs where needed
            size_t gi = 0;
            std::vector<int32_t> res;
            int at = 0;   // position in nseed
            for (int c = 0; c < K; ++c) {
                if (size[c] <= S) {
                    remap[at] = (int)res.size();
                    res.push_back(nseed[at]);
                    ++at;
                    continue;
                }
                const hk::PdGroup &g = gr[gi];
                const int nm = g.na, nsd = g.nb, base = gbase[gi];
                const std::vector<int32_t> &lab = glab[gi];
                bool split = false;
                for (int t = 1; t < nm; ++t) split = split || lab[t] != lab[0];
                if (split) {
                    const int r0 = (int)res.size();
                    for (int e = 0; e < nsd; ++e) res.push_back(nseed[base + e]);
                    for (int t = 0; t < nm; ++t) nlab[mem[c][t]] = r0 + lab[t];
                } else {
                    int cnt = 0;
                    for (int t = 0; t < N; ++t) {
                        const int x = perm_host[t];
                        if (label[x] != c) continue;
                        if (cnt % S == 0) res.push_back(x);
                        nlab[x] = (int32_t)res.size() - 1;
                        ++cnt;
                    }
                }
                at += nsd;
                ++gi;
            }
            // the kept clusters' labels were set against nseed positions: move them
            for (int x = 0; x < N; ++x)
                if (size[label[x]] <= S) nlab[x] = remap[nlab[x]];
            nseed.swap(res);
        }
        // drop empty clusters, keeping the order
        const int NK = (int)nseed.size();
        std::vector<int> sz(NK, 0), map(NK);
        for (int x = 0; x < N; ++x) sz[nlab[x]]++;
        int K2 = 0;
        for (int c = 0; c < NK; ++c) map[c] = sz[c] > 0 ? K2++ : -1;
        seed.assign(K2, 0);
        size.assign(std::max(N + 1, K2), 0);
        for (int c = 0; c < NK; ++c)
            if (map[c] >= 0) {
                seed[map[c]] = nseed[c];
                size[map[c]] = sz[c];
            }
        for (int x = 0; x < N; ++x) label[x] = map[nlab[x]];
        K = K2;
        if (ctx->progress) fprintf(stderr, "halign_nj_tree: divide pass, %d clusters\n", K);
    }
    // distance matrices: each cluster over its rows (row order), then the seeds
    std::vector<int32_t> rows;
    std::vector<int64_t> coff(K + 1, 0);
    std::vector<int> csize(K, 0);
    for (int x = 0; x < N; ++x) csize[label[x]]++;
    for (int c = 0; c < K; ++c) coff[c + 1] = coff[c] + csize[c];
    rows.resize(N + K);
    {
        std::vector<int64_t> at(coff.begin(), coff.end() - 1);
        for (int x = 0; x < N; ++x) rows[at[label[x]]++] = x;
        for (int c = 0; c < K; ++c) rows[N + c] = seed[c];
    }
    if (ctx->progress) {
        int mx = 0;
        for (int c = 0; c < K; ++c) mx = std::max(mx, csize[c]);
        fprintf(stderr, "halign_nj_tree: %d rows, %d clusters (largest %d rows), %d seeds joined last\n", N, K, mx, K);
    }
    std::vector<hk::PdGroup> gr(K + 1);
    std::vector<hk::NjGroup> ng(K + 1);
    int64_t dtot = 0;
    for (int c = 0; c <= K; ++c) {
        const int64_t r0 = c < K ? coff[c] : N;
        const int sz = c < K ? csize[c] : K;
        gr[c] = hk::PdGroup{r0, r0, sz, sz, dtot, sz, 1, 0, 0};
        ng[c].n = sz;
        ng[c].d0 = dtot;
        dtot += (int64_t)sz * sz;
    }
    // clusters of at most 64 rows, consecutive in `rows`, share 64-row tiles:
    // one square group over the span (its pairs across clusters are computed
    // and not used), each cluster's block then copied to its own matrix; a
    // distance depends on its two rows alone, so the values are the same
    std::vector<hk::PdGroup> gp;
    std::vector<hk::PdExtract> ext;
    int64_t ttot = dtot;
    for (int c = 0; c < K;) {
        if (csize[c] > hk::kPdTile) {
            gp.push_back(gr[c++]);
            continue;
        }
        const int first = c;
        const int64_t R0 = coff[c];
        int span = 0;
        while (c < K && csize[c] <= hk::kPdTile && span + csize[c] <= hk::kPdTile) span += csize[c++];
        if (c - first == 1) {
            gp.push_back(gr[first]);
            continue;
        }
        gp.push_back(hk::PdGroup{R0, R0, span, span, ttot, span, 1, 0, 0});
        for (int q = first; q < c; ++q)
            if (csize[q] > 0) {
                const int64_t off = coff[q] - R0;
                ext.push_back(hk::PdExtract{ttot + off * span + off, span, ng[q].d0, csize[q]});
            }
        ttot += (int64_t)span * span;
    }
    gp.push_back(gr[K]);
    RCHK(grow(ctx, ctx->njD, 8 * (size_t)ttot));
    RCHK(pdist_groups(ctx, msa, width, rows, gp, (double *)ctx->njD.p, nullptr, nullptr, st));
    if (!ext.empty()) {
        RCHK(grow(ctx, ctx->njrows, sizeof(hk::PdExtract) * ext.size()));
        HCHK(hipMemcpyAsync(ctx->njrows.p, ext.data(), sizeof(hk::PdExtract) * ext.size(), hipMemcpyHostToDevice,
                            st));
        hipLaunchKernelGGL(hk::pd_extract_kernel, dim3((unsigned)ext.size()), dim3(256), 0, st,
                           (double *)ctx->njD.p, (const hk::PdExtract *)ctx->njrows.p);
        HCHK(hipGetLastError());
        HCHK(hipStreamSynchronize(st));   // the small joins may run on another stream
    }
    // the joins: small problems in one launch, large ones over the chip; tree
    // g at tp/tb offset ng[g].t0 (2n + 1 entries each), node count tn[g]
    std::vector<int32_t> tp, tn(K + 1);
    std::vector<double> tb;
    {
        std::vector<hk::NjGroup> small;
        std::vector<int> sidx;
        int64_t nt = 0;
        for (int c = 0; c <= K; ++c) {
            ng[c].t0 = nt;
            nt += 2 * (int64_t)ng[c].n + 1;
            if (ng[c].n <= kNjBigMin) {
                small.push_back(ng[c]);
                sidx.push_back(c);
            }
        }
        tp.assign(nt, 0);
        tb.assign(nt, 0.0);
        // the small problems on a second stream, beside the chip-wide joins
        // (their matrices, scratch and trees are disjoint; the distances are
        // complete, pdist_groups having synchronised st)
        bool any_big = false;
        for (int c = 0; c <= K; ++c) any_big = any_big || ng[c].n > kNjBigMin;
        hipStream_t sst = st;
        if (any_big && !small.empty()) {
            if (!ctx->aux_stream) HCHK(hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking));
            sst = ctx->aux_stream;
        }
        NjLaunch L;
        if (!small.empty()) RCHK(nj_groups_launch(ctx, small, (double *)ctx->njD.p, L, sst));
        for (int c = 0; c <= K; ++c) {
            if (ng[c].n <= kNjBigMin) continue;
            if (ctx->progress) fprintf(stderr, "halign_nj_tree: joining %d nodes over the chip\n", ng[c].n);
            std::vector<int32_t> bp;
            std::vector<double> bb;
            int nn = 0;
            const int rc = nj_big(ctx, (double *)ctx->njD.p + ng[c].d0, ng[c].n, bp, bb, &nn, st);
            if (rc != HALIGN_OK) {   // the small joins finish before the scratch can be reused
                if (sst != st) (void)hipStreamSynchronize(sst);
                return rc;
            }
            std::copy(bp.begin(), bp.end(), tp.begin() + ng[c].t0);
            std::copy(bb.begin(), bb.end(), tb.begin() + ng[c].t0);
            tn[c] = nn;
        }
        if (!small.empty()) {
            std::vector<int32_t> sp, sn;
            std::vector<double> sb;
            RCHK(nj_groups_finish(ctx, L, sp, sb, sn, sst));
            for (size_t q = 0; q < small.size(); ++q) {
                const int c = sidx[q];
                std::copy(sp.begin() + small[q].t0, sp.begin() + small[q].t0 + 2 * ng[c].n + 1, tp.begin() + ng[c].t0);
                std::copy(sb.begin() + small[q].t0, sb.begin() + small[q].t0 + 2 * ng[c].n + 1, tb.begin() + ng[c].t0);
                tn[c] = sn[q];
            }
        }
        if (ctx->progress) fprintf(stderr, "halign_nj_tree: %zu problems joined in one launch\n", small.size());
    }
    // the merge, node numbering as documented
    int next = N;
    std::vector<int> croot(K);
    for (int c = 0; c < K; ++c) {
        const int nn = tn[c], sz = csize[c];
        const int32_t *lp = tp.data() + ng[c].t0;
        const double *lb = tb.data() + ng[c].t0;
        const int32_t *mem = rows.data() + coff[c];
        for (int v = 0; v < nn; ++v) {
            const int gv = v < sz ? mem[v] : next + v - sz;
            const int pv = lp[v];
            parent_host[gv] = pv < 0 ? -1 : (pv < sz ? mem[pv] : next + pv - sz);
            blen_host[gv] = lb[v];
            if (pv < 0) croot[c] = gv;
        }
        next += nn - sz;
    }
    {
        const int nn = tn[K];
        const int32_t *lp = tp.data() + ng[K].t0;
        const double *lb = tb.data() + ng[K].t0;
        for (int v = 0; v < nn; ++v) {
            const int gv = v < K ? croot[v] : next + v - K;
            const int pv = lp[v];
            parent_host[gv] = pv < 0 ? -1 : (pv < K ? croot[pv] : next + pv - K);
            blen_host[gv] = pv < 0 ? 0.0 : lb[v];
        }
        next += nn - K;
    }
    *nodes = next;
    return HALIGN_OK;
}

}  // extern "C"
