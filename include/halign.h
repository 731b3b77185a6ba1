/*
 * halign.h -- C ABI of the MI355X (gfx950) center-star protein MSA library.
 *
 * The library computes the protein path of HAlign-II (Wan & Zou, arXiv
 * 1704.00878, Methods, "Smith-Waterman algorithm for protein sequences with
 * Spark" and Fig. 3):
 *   1. local affine-gap Smith-Waterman of every sequence against a center
 *      sequence, with traceback (eq. 1, eq. 2; the traceback runs from the
 *      highest cell back to the first zero cell);
 *   2. the first reduction of Fig. 3: the inserted-space vectors of all
 *      pairwise alignments are merged into the longest center-star sequence;
 *   3. the second map step: each MSA row is built from its inserted-space
 *      vector and its own sequence.
 * plus center selection (exact sum of scores, or a learned proposer judged
 * exactly) and the avg SP metric of the Results section.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers unless the parameter name ends in _host.
 *  - All buffers belong to the caller; the library never frees them.
 *    Scratch memory (traceback codes, plans) is owned by the halign_ctx.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*; NULL = the null stream).  Outputs are valid once that stream
 *    synchronises.  Calls that return a value through a _host pointer
 *    synchronise the stream before returning.
 *  - Every call returns an int status: HALIGN_OK or a negative code; the
 *    message of the last failure on this thread is halign_last_error().
 *  - No C++ exception crosses this boundary.
 *  - One ctx must not be used from two threads or two streams at once.
 *
 * Residues are codes 0..alphabet-1 (NCBI order ARNDCQEGHILKMFPSTWYVBZX* for
 * the 24-letter protein alphabet); MSA gap bytes are HALIGN_GAP (255).
 */
#ifndef HALIGN_H
#define HALIGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HALIGN_OK              0
#define HALIGN_E_INVALID      -1  /* bad argument: sizes, codes, offsets, NULL */
#define HALIGN_E_NOMEM        -2  /* device allocation failed or cap exceeded */
#define HALIGN_E_DEVICE       -3  /* HIP runtime error */
#define HALIGN_E_UNSUPPORTED  -4  /* outside the supported envelope (see below) */
#define HALIGN_E_OVERFLOW     -5  /* a score bound exceeds the integer range */

#define HALIGN_GAP 255

/* flags of halign_sw_batch */
#define HALIGN_SCORE_ONLY  0u     /* score (and end cell when cells != NULL) */
#define HALIGN_TRACEBACK   1u     /* also walk back: cells, ins, aligned */

/* capture the call's launch sequence in a hipGraph and replay it on later
 * calls with identical arguments (same pointers, sizes, offsets, scoring) */
#define HALIGN_GRAPH       (1u << 8)

/* kernel routing overrides (halign_sw_batch flags, bits 4..5) */
#define HALIGN_ROUTE_AUTO   0u
#define HALIGN_ROUTE_INTER  (1u << 4)  /* one pair per lane */
#define HALIGN_ROUTE_INTRA  (2u << 4)  /* one pair per wavefront */

/* center modes of halign_msa */
#define HALIGN_CENTER_EXACT   (-1)
#define HALIGN_CENTER_LEARNED (-2)

/* Supported envelope: alphabet <= 32, every sequence length < 65536,
 * gap_open >= 0, gap_extend >= 1 (HALIGN_E_UNSUPPORTED otherwise).  Scores
 * are int32 and cannot overflow inside this envelope. */

typedef struct halign_ctx halign_ctx;

/* Substitution matrix s(a, b) and gap weights W_k = gap_open + k*gap_extend
 * (eq. 2 with an affine W_k). */
typedef struct {
    const int8_t *matrix_host;  /* alphabet x alphabet, row-major, host */
    int32_t alphabet;
    int32_t gap_open;
    int32_t gap_extend;
} halign_scoring;

/* A packed sequence set: sequence k is residues[offsets[k] .. offsets[k+1]).
 * offsets (device) and offsets_host (host) hold the same N+1 values;
 * offsets[0] == 0 and offsets are non-decreasing.  Empty sequences are legal. */
typedef struct {
    const uint8_t *residues;      /* device, total = offsets[N] bytes */
    const int64_t *offsets;       /* device, N+1 */
    const int64_t *offsets_host;  /* host,   N+1 */
    int32_t n;                    /* N */
} halign_seqs;

/* ---- context ------------------------------------------------------------ */
/* Creates a context on `device`.  workspace_cap_bytes bounds the traceback
 * scratch the context may hold (0 = a quarter of the device memory free at
 * creation); a batch whose codes exceed it is processed in chunks with
 * identical results. */
int  halign_ctx_create(int device, size_t workspace_cap_bytes, halign_ctx **out);
void halign_ctx_destroy(halign_ctx *ctx);
const char *halign_last_error(void);
/* Bytes of device scratch currently held by the context. */
int  halign_ctx_workspace_bytes(const halign_ctx *ctx, size_t *bytes_host);
/* Timing (ms) of the last halign_sw_batch stages on the ctx stream, measured
 * with HIP events: [0] forward DP kernel(s), [1] traceback walk, [2] whole call.
 * Valid after the stream synchronises. */
int  halign_ctx_last_timings(halign_ctx *ctx, float *ms_host /*[3]*/);
/* Number of workgroups/launches of the dominant forward kernel in the last
 * call (for roofline accounting) and the DP cells it covered. */
int  halign_ctx_last_stats(const halign_ctx *ctx, int64_t *stats_host /*[4]: cells, launches, route, chunks*/);

/* Autotuning of halign_sw_batch plans (off by default; also enabled by the
 * environment variable HALIGN_AUTOTUNE=1).  When on, the first call for a
 * bucket of (center length, batch size, mean length, traceback) times the
 * candidate plans -- wavefront streams of 64 lanes with R or R+1 center rows
 * per lane and one or two streams per resident wave slot, streams of 32 or 16
 * lanes with up to 16 rows per lane, the same in packed 16-bit arithmetic
 * with two streams per lane group (traceback only, when every score stays
 * below 15000), or the one-pair-per-lane kernel -- on the batch (a strided sample of
 * 65,536 pairs for batches above 4e10 cells, with the stream count scaled to
 * keep the pairs per stream) in the call's own mode, and keeps the fastest;
 * results do not depend on the plan.
 * HALIGN_TUNE_CACHE=<path> persists choices (malformed lines are ignored).
 * halign_ctx_last_plan reports {route, R, streams multiplier, lanes per
 * stream, packed (0/1: whether the last batch ran the packed kernel)} of the
 * last call (route -1 / R 0: defaults).  HALIGN_PROGRESS=1 prints one line on
 * stderr as each chunk of a chunked batch completes; HALIGN_HOST_TIMING=1 one
 * line per halign_msa call with the host time (us) between its stages. */
int  halign_ctx_set_autotune(halign_ctx *ctx, int enable);
/* halign_msa runs its pairwise batch with HALIGN_GRAPH when enabled (the
 * batch is planned and captured once, then replayed); graph_launches counts
 * replays. */
int  halign_ctx_set_graph(halign_ctx *ctx, int enable);
int  halign_ctx_graph_launches(const halign_ctx *ctx, int64_t *n_host);
int  halign_ctx_last_plan(const halign_ctx *ctx, int32_t *plan_host /*[5]*/);
/* Failure injection for tests of error handling: chunk c (0-based) of the
 * next halign_sw_batch on this ctx fails with HALIGN_E_DEVICE before its
 * launch (the call returns the error; the ctx stays usable and a repeated
 * call gives the full result). */
int  halign_debug_fail_chunk(halign_ctx *ctx, int c);

/* ---- step a1: encode ASCII to residue codes (upper/lower case; U->C,
 * O->K, other letters -> X).  ascii and codes may alias. */
int halign_encode(const uint8_t *ascii, int64_t len, uint8_t *codes, void *stream);

/* ---- pairwise SW against the center (eq. 1-2, traceback as in Fig. 2) ----
 * center[m] (device) against every sequence of seqs.
 * Outputs (device, any may be NULL except score):
 *   score[N]             best local score (int32)
 *   cells[N][4]          i0, j0, i1, j1: the core aligns center[i0, i1) with
 *                        s[j0, j1) (0-based, half-open); all 0 when score 0.
 *                        End cell = max H, ties to the smallest j, then i.
 *   ins[N][m+1]          residues of s placed in each center slot: slot 0
 *                        before center[0], slot p between center[p-1] and
 *                        center[p], slot m after center[m-1]; the unaligned
 *                        prefix of s goes to slot 0 and the suffix to slot m
 *                        (all of s to slot 0 when the score is 0).
 *   aligned[N][(m+31)/32] bit p set when center[p] faces a residue of s.
 * ins/aligned require HALIGN_TRACEBACK. */
int halign_sw_batch(halign_ctx *ctx, const halign_scoring *sc,
                    const uint8_t *center, int32_t m,
                    const halign_seqs *seqs, uint32_t flags,
                    int32_t *score, int32_t *cells, uint16_t *ins, uint32_t *aligned,
                    void *stream);

/* For callers that cannot allocate memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the score-only form
 * of halign_sw_batch (HALIGN_SCORE_ONLY, end cells through `cells`) without a
 * context and without any allocation, host or device.  Outputs as in
 * halign_sw_batch: score[N] and, when cells != NULL, cells[N][4] =
 * (0, 0, i1, j1).  Pairs run one per lane in input order (no length sort).
 * Scratch: one static device array of HALIGN_NOALLOC_SCRATCH_BYTES per GPU
 * (held from the library's first use of that GPU until the process ends);
 * the longest sequence may use at most that many bytes of strip boundary
 * rows per workgroup (512 bytes per residue, rounded up to 4 residues), which
 * covers every length the library supports; beyond that HALIGN_E_UNSUPPORTED.
 * Residue codes are not checked (codes >= alphabet give unspecified scores,
 * never out-of-bounds accesses).  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two threads) race. */
#define HALIGN_NOALLOC_SCRATCH_BYTES (64u << 20)
int halign_sw_score_noalloc(const halign_scoring *sc, const uint8_t *center, int32_t m,
                            const halign_seqs *seqs, int32_t *score, int32_t *cells, void *stream);

/* Score-only SW of anchored pairs (center selection, training targets):
 * score[64*q + l] = SW(seq anchors_host[q], seq partners_host[64*q + l]) for
 * q < nanchors, l < 64.  Index arrays are HOST arrays; score is device. */
int halign_sw_pairs(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                    const int32_t *anchors_host, int32_t nanchors, const int32_t *partners_host,
                    int32_t *score, void *stream);

/* ---- first reduction of Fig. 3 ------------------------------------------
 * G[p] = max_k ins[k][p] (p = 0..m), col[p] = sum_{q<p} (G[q] + 1) = first
 * MSA column of gap block p, *width_host = m + sum_p G[p] (synchronises). */
int halign_merge(halign_ctx *ctx, const uint16_t *ins, int32_t n, int32_t m,
                 int32_t *G, int64_t *col, int64_t *width_host, void *stream);

/* ---- second map step of Fig. 3: MSA rows ----------------------------------
 * msa[N][width]: block p has G[p] columns holding the ins[k][p] residues of
 * sequence k left-justified then gaps; then (p < m) the column of center[p]
 * holding the next residue of sequence k when aligned bit p is set, else a gap. */
int halign_emit_rows(halign_ctx *ctx, const halign_seqs *seqs, int32_t m,
                     const uint16_t *ins, const uint32_t *aligned,
                     const int32_t *G, const int64_t *col, int64_t width,
                     uint8_t *msa, void *stream);

/* ---- center selection ------------------------------------------------------
 * Exact: sums[i] = sum_{j != i} SW(seq i, seq j) (int64), center = argmax,
 * ties to the lowest index (Methods: the center is the sequence most similar
 * to the others).  *center_host is written (synchronises).
 * Both calls score pairs in packed 16-bit arithmetic when every score stays
 * below 15000 (max matrix entry x longest sequence + go + ge < 15000, go + ge
 * and ge at most 256), else in 32-bit; the
 * sums are the same either way.  HALIGN_STRIP32=1 forces the 32-bit kernel. */
int halign_center_exact(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                        int64_t *sums, int32_t *center_host, void *stream);
/* Group tiling of halign_center_exact (host only, no device needed): all
 * pairs a < b of n positions (in length order) fall into *ngroups_host groups
 * of one center position and `step` consecutive partner positions (64 for
 * the 32-bit kernel, 128 for the packed one), numbered in closed form, so
 * the search holds O(n) host data.  With g >= 0, group g is decoded into its
 * center position and first partner position (partners [p0, p0 + step),
 * those not above the center position are idle).  A caller sharding the
 * exhaustive search over devices can split [0, *ngroups_host). */
int halign_exact_tiling(int64_t n, int32_t step, int64_t g, int64_t *ngroups_host, int64_t *center_pos_host,
                        int64_t *partner0_host);
/* The judge over a partner sample: sums[q] = sum over the listed partners
 * (host array, npartners entries, sequence indices; a candidate scores 0
 * against itself) of SW(seq cand[q], partner); *center_host (optional) = the
 * candidate with the largest sum, ties to the lowest sequence index.  The
 * same partners for every candidate, so differences between candidates are
 * estimated with the sampling noise of the partners shared. */
int halign_center_judge_sample(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                               const int32_t *cand, int32_t ncand, const int32_t *partners_host, int32_t npartners,
                               int64_t *sums, int32_t *center_host, void *stream);
/* Pre-judge of halign_center_learned: candidates (0 = off, at most 256) and
 * partners of the sample. */
int  halign_ctx_set_prejudge(halign_ctx *ctx, int candidates, int partners);
/* Exact judge restricted to candidates cand[ncand] (device): sums[q] =
 * sum_{j != cand[q]} SW(seq cand[q], seq j); *center_host = the candidate
 * with the largest sum, ties to the lowest sequence index. */
int halign_center_judge(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                        const int32_t *cand, int32_t ncand, int64_t *sums,
                        int32_t *center_host, void *stream);

/* ---- learned center proposer (BF16 MLP on 3-mer counts) ------------------
 * Not in the paper: the paper's center is the sequence most similar to all
 * others (exhaustive, O(N^2) alignments).  A small MLP proposes candidates
 * whose exact sums of scores are then compared (halign_center_judge).
 *
 * Features: X[r][400a + 20b + c] = count of the 3-mer abc (codes < 20 only)
 * in sequence rows[r] (rows == NULL: r), stored as bf16 bit patterns,
 * nrows x HALIGN_FEAT, row-major. */
#define HALIGN_FEAT 8000
#define HALIGN_HID  256
#define HALIGN_EMB  64
int halign_featurize(const halign_seqs *seqs, const int32_t *rows, int32_t nrows,
                     uint16_t *X, void *stream);

/* Model for inference (device): W1 HALIGN_FEAT x HALIGN_HID bf16 bits
 * (row-major), b1 HALIGN_HID fp32, W2 HALIGN_HID x HALIGN_EMB bf16 bits, b2
 * HALIGN_EMB fp32.  Forward: Z = X W1 + b1, Hb = bf16(relu(Z)),
 * E = Hb W2 + b2, products on MFMA with fp32 accumulation. */
typedef struct {
    const uint16_t *W1; const float *b1;
    const uint16_t *W2; const float *b2;
} halign_model;

/* Z (fp32 nrows x HID, may be NULL), Hb (bf16 bits nrows x HID) and
 * E (fp32 nrows x EMB) are outputs. */
int halign_mlp_forward(halign_ctx *ctx, const halign_model *model, const uint16_t *X, int32_t nrows,
                       float *Z, uint16_t *Hb, float *E, void *stream);

/* Pair loss for pairs (r, r + npairs), r < npairs, of an E with 2*npairs rows:
 * pred = E[r] . E[r + npairs], loss = mean (pred - target)^2.  Writes dE
 * (fp32, 2*npairs x EMB) and loss_out[0] (device fp32). */
int halign_pair_loss(halign_ctx *ctx, const float *E, const float *target, int32_t npairs,
                     float *dE, float *loss_out, void *stream);

/* halign_pair_loss plus a term on groups of `group` consecutive pairs (1..64,
 * dividing npairs; 0 = none): loss += lam * mean over groups of (mean of
 * pred - target over the group)^2, the squared bias of a group's
 * predictions.  With a group per anchor (all partners of one sequence), the
 * term trains the mean prediction of each sequence against its partners,
 * the quantity the candidate score u_i sums. */
int halign_pair_loss_grouped(halign_ctx *ctx, const float *E, const float *target, int32_t npairs, int32_t group,
                             float lam, float *dE, float *loss_out, void *stream);

/* Backward of halign_mlp_forward for dE (Z and Hb from the same forward):
 * dW1 (fp32 FEAT x HID), db1 (HID), dW2 (fp32 HID x EMB), db2 (EMB).  The
 * GEMM operands dE and dZ are rounded to bf16; the bias gradients are the
 * fp32 column sums of dE and dZ. */
int halign_mlp_backward(halign_ctx *ctx, const halign_model *model, const uint16_t *X, int32_t nrows,
                        const float *Z, const uint16_t *Hb, const float *dE,
                        float *dW1, float *db1, float *dW2, float *db2, void *stream);

/* bf16 copy (round to nearest even) of n fp32 values: dst[i] = bf16 bits of src[i]. */
int halign_f32_to_bf16(const float *src, uint16_t *dst, int64_t n, void *stream);

/* Adam (bias-corrected, step t >= 1) on fp32 master weights p[n] with
 * gradient g and moments m, v; writes the bf16 copy pb when non-NULL. */
int halign_adam_step(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n,
                     float lr, float beta1, float beta2, float eps, int32_t t, void *stream);

/* Candidate scores u_i = E_i . (sum_j E_j - E_i) (fp32, fixed-order sums)
 * and the top k indices (largest u first, ties to the lower index). */
int halign_topk_center(halign_ctx *ctx, const float *E, int32_t nrows, int32_t k, float *u,
                       int32_t *top, void *stream);

/* Trainer.  Parameters (device): fp32 masters and their bf16 copies, updated
 * in place.  Training pairs: `anchors` random sequences, each with
 * `partners` random partners (1..64, 0 = 64; seeded), targets SW(a, b) / 100
 * from halign_sw_pairs (which scores 64 partners per anchor); `epochs`
 * passes of Adam over them in batches of `batch` pairs.  With 0 < ema < 1 an
 * exponential moving average of the parameters (decay `ema` per step, started
 * from the initial parameters) replaces them at the end.  loss_host[e] gets
 * the mean batch loss of epoch e (synchronises). */
typedef struct {
    float *W1, *b1, *W2, *b2;     /* fp32 masters */
    uint16_t *W1b, *W2b;          /* bf16 copies read by the forward */
} halign_params;
typedef struct {
    int32_t anchors;
    int32_t batch;
    int32_t epochs;
    float lr;
    uint64_t seed;
    float ema;                    /* 0: off */
    int32_t partners;             /* per anchor, 1..64 (0: 64) */
    float group_weight;           /* > 0: batches of whole anchors and the
                                     per-anchor term of halign_pair_loss_grouped
                                     with this weight (0: plain pair loss) */
} halign_train_opts;
int halign_train_proposer(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                          const halign_train_opts *opts, const halign_params *params,
                          float *loss_host, void *stream);

/* Learned center: featurize and embed every sequence, take the top k by u,
 * judge them exactly; *center_host = the best candidate (synchronises).
 * cand_host (optional, k entries) receives the candidates.  With a pre-judge
 * set on the ctx (halign_ctx_set_prejudge), the top `candidates` (> k) by u
 * are first scored against a common sample of `partners` sequences (evenly
 * spaced indices; halign_center_judge_sample) and the k best of that sample
 * are the ones judged exactly. */
int halign_center_learned(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                          const halign_model *model, int32_t k, int32_t *cand_host,
                          int32_t *center_host, void *stream);

/* ---- end-to-end center-star MSA -------------------------------------------
 * center >= 0: that sequence index; HALIGN_CENTER_EXACT: exhaustive search;
 * HALIGN_CENTER_LEARNED: top-16 of `model` (halign_center_learned).
 * The MSA buffer (N x width bytes) is obtained from alloc(bytes, user), since
 * width is known only after the merge; *msa receives it. */
typedef void *(*halign_alloc_fn)(size_t bytes, void *user);
int halign_msa(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
               int32_t center, const halign_model *model,
               halign_alloc_fn alloc, void *user,
               uint8_t **msa, int64_t *width_host, int32_t *center_out_host, void *stream);

/* ---- nucleotide center star (Methods, trie section) -------------------------
 * Similar nucleotide sequences: the center's segments of k bases (segment q =
 * center[q*k, q*k + k), codes 0..3 = A C G T only, and no other such segment
 * with the same string) are found in every sequence (the paper's trie with
 * failure links reports every occurrence; here a hash table of the packed
 * segments gives the same set), the largest chain of matches increasing in q
 * with non-overlapping positions p (p_next >= p + k) becomes the anchors
 * (predecessor and end chosen by the smallest (q, p) among equals), and the
 * stretches before, between and after the anchors are aligned end to end with
 * affine gaps W_k = gap_open + gap_extend*k (Gotoh's global form, traceback
 * priorities as for the local alignment).  Codes >= 4 never join an anchor.
 * alphabet >= 5; 1 <= k <= 32.
 * score: device int32 [N] (anchor residues' scores plus the stretches' global
 * scores); ins [N][m+1], aligned [N][(m+31)/32] as in halign_sw_batch; G:
 * optional device int32 [m+1], the merge (max of ins over all sequences but
 * the center).  Scratch lives in the ctx; the call synchronises (the match
 * counts and stretch sizes size it). */
int halign_nuc_align(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                     int32_t center, int32_t k, int32_t *score, uint16_t *ins, uint32_t *aligned,
                     int32_t *G, void *stream);

/* Nucleotide MSA with the given center (the paper takes the first sequence):
 * halign_nuc_align, the center's own row, the merge and the rows, as
 * halign_msa does for proteins.  score: device int32 [N]. */
int halign_nuc_msa(halign_ctx *ctx, const halign_scoring *sc, const halign_seqs *seqs,
                   int32_t center, int32_t k, int32_t *score, halign_alloc_fn alloc, void *user,
                   uint8_t **msa, int64_t *width_host, void *stream);

/* ---- evaluation (Results: avg SP) ------------------------------------------
 * out_host[0] = sum over row pairs and columns of: 1 for two different
 * residues, 2 for a residue against a gap, 0 otherwise (avg SP = out/C(N,2));
 * out_host[1] = BLOSUM column SP (S for residue pairs, -gap_extend per
 * residue/gap pair).  Synchronises. */
int halign_sp_score(const halign_scoring *sc, const uint8_t *msa, int32_t n, int64_t width,
                    int64_t *out_host, void *stream);

/* Column profile of an MSA (Results: the per-column counts that avg SP is a
 * function of).  msa: device uint8 [n][width], residue codes below alphabet
 * or HALIGN_GAP (255).  profile: device int32 [width][alphabet + 1],
 * caller-owned, overwritten: profile[x][a] = rows whose column x holds code a,
 * profile[x][alphabet] = gaps in column x.  1 <= alphabet <= 32.  Reads the
 * MSA once, in coalesced row segments (suited to 1e6 rows).  Synchronises;
 * HALIGN_E_INVALID if a byte is neither a code below alphabet nor the gap
 * (profile contents then unspecified). */
int halign_column_profile(const uint8_t *msa, int32_t n, int64_t width, int32_t alphabet,
                          int32_t *profile, void *stream);

/* ---- phylogeny (Methods, "NJ method for constructing phylogenetic trees
 * with Spark", Fig. 4) -------------------------------------------------------
 * p-distances between MSA rows: D[i * nb + j] = (columns where rows a_rows[i]
 * and b_rows[j] differ and both hold a residue, i.e. neither is HALIGN_GAP)
 * / (columns where both hold a residue), 1.0 where no column qualifies.
 * msa: device uint8 [n][width], residue codes below 128 or HALIGN_GAP (a byte
 * from 128 to 254 is not checked and compares by its low seven bits); a_rows,
 * b_rows: device int32 row indices
 * (NULL: rows 0 .. na-1, 0 .. nb-1); D: device double [na][nb]; mism, comp:
 * device int32 [na][nb] (the two counts) or NULL.  The counts are exact and
 * the quotient is one IEEE division.  Asynchronous on stream. */
int halign_pdist(halign_ctx *ctx, const uint8_t *msa, int32_t n, int64_t width, const int32_t *a_rows,
                 int32_t na, const int32_t *b_rows, int32_t nb, double *D, int32_t *mism, int32_t *comp,
                 void *stream);

/* Neighbour joining (Saitou and Nei) over the n x n device distance matrix D
 * (symmetric, zero diagonal; not modified): with m active nodes, r_i = sum
 * over active k of d(i, k) in slot order, Q(i, j) = (m - 2) d(i, j) - r_i -
 * r_j; the smallest Q is joined (ties to the smallest i, then j, i < j) with
 * lengths d(i, j) / 2 + (r_i - r_j) / (2 (m - 2)) and d(i, j) minus that; the
 * new node takes slot i, d(u, k) = (d(i, k) + d(j, k) - d(i, j)) / 2.  Three
 * nodes left meet at a centre (three-point lengths), two at a centre (d / 2
 * each).  Every double operation rounds on its own, in that order.  Output:
 * parent_host, blen_host (host, 2n + 1 entries): nodes 0 .. n-1 are the
 * leaves, joins number n, n + 1, ...; the root has parent -1; *nodes = the
 * node count.  Synchronises. */
int halign_nj(halign_ctx *ctx, const double *D, int32_t n, int32_t *parent_host, double *blen_host,
              int32_t *nodes, void *stream);

/* The tree of an MSA (Fig. 4: sample, distances, clustering, per-cluster
 * neighbour joining, merge).  perm_host: a permutation of 0 .. n-1 (the
 * random draw; the sample is its first ceil(n / 10) rows).  Every row goes
 * to its nearest sample row (ties to the earlier); then, once and in cluster
 * order, a cluster of fewer than 3 rows joins the cluster whose seed is
 * nearest its seed (ties to the lower cluster); then, once, a cluster of
 * more than ceil(n / 10) rows is divided among its first ceil(size / 10) rows
 * in permutation order (nearest, ties to the earlier); empty clusters are
 * dropped.  Each cluster is joined (halign_nj over its rows in row order) and
 * so are the clusters' seeds; each cluster's root replaces its leaf in the
 * seeds' tree.  parent_host, blen_host: host, 2n + 2 entries; nodes 0 .. n-1
 * are the rows, then each cluster's joins (cluster order), then the seeds'
 * tree's joins; *nodes = the node count.  Scratch lives in the ctx (the
 * distance matrices of the clusters and of the seeds).  Synchronises. */
int halign_nj_tree(halign_ctx *ctx, const uint8_t *msa, int32_t n, int64_t width, const int32_t *perm_host,
                   int32_t *parent_host, double *blen_host, int32_t *nodes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HALIGN_H */
