/*
 * CPU oracle for the center-star protein MSA path of HAlign-II
 * (Wan & Zou, arXiv 1704.00878).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition the HIP library is checked against.  It shares no code, header
 * or table with the library; only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  Everything is plain single-threaded C
 * over full DP matrices, int32 arithmetic, no SIMD.
 *
 * Notation: center c (length m, rows i = 1..m), sequence s (length n, columns
 * j = 1..n).  Scoring: substitution matrix S (alphabet x alphabet, row-major
 * int8) and gap cost W_k = go + ge * k for a gap of k residues.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - W_k = go + ge*k (a gap of k residues costs go + ge*k).
 *  - End cell: the maximum H; ties go to the smallest j, then the smallest i.
 *  - Traceback priority at an H cell: stop when H == 0, else the diagonal,
 *    else the horizontal gap (s_j against '-'), else the vertical gap
 *    (c_i against '-'); a gap is followed back to the shortest length that
 *    reaches the cell's value.
 *  - Flanks: the unaligned prefix of s goes before c_1 (slot 0), the
 *    unaligned suffix after c_m (slot m).
 *  - Merge: G[p] = max_k ins_k[p]; rows are not re-aligned afterwards.
 *  - Rows: inserted residues are left-justified in their gap block.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NEG (-(1 << 29))
#define ORC_GAP 255

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

static int imax(int a, int b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------
 * Encoding of protein text into residue codes (the sequences the Methods
 * section distributes are protein letters): code = position of the letter in
 * the NCBI order ARNDCQEGHILKMFPSTWYVBZX* (upper or lower case); the rare
 * residues U (selenocysteine) and O (pyrrolysine) take the codes of C and K;
 * every other byte is X.  A plain search of the order string per byte.
 * ---------------------------------------------------------------------- */
void orc_encode(const uint8_t *ascii, int64_t len, uint8_t *codes)
{
    static const char order[] = "ARNDCQEGHILKMFPSTWYVBZX*";
    for (int64_t x = 0; x < len; x++) {
        int ch = ascii[x];
        if (ch >= 'a' && ch <= 'z') ch = ch - 'a' + 'A';
        if (ch == 'U') ch = 'C';
        if (ch == 'O') ch = 'K';
        int code = 22;                       /* X */
        for (int k = 0; k < 24; k++)
            if (order[k] == ch) { code = k; break; }
        codes[x] = (uint8_t)code;
    }
}

/* ------------------------------------------------------------------------
 * Literal eq. 2 (Methods, Smith-Waterman section) with an arbitrary gap
 * weight table W[1..], O(m n (m + n)).  Returns the best score; fills the
 * full H matrix ((m+1) x (n+1), row-major) when H is non-NULL.
 * Boundary per eq. 1: H(i,0) = H(0,j) = 0.
 * ---------------------------------------------------------------------- */
int orc_sw_eq2(const int8_t *S, int alpha, const int32_t *W /* W[k], k=0..max(m,n) */,
               const uint8_t *c, int m, const uint8_t *s, int n, int32_t *H)
{
    int own = 0;
    if (!H) {
        H = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1) * (size_t)(n + 1));
        if (!H) return ORC_ENOMEM;
        own = 1;
    }
    const int ld = n + 1;
    int best = 0;
    for (int i = 0; i <= m; i++) H[(size_t)i * ld] = 0;
    for (int j = 0; j <= n; j++) H[j] = 0;
    for (int i = 1; i <= m; i++) {
        for (int j = 1; j <= n; j++) {
            int h = H[(size_t)(i - 1) * ld + (j - 1)] + S[c[i - 1] * alpha + s[j - 1]];
            for (int k = 1; k <= i; k++) h = imax(h, H[(size_t)(i - k) * ld + j] - W[k]);
            for (int l = 1; l <= j; l++) h = imax(h, H[(size_t)i * ld + (j - l)] - W[l]);
            h = imax(h, 0);
            H[(size_t)i * ld + j] = h;
            if (h > best) best = h;
        }
    }
    if (own) free(H);
    return best;
}

/* Traceback over a literal eq. 2 matrix: ops gets 'M','I' (s_j vs gap) or
 * 'D' (c_i vs gap) in forward order; returns the number of ops.
 * cells = (i0, j0, i1, j1), 0-based half-open core. */
int orc_sw_eq2_path(const int8_t *S, int alpha, const int32_t *W,
                    const uint8_t *c, int m, const uint8_t *s, int n,
                    const int32_t *H, int32_t *cells, char *ops)
{
    const int ld = n + 1;
    int best = 0, bi = 0, bj = 0;
    /* column-major scan: the first maximum seen is the smallest j, then i */
    for (int j = 1; j <= n; j++)
        for (int i = 1; i <= m; i++)
            if (H[(size_t)i * ld + j] > best) { best = H[(size_t)i * ld + j]; bi = i; bj = j; }
    int len = 0;
    int i = bi, j = bj;
    if (best > 0) {
        while (H[(size_t)i * ld + j] != 0) {
            int h = H[(size_t)i * ld + j];
            if (h == H[(size_t)(i - 1) * ld + (j - 1)] + S[c[i - 1] * alpha + s[j - 1]]) {
                ops[len++] = 'M'; i--; j--; continue;
            }
            int moved = 0;
            for (int l = 1; l <= j && !moved; l++)
                if (h == H[(size_t)i * ld + (j - l)] - W[l]) {
                    for (int t = 0; t < l; t++) ops[len++] = 'I';
                    j -= l; moved = 1;
                }
            for (int k = 1; k <= i && !moved; k++)
                if (h == H[(size_t)(i - k) * ld + j] - W[k]) {
                    for (int t = 0; t < k; t++) ops[len++] = 'D';
                    i -= k; moved = 1;
                }
            if (!moved) return ORC_EINVAL; /* cannot happen for a valid H */
        }
    }
    for (int a = 0, b = len - 1; a < b; a++, b--) { char t = ops[a]; ops[a] = ops[b]; ops[b] = t; }
    cells[0] = i; cells[1] = j; cells[2] = bi; cells[3] = bj;
    return len;
}

/* ------------------------------------------------------------------------
 * Affine special case of eq. 2 (Gotoh's three-matrix form), which equals
 * eq. 2 exactly when W_k = go + ge*k:
 *   E(i,j) = max(E(i,j-1) - ge, H(i,j-1) - go - ge)   horizontal gap
 *   F(i,j) = max(F(i-1,j) - ge, H(i-1,j) - go - ge)   vertical gap
 *   H(i,j) = max(0, H(i-1,j-1) + S[c_i][s_j], E(i,j), F(i,j))
 * with H(i,0) = H(0,j) = 0 (eq. 1) and E(i,0) = F(0,j) = -inf.
 *
 * Outputs (any may be NULL):
 *   cells[4]   = i0, j0, i1, j1 (0-based half-open core; all 0 if score 0)
 *   ins[m+1]   = residues of s placed in each center slot (slot p lies
 *                between c_p and c_{p+1}; slot 0 before c_1, slot m after c_m)
 *   aligned[m] = 1 where c_{p+1} faces a residue of s
 *   ops, *nops = the core as 'M'/'I'/'D' in forward order
 * Returns the score, or a negative error.
 * ---------------------------------------------------------------------- */
int orc_sw(const int8_t *S, int alpha, int go, int ge,
           const uint8_t *c, int m, const uint8_t *s, int n,
           int32_t *cells, uint16_t *ins, uint8_t *aligned, char *ops, int32_t *nops)
{
    if (m < 0 || n < 0 || alpha <= 0) return ORC_EINVAL;
    for (int i = 0; i < m; i++) if (c[i] >= alpha) return ORC_EINVAL;
    for (int j = 0; j < n; j++) if (s[j] >= alpha) return ORC_EINVAL;
    const size_t ld = (size_t)n + 1, sz = ((size_t)m + 1) * ld;
    int32_t *H = (int32_t *)malloc(sizeof(int32_t) * sz);
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * sz);
    int32_t *F = (int32_t *)malloc(sizeof(int32_t) * sz);
    if (!H || !E || !F) { free(H); free(E); free(F); return ORC_ENOMEM; }
    const int goe = go + ge;
    for (size_t j = 0; j <= (size_t)n; j++) { H[j] = 0; E[j] = ORC_NEG; F[j] = ORC_NEG; }
    for (int i = 1; i <= m; i++) {
        int32_t *Hi = H + (size_t)i * ld, *Ei = E + (size_t)i * ld, *Fi = F + (size_t)i * ld;
        const int32_t *Hu = Hi - ld, *Fu = Fi - ld;
        const int8_t *Srow = S + c[i - 1] * alpha;
        Hi[0] = 0; Ei[0] = ORC_NEG; Fi[0] = ORC_NEG;
        for (int j = 1; j <= n; j++) {
            int e = imax(Ei[j - 1] - ge, Hi[j - 1] - goe);
            int f = imax(Fu[j] - ge, Hu[j] - goe);
            int h = imax(imax(0, Hu[j - 1] + Srow[s[j - 1]]), imax(e, f));
            Ei[j] = e; Fi[j] = f; Hi[j] = h;
        }
    }
    /* End cell: max H, ties to the smallest j, then the smallest i. */
    int best = 0, bi = 0, bj = 0;
    for (int j = 1; j <= n; j++)
        for (int i = 1; i <= m; i++) {
            int h = H[(size_t)i * ld + j];
            if (h > best) { best = h; bi = i; bj = j; }
        }
    /* Traceback from (bi, bj) until a zero cell (state machine over H/E/F). */
    if (ins) memset(ins, 0, sizeof(uint16_t) * ((size_t)m + 1));
    if (aligned) memset(aligned, 0, (size_t)m);
    int i = bi, j = bj, len = 0;
    enum { ST_H, ST_E, ST_F } st = ST_H;
    if (best > 0) {
        for (;;) {
            const size_t at = (size_t)i * ld + j;
            if (st == ST_H) {
                if (H[at] == 0) break;
                if (H[at] == H[at - ld - 1] + S[c[i - 1] * alpha + s[j - 1]]) {
                    if (ops) ops[len] = 'M';
                    if (aligned) aligned[i - 1] = 1;
                    len++; i--; j--;
                } else if (H[at] == E[at]) {
                    st = ST_E;
                } else {
                    st = ST_F;
                }
            } else if (st == ST_E) {
                /* s_j faces a gap after c_i: it lands in slot i */
                if (ops) ops[len] = 'I';
                if (ins) ins[i] += 1;
                len++;
                int ext = E[at - 1] - ge > H[at - 1] - goe;
                j--;
                if (!ext) st = ST_H;
            } else {
                if (ops) ops[len] = 'D';
                len++;
                int ext = F[at - ld] - ge > H[at - ld] - goe;
                i--;
                if (!ext) st = ST_H;
            }
        }
    }
    free(H); free(E); free(F);
    int i0 = i, j0 = j, i1 = bi, j1 = bj;
    if (best == 0) { i0 = j0 = i1 = j1 = 0; }
    if (ops) for (int a = 0, b = len - 1; a < b; a++, b--) { char t = ops[a]; ops[a] = ops[b]; ops[b] = t; }
    if (nops) *nops = len;
    if (cells) { cells[0] = i0; cells[1] = j0; cells[2] = i1; cells[3] = j1; }
    if (ins) {
        if (best == 0) {
            ins[0] = (uint16_t)n;                    /* no core: all of s before c_1 */
        } else {
            ins[0] = (uint16_t)(ins[0] + j0);        /* prefix of s before c_1 */
            ins[m] = (uint16_t)(ins[m] + (n - j1));  /* suffix of s after c_m */
        }
    }
    return best;
}

/* Score only: same recurrence, rolling rows. */
int orc_sw_score(const int8_t *S, int alpha, int go, int ge,
                 const uint8_t *c, int m, const uint8_t *s, int n)
{
    int32_t *Hr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *Fr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!Hr || !Fr) { free(Hr); free(Fr); return ORC_ENOMEM; }
    const int goe = go + ge;
    for (int j = 0; j <= n; j++) { Hr[j] = 0; Fr[j] = ORC_NEG; }
    int best = 0;
    for (int i = 1; i <= m; i++) {
        const int8_t *Srow = S + c[i - 1] * alpha;
        int hdiag = 0, hleft = 0, e = ORC_NEG;
        for (int j = 1; j <= n; j++) {
            e = imax(e - ge, hleft - goe);
            int f = imax(Fr[j] - ge, Hr[j] - goe);
            int h = imax(imax(0, hdiag + Srow[s[j - 1]]), imax(e, f));
            hdiag = Hr[j];
            Hr[j] = h; Fr[j] = f; hleft = h;
            if (h > best) best = h;
        }
    }
    free(Hr); free(Fr);
    return best;
}

/* ------------------------------------------------------------------------
 * Batch: every sequence against the center (the first map step of Fig. 3).
 * ---------------------------------------------------------------------- */
int orc_sw_batch(const int8_t *S, int alpha, int go, int ge,
                 const uint8_t *center, int m,
                 const uint8_t *res, const int64_t *off, int nseq,
                 int32_t *score, int32_t *cells, uint16_t *ins, uint8_t *aligned)
{
    for (int k = 0; k < nseq; k++) {
        const uint8_t *s = res + off[k];
        int n = (int)(off[k + 1] - off[k]);
        int r = orc_sw(S, alpha, go, ge, center, m, s, n,
                       cells ? cells + 4 * (size_t)k : NULL,
                       ins ? ins + (size_t)k * (m + 1) : NULL,
                       aligned ? aligned + (size_t)k * m : NULL, NULL, NULL);
        if (r < 0) return r;
        score[k] = r;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * First reduction of Fig. 3: the longest center-star sequence.
 *   G[p]   = max_k ins_k[p]                     p = 0..m
 *   col[p] = sum_{q<p} (G[q] + 1)               first column of block p
 *   width  = m + sum_p G[p]
 * ---------------------------------------------------------------------- */
int orc_merge(const uint16_t *ins, int nseq, int m, int32_t *G, int64_t *col, int64_t *width)
{
    for (int p = 0; p <= m; p++) G[p] = 0;
    for (int k = 0; k < nseq; k++)
        for (int p = 0; p <= m; p++)
            if (ins[(size_t)k * (m + 1) + p] > G[p]) G[p] = ins[(size_t)k * (m + 1) + p];
    int64_t acc = 0;
    for (int p = 0; p <= m; p++) { col[p] = acc; acc += G[p] + 1; }
    *width = acc - 1;
    return ORC_OK;
}

/* Second map step: each row from its inserted-space vector and sequence.
 * Block p holds G[p] columns with the ins[p] residues of s left-justified,
 * then (p < m) one column for c_{p+1}: the next residue of s when
 * aligned[p], else a gap.  msa is nseq x width, gap byte 255. */
int orc_rows(const uint8_t *res, const int64_t *off, int nseq, int m,
             const uint16_t *ins, const uint8_t *aligned, const int32_t *G,
             int64_t width, uint8_t *msa)
{
    for (int k = 0; k < nseq; k++) {
        const uint8_t *s = res + off[k];
        int64_t n = off[k + 1] - off[k];
        uint8_t *row = msa + (size_t)k * (size_t)width;
        int64_t col = 0, j = 0;
        for (int p = 0; p <= m; p++) {
            int a = ins[(size_t)k * (m + 1) + p];
            for (int t = 0; t < G[p]; t++) row[col++] = (t < a) ? s[j++] : ORC_GAP;
            if (p < m) row[col++] = aligned[(size_t)k * m + p] ? s[j++] : ORC_GAP;
        }
        if (col != width || j != n) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* Whole center-star MSA for a given center index (the center's own row is
 * the gapped center: its inserted-space vector is all zero). */
int orc_msa(const int8_t *S, int alpha, int go, int ge,
            const uint8_t *res, const int64_t *off, int nseq, int center,
            int32_t *score, int32_t *cells, uint16_t *ins, uint8_t *aligned,
            int32_t *G, int64_t *col, int64_t *width)
{
    if (center < 0 || center >= nseq) return ORC_EINVAL;
    const uint8_t *c = res + off[center];
    int m = (int)(off[center + 1] - off[center]);
    int r = orc_sw_batch(S, alpha, go, ge, c, m, res, off, nseq, score, cells, ins, aligned);
    if (r < 0) return r;
    memset(ins + (size_t)center * (m + 1), 0, sizeof(uint16_t) * ((size_t)m + 1));
    memset(aligned + (size_t)center * m, 1, (size_t)m);
    return orc_merge(ins, nseq, m, G, col, width);
}

/* ------------------------------------------------------------------------
 * Exact center: argmax_i sum_{j != i} SW(s_i, s_j); ties to the lowest i.
 * sums[nseq] receives every candidate's sum.
 * ---------------------------------------------------------------------- */
int orc_center_exact(const int8_t *S, int alpha, int go, int ge,
                     const uint8_t *res, const int64_t *off, int nseq, int64_t *sums)
{
    for (int a = 0; a < nseq; a++) sums[a] = 0;
    for (int a = 0; a < nseq; a++)
        for (int b = 0; b < nseq; b++) {
            if (a == b) continue;
            int r = orc_sw_score(S, alpha, go, ge, res + off[a], (int)(off[a + 1] - off[a]),
                                 res + off[b], (int)(off[b + 1] - off[b]));
            if (r < 0) return r;
            sums[a] += r;
        }
    int best = 0;
    for (int a = 1; a < nseq; a++) if (sums[a] > sums[best]) best = a;
    return best;
}

/* Sum of judge scores for candidate centers only (the exact judge). */
int orc_center_judge(const int8_t *S, int alpha, int go, int ge,
                     const uint8_t *res, const int64_t *off, int nseq,
                     const int32_t *cand, int ncand, int64_t *sums)
{
    for (int q = 0; q < ncand; q++) {
        int a = cand[q];
        sums[q] = 0;
        for (int b = 0; b < nseq; b++) {
            if (b == a) continue;
            int r = orc_sw_score(S, alpha, go, ge, res + off[a], (int)(off[a + 1] - off[a]),
                                 res + off[b], (int)(off[b + 1] - off[b]));
            if (r < 0) return r;
            sums[q] += r;
        }
    }
    int best = 0;
    for (int q = 1; q < ncand; q++)
        if (sums[q] > sums[best] || (sums[q] == sums[best] && cand[q] < cand[best])) best = q;
    return cand[best];
}

/* ------------------------------------------------------------------------
 * avg SP (Results, datasets section): over all row pairs and columns, +1 for
 * two different residues, +2 for a residue against a gap, 0 otherwise;
 * summed and divided by the number of row pairs.  Returns the numerator;
 * written as the explicit pair loop.
 * ---------------------------------------------------------------------- */
int64_t orc_sp_pairs(const uint8_t *msa, int nseq, int64_t width)
{
    int64_t total = 0;
    for (int a = 0; a < nseq; a++)
        for (int b = a + 1; b < nseq; b++)
            for (int64_t x = 0; x < width; x++) {
                uint8_t u = msa[(size_t)a * width + x], v = msa[(size_t)b * width + x];
                if (u == ORC_GAP && v == ORC_GAP) continue;
                if (u == ORC_GAP || v == ORC_GAP) total += 2;
                else if (u != v) total += 1;
            }
    return total;
}

/* Same quantity by column counts (what scales to large N). */
int64_t orc_sp_columns(const uint8_t *msa, int nseq, int64_t width)
{
    int64_t total = 0;
    int64_t cnt[256];
    for (int64_t x = 0; x < width; x++) {
        memset(cnt, 0, sizeof cnt);
        for (int a = 0; a < nseq; a++) cnt[msa[(size_t)a * width + x]]++;
        int64_t g = cnt[ORC_GAP], r = nseq - g, same = 0;
        for (int t = 0; t < 255; t++) same += cnt[t] * (cnt[t] - 1) / 2;
        total += (r * (r - 1) / 2 - same) + 2 * g * r;
    }
    return total;
}

/* Column profile (Results, datasets section: the per-column counts from which
 * the avg SP of an alignment follows): out[x * (alpha + 1) + a] = number of
 * rows whose column x holds residue code a (a < alpha); slot alpha counts the
 * gaps.  Returns 0, or -1 if a byte is neither a residue code below alpha nor
 * the gap code. */
int orc_column_profile(const uint8_t *msa, int nseq, int64_t width, int alpha, int32_t *out)
{
    memset(out, 0, sizeof(int32_t) * (size_t)width * (size_t)(alpha + 1));
    for (int a = 0; a < nseq; a++)
        for (int64_t x = 0; x < width; x++) {
            uint8_t u = msa[(size_t)a * width + x];
            if (u == ORC_GAP) out[x * (alpha + 1) + alpha]++;
            else if (u < alpha) out[x * (alpha + 1) + u]++;
            else return -1;
        }
    return 0;
}

/* BLOSUM column SP: S for residue pairs, -ge per residue/gap pair, 0 gap/gap. */
int64_t orc_sp_blosum(const int8_t *S, int alpha, int ge, const uint8_t *msa, int nseq, int64_t width)
{
    int64_t total = 0;
    for (int a = 0; a < nseq; a++)
        for (int b = a + 1; b < nseq; b++)
            for (int64_t x = 0; x < width; x++) {
                uint8_t u = msa[(size_t)a * width + x], v = msa[(size_t)b * width + x];
                if (u == ORC_GAP && v == ORC_GAP) continue;
                if (u == ORC_GAP || v == ORC_GAP) total -= ge;
                else total += S[u * alpha + v];
            }
    return total;
}
