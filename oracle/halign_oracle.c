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

/* ========================================================================
 * Nucleotide center star (Methods, "Trie trees method for similar
 * nucleotide sequences"): the first sequence is the center; a trie of the
 * center's segments with failure links finds the segments that recur in
 * each sequence; those matched segments are kept as they are and only the
 * unmatched stretches between them are aligned.
 *
 * Readings of the paper (it gives no parameters):
 *  - Segments: the center is cut into consecutive segments of k residues
 *    (segment q covers c[q*k, q*k + k)); a segment is indexed when it holds
 *    only codes 0..3 (A, C, G, T) and no other indexed segment has the same
 *    string.  The trailing partial segment is never indexed.
 *  - Matches: every (q, p) with s[p, p + k) equal to indexed segment q (the
 *    trie with failure links, Aho-Corasick, reports them in order of p;
 *    a byte >= 4 in s returns the automaton to its root).
 *  - Anchors: a chain of matches strictly increasing in q with
 *    p_next >= p + k, of the largest size.  best[i] = 1 + max best[j] over
 *    earlier matches j (p_j + k <= p_i, q_j < q_i); the predecessor of i is,
 *    among those j with best[j] = best[i] - 1, the one with the smallest
 *    (q_j, p_j); the chain ends at the match with the largest best, ties to
 *    the smallest (q, p).
 *  - Between anchors (and before the first and after the last), the center
 *    stretch and the sequence stretch are aligned end to end with affine
 *    gaps (Gotoh's global form, W_k = go + ge*k, the same traceback
 *    priorities as the local alignment: diagonal, then s residue against a
 *    gap, then center residue against a gap; a gap is followed back to the
 *    shortest length reaching the value).
 *  - Output: the same center-star vector as the protein path (ins[m+1]
 *    slots, aligned[m]), so the merge and the rows are unchanged; score =
 *    sum of S over the anchors' residues plus the stretches' global scores.
 * ====================================================================== */

/* Trie (goto function over codes 0..3) of the indexed segments with failure
 * links; node 0 is the root.  out[v] = segment ending at node v, or -1. */
typedef struct { int32_t *go; int32_t *fail; int32_t *out; int nn; } orc_trie;

static void orc_trie_free(orc_trie *t) { free(t->go); free(t->fail); free(t->out); }

/* Indexed segments of c: idx[q] = 1 when segment q is indexed. */
static int orc_nuc_index(const uint8_t *c, int m, int k, uint8_t *idx)
{
    const int ns = k > 0 ? m / k : 0;
    for (int q = 0; q < ns; q++) {
        idx[q] = 1;
        for (int t = 0; t < k; t++) if (c[q * k + t] > 3) { idx[q] = 0; break; }
    }
    for (int q = 0; q < ns; q++) {
        if (!idx[q]) continue;
        for (int r = q + 1; r < ns; r++)
            if (idx[r] && memcmp(c + q * k, c + r * k, (size_t)k) == 0) {
                /* a repeated segment string is dropped everywhere */
                for (int x = r; x < ns; x++)
                    if (x != q && memcmp(c + q * k, c + x * k, (size_t)k) == 0) idx[x] = 2;
                idx[q] = 2;
                break;
            }
    }
    for (int q = 0; q < ns; q++) if (idx[q] == 2) idx[q] = 0;
    return ns;
}

static int orc_trie_build(const uint8_t *c, int m, int k, orc_trie *t)
{
    const int ns = k > 0 ? m / k : 0;
    uint8_t *idx = (uint8_t *)calloc((size_t)ns + 1, 1);
    const int cap = ns * k + 1;
    t->go = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)cap);
    t->fail = (int32_t *)calloc((size_t)cap, sizeof(int32_t));
    t->out = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    if (!idx || !t->go || !t->fail || !t->out || !queue) {
        free(idx); free(queue); orc_trie_free(t); return ORC_ENOMEM;
    }
    orc_nuc_index(c, m, k, idx);
    for (int v = 0; v < cap; v++) { t->out[v] = -1; for (int a = 0; a < 4; a++) t->go[4 * v + a] = -1; }
    int nn = 1;
    for (int q = 0; q < ns; q++) {
        if (!idx[q]) continue;
        int v = 0;
        for (int d = 0; d < k; d++) {
            int a = c[q * k + d];
            if (t->go[4 * v + a] < 0) t->go[4 * v + a] = nn++;
            v = t->go[4 * v + a];
        }
        t->out[v] = q;
    }
    /* failure links by breadth-first order; missing edges become the
     * failure target's edges (the goto function of the automaton) */
    int head = 0, tail = 0;
    for (int a = 0; a < 4; a++) {
        int u = t->go[a];
        if (u < 0) t->go[a] = 0;
        else { t->fail[u] = 0; queue[tail++] = u; }
    }
    while (head < tail) {
        int v = queue[head++];
        for (int a = 0; a < 4; a++) {
            int u = t->go[4 * v + a];
            if (u < 0) { t->go[4 * v + a] = t->go[4 * t->fail[v] + a]; continue; }
            t->fail[u] = t->go[4 * t->fail[v] + a];
            queue[tail++] = u;
        }
    }
    t->nn = nn;
    free(idx); free(queue);
    return ORC_OK;
}

/* All matches (q, p) of the indexed center segments in s, in order of p.
 * Returns the number of matches (at most cap are written), or an error. */
int orc_nuc_matches(const uint8_t *c, int m, const uint8_t *s, int n, int k,
                    int32_t *mq, int32_t *mp, int cap)
{
    if (k < 1 || m < 0 || n < 0) return ORC_EINVAL;
    orc_trie t;
    int r = orc_trie_build(c, m, k, &t);
    if (r < 0) return r;
    int v = 0, cnt = 0;
    for (int j = 0; j < n; j++) {
        if (s[j] > 3) { v = 0; continue; }
        v = t.go[4 * v + s[j]];
        /* all segments have length k, so only the node itself can end one
         * (a shorter suffix along the failure chain is never a segment) */
        if (t.out[v] >= 0) {
            if (cnt < cap) { mq[cnt] = t.out[v]; mp[cnt] = j - k + 1; }
            cnt++;
        }
    }
    orc_trie_free(&t);
    return cnt;
}

/* Anchor chain over matches (mq, mp) in order of p (the reading above).
 * chain[] receives the chosen match indices in increasing order; returns
 * the chain length. */
int orc_nuc_chain(const int32_t *mq, const int32_t *mp, int a, int k, int32_t *chain)
{
    if (a <= 0) return 0;
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * (size_t)a);
    int32_t *pred = (int32_t *)malloc(sizeof(int32_t) * (size_t)a);
    if (!best || !pred) { free(best); free(pred); return ORC_ENOMEM; }
    for (int i = 0; i < a; i++) {
        int b = 0;
        for (int j = 0; j < i; j++)
            if (mp[j] + k <= mp[i] && mq[j] < mq[i] && best[j] > b) b = best[j];
        best[i] = b + 1;
        pred[i] = -1;
        for (int j = 0; j < i; j++) {
            if (mp[j] + k > mp[i] || mq[j] >= mq[i] || best[j] != b) continue;
            if (pred[i] < 0 || mq[j] < mq[pred[i]] || (mq[j] == mq[pred[i]] && mp[j] < mp[pred[i]])) pred[i] = j;
        }
    }
    int e = 0;
    for (int i = 1; i < a; i++)
        if (best[i] > best[e] || (best[i] == best[e] && (mq[i] < mq[e] || (mq[i] == mq[e] && mp[i] < mp[e])))) e = i;
    const int len = best[e];
    for (int x = len - 1, i = e; x >= 0; x--, i = pred[i]) chain[x] = i;
    free(best); free(pred);
    return len;
}

/* Global affine alignment of c[0, mc) against s[0, nc) (Gotoh, end to end):
 * H(0,0) = 0, H(i,0) = F(i,0) = -(go + ge*i), H(0,j) = E(0,j) = -(go + ge*j).
 * Writes the moves into the center-star vector at center offset cb and
 * returns the score. */
static int orc_global(const int8_t *S, int alpha, int go, int ge, const uint8_t *c, int mc, const uint8_t *s,
                      int nc, int cb, uint16_t *ins, uint8_t *aligned, int *err)
{
    const size_t ld = (size_t)nc + 1, sz = ((size_t)mc + 1) * ld;
    int32_t *H = (int32_t *)malloc(sizeof(int32_t) * sz);
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * sz);
    int32_t *F = (int32_t *)malloc(sizeof(int32_t) * sz);
    if (!H || !E || !F) { free(H); free(E); free(F); *err = ORC_ENOMEM; return 0; }
    const int goe = go + ge;
    H[0] = 0; E[0] = ORC_NEG; F[0] = ORC_NEG;
    for (int j = 1; j <= nc; j++) { H[j] = -(go + ge * j); E[j] = H[j]; F[j] = ORC_NEG; }
    for (int i = 1; i <= mc; i++) {
        int32_t *Hi = H + (size_t)i * ld, *Ei = E + (size_t)i * ld, *Fi = F + (size_t)i * ld;
        const int32_t *Hu = Hi - ld, *Fu = Fi - ld;
        Hi[0] = -(go + ge * i); Ei[0] = ORC_NEG; Fi[0] = Hi[0];
        for (int j = 1; j <= nc; j++) {
            int e = imax(Ei[j - 1] - ge, Hi[j - 1] - goe);
            int f = imax(Fu[j] - ge, Hu[j] - goe);
            int h = imax(Hu[j - 1] + S[c[i - 1] * alpha + s[j - 1]], imax(e, f));
            Ei[j] = e; Fi[j] = f; Hi[j] = h;
        }
    }
    const int score = H[(size_t)mc * ld + nc];
    int i = mc, j = nc;
    enum { ST_H, ST_E, ST_F } st = ST_H;
    while (i > 0 || j > 0) {
        const size_t at = (size_t)i * ld + j;
        if (st == ST_H) {
            if (i > 0 && j > 0 && H[at] == H[at - ld - 1] + S[c[i - 1] * alpha + s[j - 1]]) {
                aligned[cb + i - 1] = 1;
                i--; j--;
            } else if (H[at] == E[at]) {
                st = ST_E;
            } else {
                st = ST_F;
            }
        } else if (st == ST_E) {
            ins[cb + i] += 1;   /* s_j after c_{cb+i}: slot cb + i */
            int ext = j > 1 && E[at - 1] - ge > H[at - 1] - goe;
            j--;
            if (!ext) st = ST_H;
        } else {
            int ext = i > 1 && F[at - ld] - ge > H[at - ld] - goe;
            i--;
            if (!ext) st = ST_H;
        }
    }
    free(H); free(E); free(F);
    return score;
}

/* Pairwise nucleotide center-star alignment of s against center c.
 * ins[m+1], aligned[m] (zeroed here); *nanchors (may be NULL) receives the
 * chain length.  Returns 0 and the score in *score, or a negative error. */
int orc_nuc_align(const int8_t *S, int alpha, int go, int ge, int k,
                  const uint8_t *c, int m, const uint8_t *s, int n,
                  int32_t *score, uint16_t *ins, uint8_t *aligned, int32_t *nanchors)
{
    if (k < 1 || m < 0 || n < 0 || alpha < 5) return ORC_EINVAL;
    for (int i = 0; i < m; i++) if (c[i] >= alpha) return ORC_EINVAL;
    for (int j = 0; j < n; j++) if (s[j] >= alpha) return ORC_EINVAL;
    memset(ins, 0, sizeof(uint16_t) * ((size_t)m + 1));
    memset(aligned, 0, (size_t)m);
    const int cap = n + 1;
    int32_t *mq = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *mp = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *ch = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    if (!mq || !mp || !ch) { free(mq); free(mp); free(ch); return ORC_ENOMEM; }
    int a = orc_nuc_matches(c, m, s, n, k, mq, mp, cap);
    int len = a < 0 ? a : orc_nuc_chain(mq, mp, a, k, ch);
    if (len < 0) { free(mq); free(mp); free(ch); return len; }
    int total = 0, err = 0, ci = 0, sj = 0;   /* next unaligned center / sequence position */
    for (int x = 0; x <= len && !err; x++) {
        const int qc = x < len ? mq[ch[x]] * k : m;   /* stretch ends at the anchor (or the ends) */
        const int ps = x < len ? mp[ch[x]] : n;
        total += orc_global(S, alpha, go, ge, c + ci, qc - ci, s + sj, ps - sj, ci, ins, aligned, &err);
        if (x < len) {
            for (int t = 0; t < k; t++) {
                aligned[qc + t] = 1;
                total += S[c[qc + t] * alpha + s[ps + t]];
            }
            ci = qc + k;
            sj = ps + k;
        }
    }
    free(mq); free(mp); free(ch);
    if (err) return err;
    if (nanchors) *nanchors = len;
    *score = total;
    return ORC_OK;
}

/* Nucleotide MSA with sequence 0 as the center: every pair's vectors, then
 * the merge (the center's own row is the gapped center). */
int orc_nuc_msa(const int8_t *S, int alpha, int go, int ge, int k,
                const uint8_t *res, const int64_t *off, int nseq,
                int32_t *score, uint16_t *ins, uint8_t *aligned,
                int32_t *G, int64_t *col, int64_t *width)
{
    if (nseq < 1) return ORC_EINVAL;
    const uint8_t *c = res + off[0];
    const int m = (int)(off[1] - off[0]);
    for (int x = 0; x < nseq; x++) {
        int r = orc_nuc_align(S, alpha, go, ge, k, c, m, res + off[x], (int)(off[x + 1] - off[x]),
                              score + x, ins + (size_t)x * (m + 1), aligned + (size_t)x * m, NULL);
        if (r < 0) return r;
    }
    memset(ins, 0, sizeof(uint16_t) * ((size_t)m + 1));
    memset(aligned, 1, (size_t)m);
    return orc_merge(ins, nseq, m, G, col, width);
}

/* ========================================================================
 * Phylogeny from the MSA (Methods, "NJ method for constructing phylogenetic
 * trees with Spark", Fig. 4): pairwise distances between MSA rows, a sampled
 * clustering, neighbour joining (Saitou and Nei, the paper's ref. 22) inside
 * each cluster and over the clusters, the cluster trees grafted onto the
 * cluster-level tree.  Readings this section fixes (the paper names the steps
 * and nothing more):
 *  - Distance: the p-distance of two rows, mismatching columns over the
 *    columns where both rows hold a residue (any byte but the gap byte); 1
 *    when no column qualifies.
 *  - Neighbour joining: with m active nodes, r_i = sum over active k of
 *    d(i, k) (summed in slot order), Q(i, j) = (m - 2) d(i, j) - r_i - r_j;
 *    the pair with the smallest Q is joined, ties to the smallest i, then j
 *    (i < j); branch lengths d(i, j) / 2 + (r_i - r_j) / (2 (m - 2)) and
 *    d(i, j) minus that; the new node takes slot i, slot j is dropped, and
 *    d(u, k) = (d(i, k) + d(j, k) - d(i, j)) / 2.  Three nodes left join at a
 *    centre with the three-point lengths; two at a centre with d / 2 each.
 *    Negative lengths are kept.  Every step is an IEEE double operation in
 *    the order written (no fused multiply-add).
 *  - Tree layout: nodes 0 .. n-1 are the leaves, joins number the new nodes
 *    n, n + 1, ... in order; parent[] and blen[] per node, the root (the last
 *    centre, or the single leaf) has parent -1.
 *  - Clustering: the sample is the first ceil(N / 10) entries of a given
 *    permutation (the random draw is an input); every row is labelled with
 *    its nearest sample row (ties to the earlier sample position).  Then, once
 *    and in cluster order, a cluster of fewer than 3 rows is merged into the
 *    cluster whose seed is nearest its own seed (ties to the lower cluster;
 *    not when it is the only cluster); then, until no cluster has more than
 *    ceil(N / 10) rows ("divided ... until balanced construction"), each such
 *    cluster is divided: its first ceil(size / 10) rows in permutation order
 *    become seeds and its rows are relabelled among them (nearest, ties to
 *    the earlier); when every row stays with one seed (near-identical rows),
 *    it is cut into runs of ceil(N / 10) of its rows in permutation order.
 *    Clusters are numbered by their seeds' sample order (divided ones in
 *    place, in their new seeds' order); a cluster left empty (its seed went
 *    to an identical earlier seed) is dropped after each pass.
 *  - Merge: neighbour joining over each cluster's rows (slots in row order)
 *    and over the clusters' seeds (the cluster-level tree); each cluster's
 *    root replaces the cluster's leaf in the cluster-level tree (keeping that
 *    leaf's branch length).  Node numbering: rows 0 .. N-1, then each
 *    cluster's internal nodes (cluster order), then the cluster-level tree's
 *    internal nodes.
 * ------------------------------------------------------------------------ */

/* p-distance counts of rows a and b of an MSA with w columns. */
void orc_pdist_counts(const uint8_t *msa, int64_t w, int a, int b, int64_t *mism, int64_t *comp)
{
    const uint8_t *x = msa + (size_t)a * w, *y = msa + (size_t)b * w;
    int64_t mm = 0, cc = 0;
    for (int64_t c = 0; c < w; c++) {
        if (x[c] != ORC_GAP && y[c] != ORC_GAP) {
            cc++;
            if (x[c] != y[c]) mm++;
        }
    }
    *mism = mm;
    *comp = cc;
}

double orc_pdist(const uint8_t *msa, int64_t w, int a, int b)
{
    int64_t mm, cc;
    orc_pdist_counts(msa, w, a, b, &mm, &cc);
    return cc > 0 ? (double)mm / (double)cc : 1.0;
}

/* Neighbour joining over the n x n distance matrix D (row-major, symmetric,
 * zero diagonal; not modified).  parent and blen take the tree (2n - 2 nodes
 * for n >= 3, 3 for n = 2, 1 for n = 1); returns the node count or < 0. */
int orc_nj(const double *D, int n, int *parent, double *blen)
{
    if (n < 1) return ORC_EINVAL;
    double *d = malloc(sizeof(double) * (size_t)n * n);
    double *r = malloc(sizeof(double) * (size_t)n);
    int *id = malloc(sizeof(int) * (size_t)n);
    char *act = malloc((size_t)n);
    if (!d || !r || !id || !act) { free(d); free(r); free(id); free(act); return ORC_ENOMEM; }
    memcpy(d, D, sizeof(double) * (size_t)n * n);
    for (int s = 0; s < n; s++) { id[s] = s; act[s] = 1; }
    int next = n, m = n;
    while (m > 3) {
        for (int i = 0; i < n; i++) {
            if (!act[i]) continue;
            double sum = 0.0;
            for (int k = 0; k < n; k++)
                if (act[k]) sum += d[(size_t)i * n + k];
            r[i] = sum;
        }
        double best = 0.0;
        int bi = -1, bj = -1;
        for (int i = 0; i < n; i++) {
            if (!act[i]) continue;
            for (int j = i + 1; j < n; j++) {
                if (!act[j]) continue;
                const double q = (double)(m - 2) * d[(size_t)i * n + j] - r[i] - r[j];
                if (bi < 0 || q < best) { best = q; bi = i; bj = j; }
            }
        }
        const double dij = d[(size_t)bi * n + bj];
        const double li = 0.5 * dij + (r[bi] - r[bj]) / (2.0 * (double)(m - 2));
        const double lj = dij - li;
        const int u = next++;
        parent[id[bi]] = u; blen[id[bi]] = li;
        parent[id[bj]] = u; blen[id[bj]] = lj;
        for (int k = 0; k < n; k++) {
            if (!act[k] || k == bi || k == bj) continue;
            const double v = (d[(size_t)bi * n + k] + d[(size_t)bj * n + k] - dij) * 0.5;
            d[(size_t)bi * n + k] = v;
            d[(size_t)k * n + bi] = v;
        }
        act[bj] = 0;
        id[bi] = u;
        m--;
    }
    int s[3], t = 0;
    for (int i = 0; i < n && t < 3; i++)
        if (act[i]) s[t++] = i;
    if (m == 3) {
        const double dab = d[(size_t)s[0] * n + s[1]], dac = d[(size_t)s[0] * n + s[2]],
                     dbc = d[(size_t)s[1] * n + s[2]];
        const int u = next++;
        parent[id[s[0]]] = u; blen[id[s[0]]] = (dab + dac - dbc) * 0.5;
        parent[id[s[1]]] = u; blen[id[s[1]]] = (dab + dbc - dac) * 0.5;
        parent[id[s[2]]] = u; blen[id[s[2]]] = (dac + dbc - dab) * 0.5;
        parent[u] = -1; blen[u] = 0.0;
    } else if (m == 2) {
        const double dab = d[(size_t)s[0] * n + s[1]];
        const int u = next++;
        parent[id[s[0]]] = u; blen[id[s[0]]] = dab * 0.5;
        parent[id[s[1]]] = u; blen[id[s[1]]] = dab * 0.5;
        parent[u] = -1; blen[u] = 0.0;
    } else {
        parent[id[s[0]]] = -1; blen[id[s[0]]] = 0.0;
    }
    free(d); free(r); free(id); free(act);
    return next;
}

/* The clusters of the reading above: label[x] = cluster of row x; returns
 * the cluster count K (seed[c] = the seed row of cluster c) or < 0. */
int orc_nj_clusters(const uint8_t *msa, int nseq, int64_t w, const int32_t *perm, int32_t *label, int32_t *seed)
{
    if (nseq < 1) return ORC_EINVAL;
    const int S = (nseq + 9) / 10;
    int K = S;
    for (int c = 0; c < S; c++) seed[c] = perm[c];
    for (int x = 0; x < nseq; x++) {   /* nearest sample row */
        double best = 0.0;
        int bc = -1;
        for (int c = 0; c < S; c++) {
            const double dd = orc_pdist(msa, w, x, seed[c]);
            if (bc < 0 || dd < best) { best = dd; bc = c; }
        }
        label[x] = bc;
    }
    int *size = calloc((size_t)nseq + 1, sizeof(int));
    int *map = malloc(sizeof(int) * ((size_t)nseq + 1));
    if (!size || !map) { free(size); free(map); return ORC_ENOMEM; }
    for (int x = 0; x < nseq; x++) size[label[x]]++;
    /* merge clusters of fewer than 3 rows into the cluster of the nearest
     * seed, once, in cluster order (sizes update as clusters merge) */
    for (int c = 0; c < K && K > 1; c++) {
        if (size[c] == 0 || size[c] >= 3) continue;
        double best = 0.0;
        int bc = -1;
        for (int e = 0; e < K; e++) {
            if (e == c || size[e] == 0) continue;
            const double dd = orc_pdist(msa, w, seed[c], seed[e]);
            if (bc < 0 || dd < best) { best = dd; bc = e; }
        }
        if (bc < 0) continue;   /* the only cluster left */
        for (int x = 0; x < nseq; x++)
            if (label[x] == c) label[x] = bc;
        size[bc] += size[c];
        size[c] = 0;
    }
    /* renumber the clusters left (in order) */
    int K2 = 0;
    for (int c = 0; c < K; c++) map[c] = size[c] > 0 ? K2++ : -1;
    for (int c = 0; c < K; c++)
        if (map[c] >= 0) { seed[map[c]] = seed[c]; size[map[c]] = size[c]; }
    for (int x = 0; x < nseq; x++) label[x] = map[label[x]];
    K = K2;
    /* divide clusters of more than ceil(N / 10) rows until none is left: a
     * cluster is replaced, in place, by the clusters of its first
     * ceil(size / 10) rows in permutation order (its rows relabelled among
     * them, nearest, ties to the earlier); when every row stays with one of
     * them, by consecutive runs of ceil(N / 10) of its rows in permutation
     * order instead; empty clusters are dropped after each pass */
    int32_t *nseed = malloc(sizeof(int32_t) * (size_t)nseq);
    int32_t *nlab = malloc(sizeof(int32_t) * (size_t)nseq);
    if (!nseed || !nlab) { free(size); free(map); free(nseed); free(nlab); return ORC_ENOMEM; }
    for (;;) {
        int big = 0;
        for (int c = 0; c < K; c++) big |= size[c] > S;
        if (!big) break;
        int NK = 0;
        for (int c = 0; c < K; c++) {
            if (size[c] <= S) {
                for (int x = 0; x < nseq; x++)
                    if (label[x] == c) nlab[x] = NK;
                nseed[NK++] = seed[c];
                continue;
            }
            const int ns = (size[c] + 9) / 10;
            const int base = NK;
            for (int t = 0; t < nseq && NK - base < ns; t++)   /* the cluster's rows in permutation order */
                if (label[perm[t]] == c) nseed[NK++] = perm[t];
            int first = -1, split = 0;
            for (int x = 0; x < nseq; x++) {
                if (label[x] != c) continue;
                double best = 0.0;
                int bc = -1;
                for (int e = base; e < NK; e++) {
                    const double dd = orc_pdist(msa, w, x, nseed[e]);
                    if (bc < 0 || dd < best) { best = dd; bc = e; }
                }
                nlab[x] = bc;
                if (first < 0) first = bc;
                else if (bc != first) split = 1;
            }
            if (!split) {   /* runs of S rows in permutation order */
                NK = base;
                int cnt = 0;
                for (int t = 0; t < nseq; t++) {
                    const int x = perm[t];
                    if (label[x] != c) continue;
                    if (cnt % S == 0) nseed[NK++] = x;
                    nlab[x] = NK - 1;
                    cnt++;
                }
            }
        }
        /* drop empty clusters (a seed taken by an identical earlier seed), keeping the order */
        for (int c = 0; c < NK; c++) size[c] = 0;
        for (int x = 0; x < nseq; x++) size[nlab[x]]++;
        K2 = 0;
        for (int c = 0; c < NK; c++) map[c] = size[c] > 0 ? K2++ : -1;
        for (int c = 0; c < NK; c++)
            if (map[c] >= 0) { seed[map[c]] = nseed[c]; size[map[c]] = size[c]; }
        for (int x = 0; x < nseq; x++) label[x] = map[nlab[x]];
        K = K2;
    }
    free(size); free(map); free(nseed); free(nlab);
    return K;
}

/* The whole tree: clusters, neighbour joining in each cluster and over the
 * cluster seeds, the merge.  parent / blen have room for 2 N nodes; returns
 * the node count (the root is the node with parent -1) or < 0. */
int orc_nj_tree(const uint8_t *msa, int nseq, int64_t w, const int32_t *perm, int32_t *parent, double *blen)
{
    if (nseq < 1) return ORC_EINVAL;
    int32_t *label = malloc(sizeof(int32_t) * (size_t)nseq);
    int32_t *seed = malloc(sizeof(int32_t) * (size_t)nseq);
    int *croot = malloc(sizeof(int) * (size_t)nseq);
    if (!label || !seed || !croot) { free(label); free(seed); free(croot); return ORC_ENOMEM; }
    const int K = orc_nj_clusters(msa, nseq, w, perm, label, seed);
    if (K < 0) { free(label); free(seed); free(croot); return K; }
    int next = nseq;
    int *rows = malloc(sizeof(int) * (size_t)nseq);
    int *lp = malloc(sizeof(int) * 2 * (size_t)nseq);
    double *lb = malloc(sizeof(double) * 2 * (size_t)nseq);
    double *D = NULL;
    int err = (!rows || !lp || !lb) ? ORC_ENOMEM : ORC_OK;
    for (int c = 0; c < K && !err; c++) {
        int n = 0;
        for (int x = 0; x < nseq; x++)
            if (label[x] == c) rows[n++] = x;
        free(D);
        D = malloc(sizeof(double) * (size_t)n * n);
        if (!D) { err = ORC_ENOMEM; break; }
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++)
                D[(size_t)a * n + b] = a == b ? 0.0 : orc_pdist(msa, w, rows[a], rows[b]);
        const int nn = orc_nj(D, n, lp, lb);
        if (nn < 0) { err = nn; break; }
        /* local node v: a leaf (v < n) is rows[v], an internal one next + v - n */
        for (int v = 0; v < nn; v++) {
            const int gv = v < n ? rows[v] : next + v - n;
            const int pv = lp[v];
            parent[gv] = pv < 0 ? -1 : (pv < n ? rows[pv] : next + pv - n);
            blen[gv] = lb[v];
            if (pv < 0) croot[c] = gv;
        }
        next += nn - n;
    }
    if (!err) {   /* the cluster-level tree over the seeds */
        free(D);
        D = malloc(sizeof(double) * (size_t)K * K);
        if (!D) err = ORC_ENOMEM;
        else {
            for (int a = 0; a < K; a++)
                for (int b = 0; b < K; b++)
                    D[(size_t)a * K + b] = a == b ? 0.0 : orc_pdist(msa, w, seed[a], seed[b]);
            const int nn = orc_nj(D, K, lp, lb);
            if (nn < 0) err = nn;
            else {
                /* leaf c of this tree is cluster c's root; internal nodes follow */
                for (int v = 0; v < nn; v++) {
                    const int gv = v < K ? croot[v] : next + v - K;
                    const int pv = lp[v];
                    parent[gv] = pv < 0 ? -1 : (pv < K ? croot[pv] : next + pv - K);
                    blen[gv] = pv < 0 ? 0.0 : lb[v];
                }
                next += nn - K;
            }
        }
    }
    free(D); free(rows); free(lp); free(lb); free(label); free(seed); free(croot);
    return err ? err : next;
}
