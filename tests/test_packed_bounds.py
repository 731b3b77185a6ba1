"""Host-side checks of the biased 16-bit arithmetic of the packed kernels.

The packed wavefront and strip kernels hold every H, E*, F* and H - go - ge
plus a bias and take three-way maxima with v_pk_maximum3_f16 on the bit
patterns.  That is exact only if (1) non-negative 16-bit patterns below 0x7c00
order as halves the way they order as integers, and (2) the bias, the padding
profile entry and the host bounds keep every operand in that range and the
padding entry below the floor.  (1) is checked exhaustively, (2) on the
constants as the sources define them, and both together by running the
recurrence in that arithmetic on the host against the oracle at scores up to
the bound.
"""
import os
import re

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1704_00878_amd", "csrc")


def _constants():
    src = open(os.path.join(CSRC, "pk16.hpp")).read()
    bias = int(re.search(r"constexpr int kBias16 = (-?\d+);", src).group(1))
    pad = int(re.search(r"constexpr int kPadProf16 = (-?\d+);", src).group(1))
    host = open(os.path.join(CSRC, "halign.hip")).read()
    bounds = {int(b) for b in re.findall(r"< (\d+) && S\.goe <= 256", host)}
    bounds |= {int(b) for b in re.findall(r"S\.goe <= 256 && S\.ge <= 256 && \(int64_t\)smax \* lmax \+ S\.goe < (\d+)",
                                          host)}
    return bias, pad, bounds


def test_half_order_matches_integer_order():
    x = np.arange(0, 0x7C00, dtype=np.uint16)
    h = x.view(np.float16)
    assert np.isfinite(h).all() and (h >= 0).all()
    assert (np.diff(h.astype(np.float64)) > 0).all()
    assert not np.isfinite(np.array([0x7C01], np.uint16).view(np.float16)).all()   # NaN just above


def test_bias_and_padding_constants():
    B, P, bounds = _constants()
    assert bounds == {15000}, bounds
    Hb, gmax, smin = 15000, 256, -128   # H < Hb, go + ge <= 256 and ge <= 256, int8 scores
    # smallest operands: E* - ge and F* - ge (E*, F* >= 0), H - go - ge, a real
    # diagonal (H - go - ge) + (S + go + ge) and a padded one (H - go - ge) + pad
    assert B - gmax >= 0
    assert B + smin >= 0
    assert B - gmax + P >= 0
    # largest operand: H + bias
    assert B + Hb - 1 <= 0x7BFF
    # a padded diagonal never reaches the floor (bias), whatever H and go + ge
    assert (B + Hb - 1) + P < B


def _sw_biased(S, go, ge, c, s, B, P, npad=3):
    """Score-only SW with the kernels' biased arithmetic: E*, F*, H as
    three-way half maxima of 16-bit patterns, npad padding rows and columns
    after the real ones.  Returns the best H over the real cells and asserts
    that every operand stays in [0, 0x7c00)."""
    goe = go + ge
    m, n = len(c), len(s)
    M, N = m + npad, n + npad
    prof = np.full((N, M), P, np.int64)   # prof[j][i]: S + go + ge of row i, column j
    for j in range(n):
        prof[j, :m] = S[c, s[j]].astype(np.int64) + goe

    def max3h(a, b, d):
        v = np.array([a, b, d], np.int64)
        assert (v >= 0).all() and (v < 0x7C00).all(), v
        return int(v.astype(np.uint16).view(np.float16).max().view(np.uint16))

    init = B - goe
    hg = [init] * M        # H - go - ge of the previous column, per row
    e = [init] * M         # E* of the previous column, per row
    best = B
    for j in range(N):
        upg, upf = init, init
        diag = init
        for i in range(M):
            en = max3h(e[i] - ge, hg[i], B)
            fn = max3h(upf - ge, upg, B)
            hd = diag + int(prof[j, i])
            h = max3h(hd, en, fn)
            if i < m and j < n:
                best = max(best, h)
            else:   # a padded diagonal stays below the floor
                assert hd < B
            diag = hg[i]
            hg[i] = h - goe
            e[i] = en
            upg, upf = hg[i], fn
    return best - B


def test_biased_recurrence_matches_oracle_up_to_the_bound():
    B, P, _ = _constants()
    rng = np.random.default_rng(4)
    # a scoring matrix with a large diagonal so that H comes close to 15000
    S = rng.integers(-128, 10, size=(4, 4)).astype(np.int8)
    np.fill_diagonal(S, [50, 7, 3, 1])
    c = np.zeros(299, np.uint8)                  # 50 * 299 = 14950 < 15000
    mixed = (rng.integers(0, 4, 120).astype(np.uint8), rng.integers(0, 4, 90).astype(np.uint8))
    cases = [(11, 1, c, c.copy()), (11, 1, c[:150], c[20:].copy()), (11, 1) + mixed,
             (0, 1) + mixed, (200, 56) + mixed, (200, 56, c[:100], c[:100].copy())]
    for go, ge, a, b in cases:
        got = _sw_biased(S.astype(np.int64), go, ge, a, b, B, P)
        ref = oracle.sw(S, go, ge, a, b)["score"]
        assert got == ref, (go, ge, len(a), len(b), got, ref)
        if len(a) == len(b) == 299:
            assert got == 14950
