"""Pins of the oracle's nucleotide center star (trie section): the trie's
matches against a plain substring search, the anchor chain against every
chain of small match sets, the global alignment of the stretches against
enumeration of every global alignment, and whole pairwise alignments by
re-scoring and by restoring both inputs."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1704_00878_amd import synth

NM, GO, GE = synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND


def _indexed(c, k):
    """Segments of c with codes 0..3 only whose string no other such segment shares."""
    segs = [bytes(c[q * k:(q + 1) * k]) for q in range(len(c) // k)]
    clean = [q for q, s in enumerate(segs) if max(s, default=0) <= 3]
    count = {}
    for q in clean:
        count[segs[q]] = count.get(segs[q], 0) + 1
    return {q: segs[q] for q in clean if count[segs[q]] == 1}


def _naive_matches(c, s, k):
    out = []
    idx = _indexed(c, k)
    for p in range(len(s) - k + 1):
        w = bytes(s[p:p + k])
        for q, seg in idx.items():
            if w == seg:
                out.append((p, q))
    return sorted(out)


@pytest.mark.parametrize("seed", range(12))
def test_trie_matches_equal_substring_search(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 6))
    c = rng.integers(0, 4, int(rng.integers(0, 60))).astype(np.uint8)
    if len(c) >= 2 * k and seed % 3 == 0:
        c[k:2 * k] = c[0:k]                   # a repeated segment (dropped from the index)
    if len(c) and seed % 4 == 1:
        c[rng.integers(0, len(c))] = 4        # an N inside a segment
    parts = [c[int(a):int(a) + int(b)] for a, b in rng.integers(0, max(len(c), 1), (6, 2))]
    parts.append(rng.integers(0, 5, 10).astype(np.uint8))
    s = np.concatenate([p for p in parts] + [np.zeros(0, np.uint8)]).astype(np.uint8)
    mq, mp = oracle.nuc_matches(c, s, k)
    assert sorted(zip(mp.tolist(), mq.tolist())) == _naive_matches(c, s, k)
    assert list(mp) == sorted(mp)


def _valid_chain(mq, mp, k, idx):
    return all(mq[idx[x]] < mq[idx[x + 1]] and mp[idx[x]] + k <= mp[idx[x + 1]] for x in range(len(idx) - 1))


@pytest.mark.parametrize("seed", range(30))
def test_chain_is_a_largest_chain(seed):
    rng = np.random.default_rng(100 + seed)
    a, k = int(rng.integers(0, 11)), int(rng.integers(1, 4))
    mp = np.sort(rng.choice(40, a, replace=False)).astype(np.int32)
    mq = rng.integers(0, 8, a).astype(np.int32)
    ch = oracle.nuc_chain(mq, mp, k)
    best = 0
    for r in range(a, 0, -1):
        if any(_valid_chain(mq, mp, k, comb) for comb in itertools.combinations(range(a), r)):
            best = r
            break
    assert len(ch) == best
    assert _valid_chain(mq, mp, k, list(ch))


def test_chain_tie_rule_hand():
    # matches (q, p) in p order, k = 2: two chains of 2 end at (3, 9); the
    # predecessor with the smaller q wins: (1, 0) -> (3, 9), not (2, 4) -> (3, 9)
    mq = np.array([2, 1, 3], np.int32)
    mp = np.array([0, 4, 9], np.int32)
    assert oracle.nuc_chain(mq, mp, 2).tolist() == [1, 2]
    # the chain ends at the smallest (q, p) among the longest: (0, 0) -> (5, 3) vs (0, 0) -> (4, 6)
    mq = np.array([0, 5, 4], np.int32)
    mp = np.array([0, 3, 6], np.int32)
    assert oracle.nuc_chain(mq, mp, 2).tolist() == [0, 2]


def _columns(c, s, ins, al):
    """The alignment the center-star vector describes, as (center code|None, seq code|None) columns."""
    cols, j = [], 0
    m = len(c)
    for p in range(m + 1):
        for _ in range(int(ins[p])):
            cols.append((None, int(s[j])))
            j += 1
        if p < m:
            if al[p]:
                cols.append((int(c[p]), int(s[j])))
                j += 1
            else:
                cols.append((int(c[p]), None))
    assert j == len(s)
    return cols


def _score_columns(S, go, ge, cols):
    tot, prev = 0, None
    for a, b in cols:
        kind = "M" if a is not None and b is not None else ("I" if a is None else "D")
        if kind == "M":
            tot += int(S[a][b])
        else:
            tot -= ge if prev == kind else go + ge
        prev = kind
    return tot


def _all_global(S, go, ge, c, s):
    """Best score over every global alignment (column sequences), by enumeration."""
    best = None

    def rec(i, j, tot, prev):
        nonlocal best
        if i == len(c) and j == len(s):
            best = tot if best is None else max(best, tot)
            return
        if i < len(c) and j < len(s):
            rec(i + 1, j + 1, tot + int(S[c[i]][s[j]]), "M")
        if j < len(s):
            rec(i, j + 1, tot - (ge if prev == "I" else go + ge), "I")
        if i < len(c):
            rec(i + 1, j, tot - (ge if prev == "D" else go + ge), "D")

    rec(0, 0, 0, None)
    return best


@pytest.mark.parametrize("seed", range(25))
def test_global_stretch_against_enumeration(seed):
    """k larger than both sequences: no anchor, one global alignment."""
    rng = np.random.default_rng(300 + seed)
    c = rng.integers(0, 5, int(rng.integers(0, 5))).astype(np.uint8)
    s = rng.integers(0, 5, int(rng.integers(0, 5))).astype(np.uint8)
    r = oracle.nuc_align(NM, GO, GE, 16, c, s)
    assert r["anchors"] == 0
    assert r["score"] == _all_global(NM, GO, GE, list(c), list(s))
    cols = _columns(c, s, r["ins"], r["aligned"])
    assert _score_columns(NM, GO, GE, cols) == r["score"]


@pytest.mark.parametrize("seed", range(8))
def test_pairwise_rescore_and_restore(seed):
    d = synth.generate_dna("dna_small", n_seqs=6, seed=400 + seed)
    c = d.seq(0)
    for x in range(1, d.n):
        s = d.seq(x)
        r = oracle.nuc_align(NM, GO, GE, 16, c, s)
        cols = _columns(c, s, r["ins"], r["aligned"])
        assert [a for a, _ in cols if a is not None] == list(c)
        assert [b for _, b in cols if b is not None] == list(s)
        assert _score_columns(NM, GO, GE, cols) == r["score"]
        assert r["anchors"] > 0


def test_identical_and_empty():
    c = synth.generate_dna("dna_small", n_seqs=1, seed=5).seq(0)
    r = oracle.nuc_align(NM, GO, GE, 16, c, c)
    assert r["anchors"] > 0 and r["aligned"].all() and r["ins"].sum() == 0
    assert r["score"] == sum(int(NM[x][x]) for x in c)
    e = np.zeros(0, np.uint8)
    r = oracle.nuc_align(NM, GO, GE, 16, c, e)
    assert r["ins"].sum() == 0 and r["aligned"].sum() == 0 and r["score"] == -(GO + GE * len(c))
    r = oracle.nuc_align(NM, GO, GE, 16, e, c[:20])
    assert r["ins"].tolist() == [20] and r["score"] == -(GO + GE * 20)


def test_hand_case():
    """k = 4: center ACGT|TTGA|CCCC|AG, sequence ACGT + T + TTGA + GG + CCCC.
    Segments 0-2 are indexed; all three match, in order, so the anchors are
    ACGT (p 0), TTGA (p 5) and CCCC (p 11).  Between the first two anchors the
    center stretch is empty and the sequence stretch is T: one insertion in
    slot 4; between the second and third, GG in slot 8; after the last anchor
    the center's AG face nothing (two center residues against gaps)."""
    enc = {ch: i for i, ch in enumerate("ACGTN")}
    c = np.array([enc[x] for x in "ACGTTTGACCCCAG"], np.uint8)
    s = np.array([enc[x] for x in "ACGTTTTGAGGCCCC"], np.uint8)
    r = oracle.nuc_align(NM, GO, GE, 4, c, s)
    assert r["anchors"] == 3
    want_ins = [0] * 15
    want_ins[4], want_ins[8] = 1, 2
    assert r["ins"].tolist() == want_ins
    assert r["aligned"].tolist() == [1] * 12 + [0, 0]
    # 12 matches (+24), an insertion of 1 (-7), of 2 (-9), a deletion of 2 (-9)
    assert r["score"] == 24 - 7 - 9 - 9
