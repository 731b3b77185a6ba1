"""Oracle SW pins: brute force, the literal eq. 2 form, closed forms, invariants."""
import itertools

import numpy as np
import pytest

import oracle
from brute import best_local, rescore
from paper_1704_00878_amd import synth

B62 = synth.BLOSUM62
GO, GE = synth.GAP_OPEN, synth.GAP_EXTEND


def _check_alignment(S, go, ge, c, s, r):
    """Invariants every oracle result must satisfy."""
    score, cells, ins, al, ops = r["score"], r["cells"], r["ins"], r["aligned"], r["ops"]
    i0, j0, i1, j1 = [int(x) for x in cells]
    m, n = len(c), len(s)
    if score == 0:
        assert ops == "" and (i0, j0, i1, j1) == (0, 0, 0, 0)
        assert ins[0] == n and ins[1:].sum() == 0 and al.sum() == 0
        return
    assert ops[0] == "M" and ops[-1] == "M"
    assert rescore(S, go, ge, c, s, i0, j0, ops) == score
    assert ops.count("M") + ops.count("D") == i1 - i0
    assert ops.count("M") + ops.count("I") == j1 - j0
    assert int(ins.sum()) + int(al.sum()) == n
    assert ins[0] == j0 + 0 and ins[m] >= n - j1
    # rebuild s from the center-star vector: slots and aligned columns in order
    pos = 0
    rebuilt = []
    for p in range(m + 1):
        rebuilt += list(s[pos:pos + ins[p]])
        pos += ins[p]
        if p < m and al[p]:
            rebuilt.append(s[pos])
            pos += 1
    assert pos == n and (np.array(rebuilt, dtype=np.uint8) == s).all()


def _small_matrix(rng, k):
    A = rng.integers(-3, 4, size=(k, k))
    A = np.triu(A) + np.triu(A, 1).T
    np.fill_diagonal(A, rng.integers(1, 6, size=k))
    return A.astype(np.int8)


@pytest.mark.parametrize("alpha", [2, 3])
def test_brute_force_exhaustive_tiny(alpha):
    """Every pair of sequences up to length 3 over a tiny alphabet."""
    rng = np.random.default_rng(7 + alpha)
    S = _small_matrix(rng, alpha)
    words = [np.array(w, np.uint8) for L in range(1, 4) for w in itertools.product(range(alpha), repeat=L)]
    for go, ge in [(1, 1), (0, 1), (2, 1), (3, 2)]:
        for c in words:
            for s in words:
                r = oracle.sw(S, go, ge, c, s, want_ops=True)
                best, opt = best_local(S, go, ge, c, s)
                assert r["score"] == best
                _check_alignment(S, go, ge, c, s, r)
                if best > 0:
                    ends = sorted({(a[4], a[3]) for a in opt})  # (j1, i1)
                    assert (int(r["cells"][3]), int(r["cells"][2])) == ends[0]
                    keys = {(a[1], a[2], a[3], a[4], a[5]) for a in opt}
                    assert tuple(int(x) for x in r["cells"]) + (r["ops"],) in keys


def test_brute_force_random_blosum():
    rng = np.random.default_rng(11)
    for _ in range(250):
        c = rng.integers(0, 20, size=rng.integers(1, 6)).astype(np.uint8)
        s = rng.integers(0, 20, size=rng.integers(1, 6)).astype(np.uint8)
        go, ge = [(11, 1), (10, 1), (0, 4), (2, 1)][rng.integers(0, 4)]
        r = oracle.sw(B62, go, ge, c, s, want_ops=True)
        best, opt = best_local(B62, go, ge, c, s)
        assert r["score"] == best
        _check_alignment(B62, go, ge, c, s, r)
        if best > 0:
            ends = sorted({(a[4], a[3]) for a in opt})
            assert (int(r["cells"][3]), int(r["cells"][2])) == ends[0]
            keys = {(a[1], a[2], a[3], a[4], a[5]) for a in opt}
            assert tuple(int(x) for x in r["cells"]) + (r["ops"],) in keys


def test_brute_force_len6_related():
    """Length-6 pairs where gaps pay off (one a mutated copy of the other)."""
    rng = np.random.default_rng(3)
    S = _small_matrix(np.random.default_rng(99), 4)
    S[np.diag_indices(4)] = 6
    for _ in range(25):
        c = rng.integers(0, 4, size=6).astype(np.uint8)
        s = c.copy()
        k = int(rng.integers(0, 6))
        s = np.delete(s, k) if rng.random() < 0.5 else np.insert(s, k, rng.integers(0, 4))
        s = s[:6]
        r = oracle.sw(S, 1, 1, c, s, want_ops=True)
        best, opt = best_local(S, 1, 1, c, s)
        assert r["score"] == best
        _check_alignment(S, 1, 1, c, s, r)


def test_gotoh_equals_literal_eq2():
    """The affine three-matrix form equals the literal eq. 2 with W_k = go + ge*k,
    including the end cell and the traceback (shortest gap on ties)."""
    rng = np.random.default_rng(5)
    for t in range(300):
        m, n = rng.integers(1, 40, size=2)
        c = rng.integers(0, 20, size=m).astype(np.uint8)
        s = rng.integers(0, 20, size=n).astype(np.uint8)
        if t % 2:  # related pair so that gaps appear
            s = np.concatenate([c[: m // 2], rng.integers(0, 20, size=3).astype(np.uint8), c[m // 2:]])
        go, ge = [(11, 1), (10, 1), (3, 1), (1, 2)][t % 4]
        W = np.array([0] + [go + ge * k for k in range(1, 200)], np.int32)
        score, H, cells, ops = oracle.sw_eq2(B62, W, c, s)
        r = oracle.sw(B62, go, ge, c, s, want_ops=True)
        assert r["score"] == score
        if score:
            assert tuple(r["cells"]) == tuple(cells)
            assert r["ops"] == ops


def test_linear_gap_independent_routine():
    """go = 0 reduces to single-matrix linear-gap SW (written here, 1-D rolling)."""
    rng = np.random.default_rng(8)
    for _ in range(100):
        c = rng.integers(0, 20, size=rng.integers(1, 60)).astype(np.uint8)
        s = rng.integers(0, 20, size=rng.integers(1, 60)).astype(np.uint8)
        d = int(rng.integers(1, 6))
        prev = [0] * (len(s) + 1)
        best = 0
        for i in range(1, len(c) + 1):
            cur = [0] * (len(s) + 1)
            for j in range(1, len(s) + 1):
                cur[j] = max(0, prev[j - 1] + int(B62[c[i - 1], s[j - 1]]), prev[j] - d, cur[j - 1] - d)
                best = max(best, cur[j])
            prev = cur
        assert oracle.sw_score(B62, 0, d, c, s) == best


def test_closed_forms():
    rng = np.random.default_rng(9)
    for _ in range(50):
        c = rng.integers(0, 20, size=rng.integers(1, 200)).astype(np.uint8)
        r = oracle.sw(B62, GO, GE, c, c, want_ops=True)
        # self alignment: identity path, score = sum of the diagonal
        assert r["score"] == int(B62[c, c].astype(int).sum())
        assert r["ops"] == "M" * len(c)
        assert tuple(r["cells"]) == (0, 0, len(c), len(c))
        # an exact substring scores its diagonal sum
        a, b = sorted(rng.integers(0, len(c) + 1, size=2))
        if b > a:
            sub = c[a:b]
            assert oracle.sw_score(B62, GO, GE, c, sub) == int(B62[sub, sub].astype(int).sum())
    # all-negative pair scores 0
    W, P = synth.ALPHABET.index("W"), synth.ALPHABET.index("P")
    r = oracle.sw(B62, GO, GE, np.full(5, W, np.uint8), np.full(7, P, np.uint8), want_ops=True)
    assert r["score"] == 0 and r["ins"][0] == 7


def test_symmetry_and_bound():
    rng = np.random.default_rng(10)
    for _ in range(100):
        a = rng.integers(0, 20, size=rng.integers(1, 120)).astype(np.uint8)
        b = rng.integers(0, 20, size=rng.integers(1, 120)).astype(np.uint8)
        ab = oracle.sw_score(B62, GO, GE, a, b)
        assert ab == oracle.sw_score(B62, GO, GE, b, a)
        assert ab <= min(oracle.sw_score(B62, GO, GE, a, a), oracle.sw_score(B62, GO, GE, b, b))
        assert ab == oracle.sw(B62, GO, GE, a, b)["score"]


def test_invariants_family_pairs():
    """Related pairs from the generator up to length 300: all invariants hold."""
    seqs = synth.generate("plain64")
    c = seqs.seq(0)
    for k in range(seqs.n):
        s = seqs.seq(k)
        r = oracle.sw(B62, GO, GE, c, s, want_ops=True)
        _check_alignment(B62, GO, GE, c, s, r)


def test_empty_and_degenerate():
    c = np.array([0, 1, 2], np.uint8)
    r = oracle.sw(B62, GO, GE, c, np.zeros(0, np.uint8), want_ops=True)
    assert r["score"] == 0 and r["ins"].sum() == 0
    r = oracle.sw(B62, GO, GE, np.zeros(0, np.uint8), c, want_ops=True)
    assert r["score"] == 0 and r["ins"][0] == 3
    with pytest.raises(ValueError):
        oracle.sw(B62, GO, GE, c, np.array([24], np.uint8))
