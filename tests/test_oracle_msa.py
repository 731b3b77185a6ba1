"""Oracle pins for the center-star merge, the rows, the exact center and avg SP."""
import numpy as np
import pytest

import oracle
from golden_cases import load, row_text
from oracle_par import sp_from_profile
from paper_1704_00878_amd import synth

B62 = synth.BLOSUM62
GO, GE = synth.GAP_OPEN, synth.GAP_EXTEND


@pytest.mark.parametrize("case", [c for c in load() if c["kind"] == "case"], ids=lambda c: c["name"])
def test_hand_cases_pairwise(case):
    r = oracle.sw(B62, case["go"], case["ge"], case["center"], case["seq"], want_ops=True)
    assert r["score"] == case["score"]
    assert tuple(int(x) for x in r["cells"]) == case["cells"]
    assert r["ops"] == case["ops"]
    assert (r["ins"] == case["ins"]).all()
    assert (r["aligned"] == case["aligned"]).all()


@pytest.mark.parametrize("case", [c for c in load() if c["kind"] == "msa"], ids=lambda c: c["name"])
def test_hand_cases_msa(case):
    seqs = synth.SeqSet.from_list(case["seqs"])
    out = oracle.msa(B62, case["go"], case["ge"], seqs.residues, seqs.offsets, case["center"])
    assert (out["G"] == case["G"]).all()
    assert [row_text(r) for r in out["msa"]] == case["rows"]
    assert oracle.sp_pairs(out["msa"]) == case["sp"]
    assert oracle.sp_columns(out["msa"]) == case["sp"]
    assert oracle.sp_blosum(B62, case["ge"], out["msa"]) == case["sp_blosum"]


def _strip_gapgap(a, b):
    keep = ~((a == 255) & (b == 255))
    return a[keep], b[keep]


def test_merge_invariants_family():
    seqs = synth.generate("plain64")
    out = oracle.msa(B62, GO, GE, seqs.residues, seqs.offsets, 0)
    msa, G, W = out["msa"], out["G"], out["width"]
    N, m = seqs.n, len(seqs.seq(0))
    assert W == m + int(G.sum())
    assert (G == out["ins"].max(axis=0)).all()
    # no all-gap column
    assert ((msa != 255).sum(axis=0) > 0).all()
    # removing gaps restores every input
    for k in range(N):
        row = msa[k]
        assert (row[row != 255] == seqs.seq(k)).all()
    # center row is the gapped center
    assert (msa[0][msa[0] != 255] == seqs.seq(0)).all()
    assert (out["ins"][0] == 0).all() and (out["aligned"][0] == 1).all()
    # projection onto (center, k) equals the N = 2 MSA of (center, s_k)
    for k in range(1, N):
        two = synth.SeqSet.from_list([seqs.seq(0), seqs.seq(k)])
        o2 = oracle.msa(B62, GO, GE, two.residues, two.offsets, 0)
        a, b = _strip_gapgap(msa[0], msa[k])
        assert (a == o2["msa"][0]).all() and (b == o2["msa"][1]).all()


def test_pairwise_from_n2():
    """N = 2 reproduces the pairwise alignment: core columns equal the ops."""
    seqs = synth.generate("plain64")
    c = seqs.seq(0)
    for k in (1, 5, 17):
        s = seqs.seq(k)
        r = oracle.sw(B62, GO, GE, c, s, want_ops=True)
        two = synth.SeqSet.from_list([c, s])
        o2 = oracle.msa(B62, GO, GE, two.residues, two.offsets, 0)
        rc, rs = o2["msa"]
        i0, j0, i1, j1 = [int(x) for x in r["cells"]]
        # columns of the core: from c_{i0+1}'s column to c_{i1}'s column
        start = int(o2["col"][i0] + o2["G"][i0])
        end = int(o2["col"][i1 - 1] + o2["G"][i1 - 1]) + 1
        ops = "".join("M" if (x != 255 and y != 255) else ("I" if x == 255 else "D")
                      for x, y in zip(rc[start:end], rs[start:end]) if not (x == 255 and y == 255))
        assert ops == r["ops"]


def test_permutation_and_replication():
    seqs = synth.generate("plain64")
    base = oracle.msa(B62, GO, GE, seqs.residues, seqs.offsets, 0)
    rng = np.random.default_rng(0)
    perm = np.concatenate([[0], 1 + rng.permutation(seqs.n - 1)])
    p = seqs.subset(perm)
    o = oracle.msa(B62, GO, GE, p.residues, p.offsets, 0)
    assert (o["G"] == base["G"]).all() and o["width"] == base["width"]
    assert (o["msa"] == base["msa"][perm]).all()
    # x3 replication (Table 1 builds its 100x/1000x sets this way)
    rep = seqs.subset(list(range(seqs.n)) * 3)
    o3 = oracle.msa(B62, GO, GE, rep.residues, rep.offsets, 0)
    assert (o3["G"] == base["G"]).all()
    assert (o3["msa"] == np.concatenate([base["msa"]] * 3)).all()


def test_sp_column_formula_matches_pair_loop():
    rng = np.random.default_rng(4)
    for _ in range(20):
        N, W = rng.integers(2, 12), rng.integers(1, 40)
        a = rng.integers(0, 6, size=(N, W)).astype(np.uint8)
        a[rng.random((N, W)) < 0.3] = 255
        assert oracle.sp_pairs(a) == oracle.sp_columns(a)


def test_center_exact_brute():
    seqs = synth.generate("plain64", n_seqs=12)
    best, sums = oracle.center_exact(B62, GO, GE, seqs.residues, seqs.offsets)
    N = seqs.n
    M = np.zeros((N, N), np.int64)
    for a in range(N):
        for b in range(N):
            if a != b:
                M[a, b] = oracle.sw(B62, GO, GE, seqs.seq(a), seqs.seq(b))["score"]
    assert (M == M.T).all()
    assert (sums == M.sum(axis=1)).all()
    assert best == int(np.argmax(M.sum(axis=1)))
    jb, js = oracle.center_judge(B62, GO, GE, seqs.residues, seqs.offsets, [5, 3, best])
    assert jb == best and js[2] == sums[best]


def test_center_ties_lowest_index():
    # identical sequences: every candidate ties, lowest index wins
    s = synth.encode("MKVLAAGIW")
    seqs = synth.SeqSet.from_list([s, s, s])
    best, sums = oracle.center_exact(B62, GO, GE, seqs.residues, seqs.offsets)
    assert best == 0 and len(set(sums.tolist())) == 1
    jb, _ = oracle.center_judge(B62, GO, GE, seqs.residues, seqs.offsets, [2, 1])
    assert jb == 1


def test_column_profile_hand():
    G = 255
    a = np.array([[0, 1, G, 2],
                  [0, G, G, 2],
                  [3, 1, 1, 2]], np.uint8)
    P = oracle.column_profile(a, 4)
    assert P.tolist() == [[2, 0, 0, 1, 0],
                          [0, 2, 0, 0, 1],
                          [0, 1, 0, 0, 2],
                          [0, 0, 3, 0, 0]]
    with pytest.raises(ValueError):
        oracle.column_profile(np.array([[4]], np.uint8), 4)


def test_column_profile_pins_sp():
    """Counts per column sum to the rows; SP and BLOSUM SP taken from the
    profile equal the explicit pair loops (a slot or column mix-up breaks the
    BLOSUM sum, whose matrix entries differ per residue)."""
    rng = np.random.default_rng(21)
    B62 = np.asarray(synth.BLOSUM62, np.int8)
    for n, w in ((2, 1), (7, 13), (40, 57)):
        a = rng.integers(0, 24, (n, w)).astype(np.uint8)
        a[rng.random((n, w)) < 0.3] = 255
        P = oracle.column_profile(a, 24)
        assert (P.sum(1) == n).all()
        sp, bl = sp_from_profile(P, B62, 1)
        assert sp == oracle.sp_pairs(a)
        assert bl == oracle.sp_blosum(B62, 1, a)
