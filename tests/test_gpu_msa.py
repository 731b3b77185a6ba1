"""GPU parity for the center-star merge, rows, center selection and avg SP,
bit-exact against the oracle through the C ABI, plus the full-size batch20k
workload in the launch configuration the benchmark times (sampled pairs
checked one by one against the oracle, properties checked on every row)."""
import numpy as np
import pytest

import oracle
from golden_cases import load, row_text
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_1704_00878_amd as H
    H.lib()
    return H


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


def _msa(H, ctx, seqs, center, sc=None):
    import torch
    sc = sc or H.Scoring()
    ds = H.DeviceSeqs(seqs)
    msa, c = H.halign_msa(ctx, sc, ds, center)
    torch.cuda.synchronize()
    return msa.cpu().numpy(), c


@pytest.mark.parametrize("center", [0, 7, 63])
def test_msa_plain64(H, ctx, center):
    seqs = synth.generate("plain64")
    got, c = _msa(H, ctx, seqs, center)
    ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, center)
    assert c == center
    assert got.shape == ref["msa"].shape
    assert (got == ref["msa"]).all()


def test_msa_hand_case(H, ctx):
    case = [c for c in load() if c["kind"] == "msa"][0]
    seqs = synth.SeqSet.from_list(case["seqs"])
    sc = H.Scoring(gap_open=case["go"], gap_extend=case["ge"])
    got, _ = _msa(H, ctx, seqs, case["center"], sc)
    assert [row_text(r) for r in got] == case["rows"]
    import torch
    sp, spb = H.halign_sp_score(sc, torch.from_numpy(got).cuda())
    assert sp == case["sp"] and spb == case["sp_blosum"]


def test_msa_edge_sets(H, ctx):
    rng = np.random.default_rng(12)
    # empty sequences, a single sequence, duplicates, unrelated sequences
    base = synth.generate("plain64", n_seqs=10)
    seqs = synth.SeqSet.from_list([base.seq(0), np.zeros(0, np.uint8), base.seq(0), base.seq(3)[:5],
                                   rng.integers(0, 20, size=300).astype(np.uint8), base.seq(9)])
    for center in (0, 4):
        got, _ = _msa(H, ctx, seqs, center)
        ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, center)
        assert (got == ref["msa"]).all()
    one = synth.SeqSet.from_list([base.seq(2)])
    got, _ = _msa(H, ctx, one, 0)
    assert (got[0] == base.seq(2)).all()


def test_msa_wide_rows(H, ctx):
    """Rows wider than one LDS chunk of columns (long unrelated flanks) and
    rows that start at every alignment modulo 16."""
    rng = np.random.default_rng(5)
    base = synth.generate("plain64", n_seqs=8)
    parts = [base.seq(0), rng.integers(0, 20, size=9000).astype(np.uint8), base.seq(3),
             rng.integers(0, 20, size=12345).astype(np.uint8), np.zeros(0, np.uint8), base.seq(5)[10:]]
    parts += [base.seq(k % 8)[: 40 + 7 * k] for k in range(17)]
    seqs = synth.SeqSet.from_list(parts)
    got, _ = _msa(H, ctx, seqs, 0)
    ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, 0)
    assert ref["width"] > 8192
    assert got.shape == ref["msa"].shape
    assert (got == ref["msa"]).all()


@pytest.mark.parametrize("kernel", ["chunk", "lds"])
def test_rows_kernels(H, ctx, kernel, monkeypatch):
    """Both row kernels on the same sets (each is the default for one range
    of center lengths): the hand case, edge sets, wide rows, rows at every
    alignment, a center longer than the lane kernel's threshold."""
    monkeypatch.setenv("HALIGN_ROWS", kernel)
    rng = np.random.default_rng(17)
    base = synth.generate("plain64", n_seqs=12)
    sets = [
        synth.SeqSet.from_list([base.seq(0), np.zeros(0, np.uint8), base.seq(0), base.seq(3)[:5],
                                rng.integers(0, 20, size=300).astype(np.uint8), base.seq(9)]),
        synth.SeqSet.from_list([base.seq(1), rng.integers(0, 20, size=3000).astype(np.uint8)]
                               + [base.seq(k % 12)[: 20 + 9 * k] for k in range(40)]),
        synth.SeqSet.from_list([rng.integers(0, 20, size=5000).astype(np.uint8)]
                               + [base.seq(k) for k in range(12)] + [np.zeros(0, np.uint8)]),
    ]
    for seqs in sets:
        got, _ = _msa(H, ctx, seqs, 0)
        ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, 0)
        assert got.shape == ref["msa"].shape
        assert (got == ref["msa"]).all()


def test_merge_and_rows_calls(H, ctx):
    """halign_merge and halign_emit_rows on oracle-made center-star vectors."""
    import torch
    seqs = synth.generate("plain64")
    ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, 0)
    N, m = seqs.n, len(seqs.seq(0))
    ins = torch.from_numpy(ref["ins"].view(np.int16)).cuda()
    G = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    col = torch.empty(m + 1, dtype=torch.int64, device="cuda")
    W = H.halign_merge(ctx, ins, N, m, G, col)
    assert W == ref["width"]
    assert (G.cpu().numpy() == ref["G"]).all() and (col.cpu().numpy() == ref["col"]).all()
    al = np.zeros((N, (m + 31) // 32), np.uint32)
    for k in range(N):
        for p in np.nonzero(ref["aligned"][k])[0]:
            al[k, p >> 5] |= np.uint32(1) << np.uint32(p & 31)
    alt = torch.from_numpy(al.view(np.int32)).cuda()
    msa = torch.empty((N, W), dtype=torch.uint8, device="cuda")
    ds = H.DeviceSeqs(seqs)
    H.halign_emit_rows(ctx, ds, m, ins, alt, G, col, W, msa)
    torch.cuda.synchronize()
    assert (msa.cpu().numpy() == ref["msa"]).all()


# center selection runs the packed 16-bit strip kernel when scores fit, else
# the 32-bit one; HALIGN_STRIP32=1 forces the 32-bit kernel
STRIPS = [None, "1"]


@pytest.fixture(params=STRIPS, ids=["strip16", "strip32"])
def strip(request, monkeypatch):
    if request.param:
        monkeypatch.setenv("HALIGN_STRIP32", request.param)
    else:
        monkeypatch.delenv("HALIGN_STRIP32", raising=False)
    return request.param


def _mixed_set(n, seed):
    """Family sequences plus an empty one, a 1-residue one and a lone
    unrelated one: spans several 128-partner groups and 16-row strips."""
    base = synth.generate("plain64", n_seqs=n, seed=seed)
    rng = np.random.default_rng(seed)
    extra = [np.zeros(0, np.uint8), np.array([4], np.uint8), rng.integers(0, 20, 97).astype(np.uint8)]
    seqs = [base.seq(k) for k in range(base.n)]
    for q, x in enumerate(extra):
        seqs.insert(37 * q + 5, x)
    return synth.SeqSet.from_list(seqs)


def test_center_exact(H, ctx, strip):
    import torch
    seqs = synth.generate("plain64", n_seqs=24, seed=9)
    best, sums = oracle.center_exact(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets)
    ds = H.DeviceSeqs(seqs)
    d = torch.empty(seqs.n, dtype=torch.int64, device="cuda")
    c = H.halign_center_exact(ctx, H.Scoring(), ds, d)
    assert c == best
    assert (d.cpu().numpy() == sums).all()


def test_center_exact_plain64_and_msa(H, ctx):
    seqs = synth.generate("plain64")
    best, sums = oracle.center_exact(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets)
    got, c = _msa(H, ctx, seqs, H.HALIGN_CENTER_EXACT)
    assert c == best
    ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, best)
    assert (got == ref["msa"]).all()


def test_center_exact_groups(H, ctx, strip):
    import torch
    seqs = _mixed_set(200, 12)
    best, sums = oracle.center_exact(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets)
    ds = H.DeviceSeqs(seqs)
    d = torch.empty(seqs.n, dtype=torch.int64, device="cuda")
    c = H.halign_center_exact(ctx, H.Scoring(), ds, d)
    assert c == best
    assert (d.cpu().numpy() == sums).all()


def test_center_exact_sliced(H, ctx, strip, monkeypatch):
    """All pairs in launches of 3 groups each (a counter reset between them)."""
    import torch
    monkeypatch.setenv("HALIGN_GROUP_SLICE", "3")
    seqs = _mixed_set(200, 14)
    best, sums = oracle.center_exact(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets)
    ds = H.DeviceSeqs(seqs)
    d = torch.empty(seqs.n, dtype=torch.int64, device="cuda")
    c = H.halign_center_exact(ctx, H.Scoring(), ds, d)
    assert c == best
    assert (d.cpu().numpy() == sums).all()


def test_center_judge_groups(H, ctx, strip):
    import torch
    seqs = _mixed_set(200, 13)
    cand = [5, 0, 42, 79, 150, 202, 6]   # includes the empty (5) and 1-residue (42) sequences
    jb, js = oracle.center_judge(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, cand)
    ds = H.DeviceSeqs(seqs)
    ct = torch.tensor(cand, dtype=torch.int32, device="cuda")
    d = torch.empty(len(cand), dtype=torch.int64, device="cuda")
    c = H.halign_center_judge(ctx, H.Scoring(), ds, ct, d)
    assert c == jb
    assert (d.cpu().numpy() == js).all()


def test_center_exact_long_falls_back(H, ctx):
    """11 x 1500 >= 15000: the 16-bit bound fails and the 32-bit kernel runs."""
    import torch
    rng = np.random.default_rng(3)
    root = rng.integers(0, 20, 1500).astype(np.uint8)
    mut = root.copy()
    mut[rng.integers(0, 1500, 200)] = rng.integers(0, 20, 200).astype(np.uint8)
    seqs = synth.SeqSet.from_list([root, mut, root[:700], rng.integers(0, 20, 300).astype(np.uint8)])
    best, sums = oracle.center_exact(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets)
    ds = H.DeviceSeqs(seqs)
    d = torch.empty(seqs.n, dtype=torch.int64, device="cuda")
    c = H.halign_center_exact(ctx, H.Scoring(), ds, d)
    assert c == best
    assert (d.cpu().numpy() == sums).all()


def test_center_exact_at_the_bound(H, ctx, strip):
    """Scores up to the 16-bit kernel's bound (max S x longest + go + ge <
    15000): tryptophan runs of 1362 residues (S = 11) score 14,982 against
    each other, with mutated copies, a shorter run and an unrelated sequence."""
    import torch
    rng = np.random.default_rng(5)
    w = np.full(1362, 17, np.uint8)   # W in the NCBI order
    mut = w.copy()
    mut[rng.integers(0, 1362, 100)] = rng.integers(0, 20, 100).astype(np.uint8)
    seqs = synth.SeqSet.from_list([w, mut, w.copy(), w[:900].copy(), rng.integers(0, 20, 400).astype(np.uint8)])
    best, sums = oracle.center_exact(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets)
    ds = H.DeviceSeqs(seqs)
    d = torch.empty(seqs.n, dtype=torch.int64, device="cuda")
    c = H.halign_center_exact(ctx, H.Scoring(), ds, d)
    assert c == best
    assert (d.cpu().numpy() == sums).all()
    assert sums[0] >= 2 * 14982


def test_center_judge(H, ctx, strip):
    import torch
    seqs = synth.generate("plain64", n_seqs=40, seed=4)
    cand = [5, 0, 17, 39, 22]
    jb, js = oracle.center_judge(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, cand)
    ds = H.DeviceSeqs(seqs)
    ct = torch.tensor(cand, dtype=torch.int32, device="cuda")
    d = torch.empty(len(cand), dtype=torch.int64, device="cuda")
    c = H.halign_center_judge(ctx, H.Scoring(), ds, ct, d)
    assert c == jb
    assert (d.cpu().numpy() == js).all()


def test_center_judge_sample(H, ctx, strip):
    """Sums over a common partner sample (a candidate against itself scores 0),
    against the oracle's pairwise scores."""
    import torch
    seqs = synth.generate("plain64", n_seqs=40, seed=14)
    cand = [5, 0, 17, 39]
    partners = [3, 5, 9, 17, 30, 39, 0, 22]
    ds = H.DeviceSeqs(seqs)
    ct = torch.tensor(cand, dtype=torch.int32, device="cuda")
    d = torch.empty(len(cand), dtype=torch.int64, device="cuda")
    c = H.halign_center_judge_sample(ctx, H.Scoring(), ds, ct, np.array(partners), d)
    want = [sum(0 if p == a else oracle.sw_score(synth.BLOSUM62, 11, 1, seqs.seq(a), seqs.seq(p)) for p in partners)
            for a in cand]
    assert list(d.cpu().numpy()) == want
    best = max(range(len(cand)), key=lambda q: (want[q], -cand[q]))
    assert c == cand[best]


def test_sw_pairs(H, ctx):
    import torch
    seqs = synth.generate("plain64", n_seqs=50, seed=6)
    rng = np.random.default_rng(2)
    anchors = rng.integers(0, seqs.n, size=3).astype(np.int32)
    partners = rng.integers(0, seqs.n, size=3 * 64).astype(np.int32)
    ds = H.DeviceSeqs(seqs)
    out = torch.empty(3 * 64, dtype=torch.int32, device="cuda")
    H.halign_sw_pairs(ctx, H.Scoring(), ds, anchors, partners, out)
    got = out.cpu().numpy()
    for q in range(3):
        for l in range(64):
            a, b = int(anchors[q]), int(partners[64 * q + l])
            want = 0 if a == b else oracle.sw_score(synth.BLOSUM62, 11, 1, seqs.seq(a), seqs.seq(b))
            assert got[64 * q + l] == want, (q, l)


def test_sp_score_random(H):
    import torch
    rng = np.random.default_rng(8)
    a = rng.integers(0, 20, size=(37, 91)).astype(np.uint8)
    a[rng.random(a.shape) < 0.3] = 255
    sp, spb = H.halign_sp_score(H.Scoring(), torch.from_numpy(a).cuda())
    assert sp == oracle.sp_columns(a) == oracle.sp_pairs(a)
    assert spb == oracle.sp_blosum(synth.BLOSUM62, 1, a)


@pytest.mark.parametrize("plan", ["default", "packed"])
def test_batch20k_full_size(H, ctx, plan, monkeypatch):
    """The benchmark's workload and launch configuration (the plan its tuner
    picks: the packed 16-bit kernel with 10 rows per lane on 32-lane streams;
    and the untuned default): every row restores its input, G and the width
    follow from the vectors, and 300 sampled pairs equal the oracle bit for
    bit."""
    import torch
    if plan == "packed":
        monkeypatch.setenv("HALIGN_STREAM_LANES", "32")
        monkeypatch.setenv("HALIGN_STREAM_PACK", "1")
    seqs = synth.generate("batch20k")
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring()
    out = H.sw_batch(ctx, sc, ds, 0, traceback=True)
    if plan == "packed":   # 32-lane streams of ceil(311 / 32) = 10 rows, packed
        assert ctx.last_plan()["packed"] == 1
    msa, c = H.halign_msa(ctx, sc, ds, 0)
    torch.cuda.synchronize()
    score = out["score"].cpu().numpy()
    cells = out["cells"].cpu().numpy()
    ins = out["ins"].cpu().numpy().view(np.uint16)
    m = len(seqs.seq(0))
    al = H.aligned_to_bool(out["aligned"].cpu().numpy(), m)
    M = msa.cpu().numpy()
    ins_c = ins.copy()
    ins_c[0] = 0
    G = ins_c.max(axis=0)
    assert M.shape == (seqs.n, m + int(G.sum()))
    assert (ins.sum(axis=1) + al.sum(axis=1) == seqs.lengths()).all()
    for k in range(seqs.n):
        row = M[k]
        assert (row[row != 255] == seqs.seq(k)).all(), k
    rng = np.random.default_rng(0)
    pick = np.concatenate([[0, 1, seqs.n - 1], rng.choice(seqs.n, size=297, replace=False)])
    c0 = seqs.seq(0)
    for k in pick:
        r = oracle.sw(synth.BLOSUM62, 11, 1, c0, seqs.seq(int(k)))
        assert score[k] == r["score"], k
        assert tuple(cells[k]) == tuple(r["cells"]), k
        assert (ins[k] == r["ins"]).all(), k
        assert (al[k] == r["aligned"]).all(), k
