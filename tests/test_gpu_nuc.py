"""Nucleotide center star (trie section) on the GPU against the oracle:
scores, center-star vectors and MSA bytes, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu
NM, GO, GE = synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND


@pytest.fixture(scope="module")
def H():
    import paper_1704_00878_amd as H
    return H


@pytest.fixture(scope="module")
def ctx(H):
    return H.Context(0)


def _bits(words, m):
    w = np.asarray(words, dtype=np.uint32)
    b = ((w[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(w.shape[0], -1)
    return b[:, :m].astype(np.uint8)


def _vectors(H, ctx, seqs, center, k):
    import torch
    ds = H.DeviceSeqs(seqs)
    N = seqs.n
    m = int(seqs.offsets[center + 1] - seqs.offsets[center])
    score = torch.empty(N, dtype=torch.int32, device="cuda")
    ins = torch.empty((N, m + 1), dtype=torch.int16, device="cuda")
    al = torch.empty((N, max((m + 31) // 32, 1)), dtype=torch.int32, device="cuda")
    G = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    H.halign_nuc_align(ctx, H.Scoring(NM, GO, GE), ds, center, k, score, ins, al, G)
    torch.cuda.synchronize()
    return (score.cpu().numpy(), ins.cpu().numpy().view(np.uint16), _bits(al.cpu().numpy().view(np.uint32), m),
            G.cpu().numpy())


def _oracle_pairs(seqs, center, k):
    c = seqs.seq(center)
    out = [oracle.nuc_align(NM, GO, GE, k, c, seqs.seq(x)) for x in range(seqs.n)]
    return (np.array([r["score"] for r in out], np.int32), np.stack([r["ins"] for r in out]),
            np.stack([r["aligned"] for r in out]) if len(c) else np.zeros((seqs.n, 0), np.uint8))


@pytest.mark.parametrize("k", [16, 4, 11, 32])
def test_vectors_dna_small(H, ctx, k):
    seqs = synth.generate_dna("dna_small")
    sc, ins, al, G = _vectors(H, ctx, seqs, 0, k)
    wsc, wins, wal = _oracle_pairs(seqs, 0, k)
    assert (sc == wsc).all()
    assert (ins == wins).all()
    assert (al == wal).all()
    assert (G == wins[1:].max(0)).all()


def test_msa_dna_small_center3(H, ctx):
    seqs = synth.generate_dna("dna_small", n_seqs=30, seed=77)
    c = 3
    sub = seqs.subset([c] + [x for x in range(seqs.n) if x != c])   # the oracle's MSA takes sequence 0
    ref = oracle.nuc_msa(NM, GO, GE, 16, sub.residues, sub.offsets)
    msa, score = H.halign_nuc_msa(ctx, H.Scoring(NM, GO, GE), H.DeviceSeqs(sub), 16, center=0)
    assert msa.shape[1] == ref["width"]
    assert (msa.cpu().numpy() == ref["msa"]).all()
    assert (score.cpu().numpy() == ref["score"]).all()
    # and with the center given by index (rows in input order)
    msa2, score2 = H.halign_nuc_msa(ctx, H.Scoring(NM, GO, GE), H.DeviceSeqs(seqs), 16, center=c)
    order = [c] + [x for x in range(seqs.n) if x != c]
    assert (msa2.cpu().numpy()[order] == ref["msa"]).all()


def test_edge_sequences(H, ctx):
    """Empty, shorter than k, all N, identical to the center, unrelated (no
    anchor: one stretch over everything), a center with repeated segments."""
    rng = np.random.default_rng(9)
    c = rng.integers(0, 4, 700).astype(np.uint8)
    c[64:80] = c[0:16]                      # a repeated segment: not indexed
    c[200] = 4                              # an N inside a segment
    seqs = synth.SeqSet.from_list([
        c, np.zeros(0, np.uint8), c[5:14], np.full(40, 4, np.uint8), c.copy(),
        rng.integers(0, 4, 260).astype(np.uint8), np.concatenate([c[300:], c[:300]]),
        np.concatenate([c[:100], rng.integers(0, 4, 50).astype(np.uint8), c[100:]])])
    sc, ins, al, G = _vectors(H, ctx, seqs, 0, 16)
    wsc, wins, wal = _oracle_pairs(seqs, 0, 16)
    assert (sc == wsc).all() and (ins == wins).all() and (al == wal).all()


def test_mito_like_subset(H, ctx):
    """64 sequences of the 16.5 kb set, every vector against the oracle."""
    seqs = synth.generate_dna("dna672", n_seqs=64)
    sc, ins, al, G = _vectors(H, ctx, seqs, 0, synth.NUC_K)
    wsc, wins, wal = _oracle_pairs(seqs, 0, synth.NUC_K)
    assert (sc == wsc).all() and (ins == wins).all() and (al == wal).all()


@pytest.mark.parametrize("kernel", ["chunk", "lds"])
def test_msa_long_center(H, ctx, kernel, monkeypatch):
    """A 16.5 kb center, with either row kernel (the LDS one needs more than
    64 KiB per workgroup here)."""
    monkeypatch.setenv("HALIGN_ROWS", kernel)
    seqs = synth.generate_dna("dna672", n_seqs=12, seed=5)
    ref = oracle.nuc_msa(NM, GO, GE, synth.NUC_K, seqs.residues, seqs.offsets)
    msa, score = H.halign_nuc_msa(ctx, H.Scoring(NM, GO, GE), H.DeviceSeqs(seqs), synth.NUC_K)
    assert msa.shape[1] == ref["width"]
    assert (msa.cpu().numpy() == ref["msa"]).all()
    assert (score.cpu().numpy() == ref["score"]).all()


def test_stretch_widths(H, ctx):
    """Stretches around the kernels' boundaries: up to 32 columns (one lane)
    or wider (a wavefront, 64-column strips, 64-row boundary chunks), with
    center spans of 0 .. 130 rows: a center region replaced by random bases."""
    rng = np.random.default_rng(31)
    c = rng.integers(0, 4, 1200).astype(np.uint8)
    sizes = [0, 1, 15, 31, 32, 33, 47, 63, 64, 65, 96, 127, 129]
    seqs = [c]
    for h in sizes:
        for w in sizes:
            s0 = 160 + int(rng.integers(0, 16))
            seqs.append(np.concatenate([c[:s0], rng.integers(0, 4, w).astype(np.uint8), c[s0 + h:]]))
    seqs = synth.SeqSet.from_list(seqs)
    sc, ins, al, G = _vectors(H, ctx, seqs, 0, 16)
    wsc, wins, wal = _oracle_pairs(seqs, 0, 16)
    assert (sc == wsc).all() and (ins == wins).all() and (al == wal).all()
    assert (G == wins[1:].max(0)).all()
