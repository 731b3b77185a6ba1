"""Phylogeny (NJ section, Fig. 4) on the GPU against the oracle, bit for bit:
p-distance counts and quotients, neighbour joining (every parent and every
branch length), and the clustered, merged tree, up to the 16.5 kb
nucleotide MSA of 672 sequences."""
import numpy as np
import pytest

import oracle
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu
GAP = 255


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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _random_msa(rng, n, w, p_gap=0.2, alpha=4, all_gap_rows=()):
    m = rng.integers(0, alpha, (n, w)).astype(np.uint8)
    m[rng.random((n, w)) < p_gap] = GAP
    for r in all_gap_rows:
        m[r] = GAP
    return m


def _families(rng, sizes, width=160, p=0.05, p_gap=0.02):
    rows = []
    for s in sizes:
        root = rng.integers(0, 4, width)
        for _ in range(s):
            r = root.copy()
            hit = rng.random(width) < p
            r[hit] = (r[hit] + rng.integers(1, 4, hit.sum())) % 4
            r = r.astype(np.uint8)
            r[rng.random(width) < p_gap] = GAP
            rows.append(r)
    return np.array(rows, np.uint8)


@pytest.mark.parametrize("n,w", [(1, 1), (5, 3), (70, 130), (130, 64), (64, 1000), (3, 0), (70, 5000), (130, 2049)])
def test_pdist_counts(H, ctx, n, w):
    import torch
    rng = np.random.default_rng(n * 1000 + w)
    m = _random_msa(rng, n, w, all_gap_rows=(0,) if n > 2 else ())
    D, mm, cc = H.halign_pdist(ctx, _dev(m), counts=True)
    torch.cuda.synchronize()
    wm, wc = oracle.pdist_counts(m)
    assert (mm.cpu().numpy() == wm).all() and (cc.cpu().numpy() == wc).all()
    assert (D.cpu().numpy() == oracle.pdist(m)).all()


@pytest.mark.parametrize("n,w", [(70, 300), (3, 67)])
def test_pdist_wide_codes(H, ctx, n, w):
    """Residue codes up to 127, next to the gap byte 255 (it differs from 127
    in bit 7 alone) and codes that share low bits with it."""
    import torch
    rng = np.random.default_rng(n + w)
    m = _random_msa(rng, n, w, alpha=128)
    m[:, ::7] = 127
    m[1, ::5] = 0x7F & GAP
    D, mm, cc = H.halign_pdist(ctx, _dev(m), counts=True)
    torch.cuda.synchronize()
    wm, wc = oracle.pdist_counts(m)
    assert (mm.cpu().numpy() == wm).all() and (cc.cpu().numpy() == wc).all()
    assert (D.cpu().numpy() == oracle.pdist(m)).all()


def test_pdist_row_lists(H, ctx):
    import torch
    rng = np.random.default_rng(5)
    m = _random_msa(rng, 90, 333)
    ra = np.array([5, 0, 89, 17, 17, 3], np.int32)
    rb = rng.permutation(90)[:71].astype(np.int32)
    D = H.halign_pdist(ctx, _dev(m), _dev(ra), _dev(rb))
    torch.cuda.synchronize()
    full = oracle.pdist(m)
    assert (D.cpu().numpy() == full[np.ix_(ra, rb)]).all()


def _nj_both(H, ctx, D):
    p, b = H.halign_nj(ctx, _dev(D))
    wp, wb = oracle.nj(D)
    assert (p == wp).all()
    assert (b == wb).all(), np.abs(b - wb).max()


@pytest.mark.parametrize("sizes", [[1], [2], [3], [4], [3, 4, 5], [20, 17, 30, 12], [60, 80, 40, 75, 45]])
def test_nj_family_distances(H, ctx, sizes):
    rng = np.random.default_rng(sum(sizes))
    m = _families(rng, sizes)
    _nj_both(H, ctx, oracle.pdist(m) * (1 - np.eye(len(m))))


def test_nj_additive_and_ties(H, ctx):
    rng = np.random.default_rng(2)
    for n in (5, 9, 33, 129, 300):
        # a tree metric with integer lengths (many exact ties in Q) and one with reals
        for integral in (True, False):
            par = [-1] + [int(rng.integers(0, v)) for v in range(1, 2 * n)]
            ln = rng.integers(1, 5, 2 * n) if integral else rng.uniform(0.1, 1.0, 2 * n)
            depth = np.zeros(2 * n)
            anc = [set([0])]
            for v in range(1, 2 * n):
                depth[v] = depth[par[v]] + ln[v]
                anc.append(anc[par[v]] | {v})
            leaves = list(range(n, 2 * n))
            D = np.zeros((n, n))
            for a in range(n):
                for b in range(n):
                    if a != b:
                        common = anc[leaves[a]] & anc[leaves[b]]
                        lca = max(common, key=lambda v: depth[v])
                        D[a, b] = depth[leaves[a]] + depth[leaves[b]] - 2 * depth[lca]
            _nj_both(H, ctx, D)
    # all distances equal: every Q ties (above 256 nodes the join runs over
    # the chip, the ties then span workgroups)
    for n in (4, 7, 64, 65, 257, 600):
        _nj_both(H, ctx, np.full((n, n), 2.5) * (1 - np.eye(n)))


@pytest.mark.parametrize("sizes", [[1], [2], [9], [10], [11], [12, 2, 8], [10, 10, 10], [40, 3, 60, 1, 25, 14],
                                   [150, 130, 120]])
def test_nj_tree_families(H, ctx, sizes):
    rng = np.random.default_rng(7 + len(sizes) * 100 + sum(sizes))
    m = _families(rng, sizes)
    for rep in range(2):
        perm = rng.permutation(len(m)).astype(np.int32)
        p, b = H.halign_nj_tree(ctx, _dev(m), perm)
        wp, wb = oracle.nj_tree(m, perm)
        assert (p == wp).all() and (b == wb).all()


def test_nj_tree_duplicates_and_gaps(H, ctx):
    """Identical rows (seeds taken by earlier identical seeds: empty clusters
    dropped), all-gap rows (distance 1 everywhere, 1 to themselves too)."""
    rng = np.random.default_rng(21)
    base = _families(rng, [6, 5])
    m = np.concatenate([base, base, base[:3], np.full((2, base.shape[1]), GAP, np.uint8)])
    for rep in range(4):
        perm = rng.permutation(len(m)).astype(np.int32)
        p, b = H.halign_nj_tree(ctx, _dev(m), perm)
        wp, wb = oracle.nj_tree(m, perm)
        assert (p == wp).all() and (b == wb).all()


def test_nj_tree_of_msas(H, ctx):
    """Trees of MSAs the library made: a protein set and a nucleotide set."""
    import torch
    seqs = synth.generate("plain64")
    msa, _ = H.halign_msa(ctx, H.Scoring(), H.DeviceSeqs(seqs), 0)
    torch.cuda.synchronize()
    perm = np.random.default_rng(1).permutation(seqs.n).astype(np.int32)
    p, b = H.halign_nj_tree(ctx, msa, perm)
    wp, wb = oracle.nj_tree(msa.cpu().numpy(), perm)
    assert (p == wp).all() and (b == wb).all()
    dna = synth.generate_dna("dna_small")
    msa, _ = H.halign_nuc_msa(ctx, H.Scoring(synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND),
                              H.DeviceSeqs(dna), synth.NUC_K)
    torch.cuda.synchronize()
    perm = np.random.default_rng(2).permutation(dna.n).astype(np.int32)
    p, b = H.halign_nj_tree(ctx, msa, perm)
    wp, wb = oracle.nj_tree(msa.cpu().numpy(), perm)
    assert (p == wp).all() and (b == wb).all()


def test_nj_tree_dna672_full_size(H, ctx):
    """The tree of the 672 x 16.5 kb nucleotide MSA in the configuration the
    benchmark times (sample from a seeded permutation), every node."""
    import torch
    print("dna672 tree: MSA", flush=True)
    dna = synth.generate_dna("dna672")
    msa, _ = H.halign_nuc_msa(ctx, H.Scoring(synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND),
                              H.DeviceSeqs(dna), synth.NUC_K)
    torch.cuda.synchronize()
    perm = synth.tree_permutation(dna.n)
    print("dna672 tree: GPU", flush=True)
    p, b = H.halign_nj_tree(ctx, msa, perm)
    print("dna672 tree: oracle", flush=True)
    wp, wb = oracle.nj_tree(msa.cpu().numpy(), perm)
    assert (p == wp).all() and (b == wb).all()
