"""The allocation-free score-only entry point against halign_sw_batch
(score-only with end cells) through the C ABI: two calls in a row on the same
GPU, the second with a smaller input, so that the second call runs on the
scratch the first one left behind."""
import numpy as np
import pytest

from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu


def _case(H, ctx, seqs, center):
    import torch
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring()
    m = ds.length(center)
    N = seqs.n
    ref = H.sw_batch(ctx, sc, ds, center, traceback=False)
    score = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    cells = torch.full((N, 4), -7, dtype=torch.int32, device="cuda")
    H.halign_sw_score_noalloc(sc, ds.seq_ptr(center), m, ds, score, cells)
    torch.cuda.synchronize()
    assert torch.equal(score, ref["score"])
    assert torch.equal(cells, ref["cells"])
    # score only, without cells
    score2 = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    H.halign_sw_score_noalloc(sc, ds.seq_ptr(center), m, ds, score2)
    torch.cuda.synchronize()
    assert torch.equal(score2, ref["score"])


def test_noalloc_matches_sw_batch_twice():
    import paper_1704_00878_amd as H
    H.lib()
    ctx = H.Context(0)
    big = synth.generate("batch20k", n_seqs=3000, seed=41)
    rng = np.random.default_rng(9)
    parts = [big.seq(k) for k in range(big.n)]
    parts[17] = np.zeros(0, np.uint8)                      # an empty sequence
    parts[18] = rng.integers(0, 24, 1).astype(np.uint8)     # one residue
    big = synth.SeqSet.from_list(parts)
    _case(H, ctx, big, 0)
    small = synth.generate("plain64", n_seqs=70, seed=42)   # fewer groups, shorter rows
    _case(H, ctx, small, 5)
    ctx.close()
