"""GPU parity at the full sizes of the workloads, in the launch plans the
benchmark and the tuner use, against the oracle (threaded over host cores,
each thread running the unchanged single-threaded routine):

- batch20k (20,000 sequences): every pair (score, cells, insertion vector,
  aligned bits) and every MSA byte, in the tuned plan, the pinned packed plan
  (10 rows per lane on 32-lane streams) and the untuned default;
- longtail200k (200,000 sequences, lengths up to 2,000): every pair and every
  MSA byte in its tuned plan (packed kernel, 7 rows per lane on 16-lane
  streams);
- ultra1m (1,000,000 sequences) through the one-pair-per-lane route with a
  workspace cap that splits the batch into chunks: 2% of the pairs and their
  MSA rows bit for bit, and on every row: the row restores its sequence and
  the width follows from the merged insertion vector."""
import numpy as np
import pytest

import oracle_par
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu

S62, GO, GE = synth.BLOSUM62, synth.GAP_OPEN, synth.GAP_EXTEND


@pytest.fixture(scope="module")
def H():
    import paper_1704_00878_amd as H
    H.lib()
    return H


def _host(H, out, m):
    return (out["score"].cpu().numpy(), out["cells"].cpu().numpy(), out["ins"].cpu().numpy().view(np.uint16),
            H.aligned_to_bool(out["aligned"].cpu().numpy(), m))


def _compare_pairs(got, ref, idx=None):
    names = ("score", "cells", "ins", "aligned")
    for name, g, r in zip(names, got, ref):
        g = g if idx is None else g[idx]
        bad = np.nonzero((g != r).reshape(len(r), -1).any(axis=1))[0]
        assert len(bad) == 0, f"{name} differs at {bad[:10]} (of {len(r)})"


def _plan(monkeypatch, lanes=None, pack=False):
    for k in ("HALIGN_STREAM_LANES", "HALIGN_STREAM_PACK", "HALIGN_ROUTE"):
        monkeypatch.delenv(k, raising=False)
    if lanes:
        monkeypatch.setenv("HALIGN_STREAM_LANES", str(lanes))
    if pack:
        monkeypatch.setenv("HALIGN_STREAM_PACK", "1")


@pytest.fixture(scope="module")
def batch20k():
    seqs = synth.generate("batch20k")
    ref = oracle_par.msa(S62, GO, GE, seqs, 0)
    return seqs, ref


@pytest.mark.parametrize("plan", ["tuned", "packed", "default"])
def test_batch20k_every_pair_and_byte(H, batch20k, plan, monkeypatch):
    import torch
    seqs, ref = batch20k
    _plan(monkeypatch, *( (32, True) if plan == "packed" else (None, False)))
    ctx = H.Context(0)
    ctx.set_autotune(plan == "tuned")
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring()
    print(f"batch20k plan {plan}", flush=True)
    out = H.sw_batch(ctx, sc, ds, 0, traceback=True)
    torch.cuda.synchronize()
    p = ctx.last_plan()
    print(f"batch20k: plan {p}", flush=True)
    if plan == "packed":   # 32-lane streams of ceil(311 / 32) = 10 rows, packed
        assert p["packed"] == 1 and ctx.last_stats()["route"] == 0
    m = len(seqs.seq(0))
    _compare_pairs(_host(H, out, m), (ref["score"], ref["cells"], ref["ins"], ref["aligned"]))
    msa, c = H.halign_msa(ctx, sc, ds, 0)
    torch.cuda.synchronize()
    M = msa.cpu().numpy()
    assert M.shape == ref["msa"].shape
    bad = np.nonzero((M != ref["msa"]).any(axis=1))[0]
    assert len(bad) == 0, f"MSA rows differ: {bad[:10]}"
    ctx.close()


@pytest.mark.timeout(600)
def test_longtail200k_every_pair_and_byte(H, monkeypatch):
    """The tuned plan of this workload: packed kernel, R = ceil(101 / 16) = 7
    rows per lane on 16-lane streams (pinned here; the center has 101
    residues)."""
    import torch
    seqs = synth.generate("longtail200k")
    m = len(seqs.seq(0))
    assert m == 101 and (m + 15) // 16 == 7
    print("longtail200k: oracle", flush=True)
    ref = oracle_par.msa(S62, GO, GE, seqs, 0)
    _plan(monkeypatch, 16, True)
    ctx = H.Context(0)
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring()
    print("longtail200k: GPU", flush=True)
    out = H.sw_batch(ctx, sc, ds, 0, traceback=True)
    torch.cuda.synchronize()
    p = ctx.last_plan()
    assert p["packed"] == 1 and ctx.last_stats()["route"] == 0
    _compare_pairs(_host(H, out, m), (ref["score"], ref["cells"], ref["ins"], ref["aligned"]))
    msa, _ = H.halign_msa(ctx, sc, ds, 0)
    torch.cuda.synchronize()
    assert tuple(msa.shape) == ref["msa"].shape
    M = msa.cpu().numpy()
    bad = np.nonzero((M != ref["msa"]).any(axis=1))[0]
    assert len(bad) == 0, f"MSA rows differ: {bad[:10]}"
    ctx.close()


@pytest.mark.timeout(900)
def test_ultra1m_strip_route_in_chunks(H, monkeypatch):
    import torch
    print("ultra1m: generating", flush=True)
    seqs = synth.generate("ultra1m")
    N = seqs.n
    c0 = seqs.seq(0)
    m = len(c0)
    _plan(monkeypatch)
    # the traceback codes of the strip route take about 25 GB here: a 5 GB cap
    # splits the batch into at least 4 chunks
    ctx = H.Context(0, workspace_cap=5 << 30)
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring()
    print("ultra1m: SW batch", flush=True)
    out = H.sw_batch(ctx, sc, ds, 0, traceback=True, route=H.HALIGN_ROUTE_INTER)
    torch.cuda.synchronize()
    st = ctx.last_stats()
    print(f"ultra1m: stats {st}", flush=True)
    assert st["route"] == 1 and st["chunks"] >= 4
    rng = np.random.default_rng(2024)
    lens = seqs.lengths()
    idx = np.unique(np.concatenate([[0, 1, N - 1, int(np.argmax(lens)), int(np.argmin(lens))],
                                    rng.choice(N, size=N // 50, replace=False)]))
    assert len(idx) >= N // 50
    ti = torch.from_numpy(idx).cuda()
    got = (out["score"][ti].cpu().numpy(), out["cells"][ti].cpu().numpy(),
           out["ins"][ti].cpu().numpy().view(np.uint16), H.aligned_to_bool(out["aligned"][ti].cpu().numpy(), m))
    print(f"ultra1m: oracle on {len(idx)} pairs", flush=True)
    ref = oracle_par.sw_batch(S62, GO, GE, c0, seqs, idx)
    _compare_pairs(got, ref)
    # merged insertion vector of the whole batch (the center's own row is zero)
    ins_all = out["ins"].view(torch.int16).to(torch.int32) & 0xFFFF
    ins_all[0] = 0
    G = ins_all.max(dim=0).values
    W = m + int(G.sum().item())
    del ins_all
    print("ultra1m: MSA", flush=True)
    msa, c = H.halign_msa(ctx, sc, ds, 0)
    torch.cuda.synchronize()
    assert c == 0 and tuple(msa.shape) == (N, W)
    # every row restores its sequence: the non-gap bytes in row order are the
    # concatenated residues, and each row holds its sequence's length of them
    B = 100_000   # rows per check (boolean indexing stays below 2^31 elements)
    for r0 in range(0, N, B):
        r1 = min(N, r0 + B)
        blk = msa[r0:r1]
        nongap = blk != 255
        assert torch.equal(nongap.sum(dim=1).cpu(), torch.from_numpy(lens[r0:r1])), r0
        assert torch.equal(blk[nongap], ds.residues[int(seqs.offsets[r0]):int(seqs.offsets[r1])]), r0
        del nongap
    # sampled rows equal the oracle's rows under the same merge
    sub = seqs.subset(idx)
    rows = oracle_par.oracle.rows(sub.residues, sub.offsets, ref[2], ref[3], G.cpu().numpy().astype(np.int32), W)
    rows[idx == 0] = oracle_par.oracle.rows(seqs.subset([0]).residues, seqs.subset([0]).offsets,
                                            np.zeros((1, m + 1), np.uint16), np.ones((1, m), np.uint8),
                                            G.cpu().numpy().astype(np.int32), W)
    M = msa[ti].cpu().numpy()
    bad = np.nonzero((M != rows).any(axis=1))[0]
    assert len(bad) == 0, f"sampled MSA rows differ: {idx[bad[:10]]}"
    ctx.close()
