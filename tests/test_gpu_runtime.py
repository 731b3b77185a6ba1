"""GPU tests of the runtime features around the kernels: hipGraph capture and
replay, the autotuner and its cache file, and ASCII encoding."""
import numpy as np
import pytest

import oracle
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_1704_00878_amd as H
    H.lib()
    return H


def _ref(seqs, center_idx):
    return oracle.sw_batch(synth.BLOSUM62, 11, 1, seqs.seq(center_idx), seqs.residues, seqs.offsets)


def _host(H, out, m):
    return (out["score"].cpu().numpy(), out["cells"].cpu().numpy(), out["ins"].cpu().numpy().view(np.uint16),
            H.aligned_to_bool(out["aligned"].cpu().numpy(), m))


@pytest.mark.parametrize("lanes", [None, "16", "pack16"])
def test_graph_replays_match_eager(H, lanes, monkeypatch):
    """Several replays, with eager work and synchronisations in between, each
    equal to the oracle; a changed argument is captured anew.  Also with
    16-lane streams and with the packed 16-bit kernel on them."""
    import torch
    if lanes:
        monkeypatch.setenv("HALIGN_STREAM_LANES", lanes.replace("pack", ""))
    if lanes and lanes.startswith("pack"):
        monkeypatch.setenv("HALIGN_STREAM_PACK", "1")
    ctx = H.Context(0)
    sc = H.Scoring()
    seqs = synth.generate("plain64", n_seqs=300, seed=31)
    ds = H.DeviceSeqs(seqs)
    ref = _ref(seqs, 0)
    out = H.sw_batch(ctx, sc, ds, 0, graph=True)
    torch.cuda.synchronize()
    for rep in range(4):
        for k in out:
            if hasattr(out[k], "fill_"):
                out[k].fill_(-7)                    # eager work between replays
        torch.cuda.synchronize()
        H.sw_batch(ctx, sc, ds, 0, graph=True, out=out)
        torch.cuda.synchronize()
        got = _host(H, out, out["m"])
        for g, r in zip(got, ref):
            assert (g == r).all(), rep
        # an eager (non-graph) call in between uses the ctx's own scratch
        other = H.sw_batch(ctx, sc, ds, 5)
        torch.cuda.synchronize()
        assert (other["score"].cpu().numpy() == _ref(seqs, 5)[0]).all()
    assert ctx.graph_launches() == 4
    # new center -> new capture, still exact
    out2 = H.sw_batch(ctx, sc, ds, 9, graph=True)
    H.sw_batch(ctx, sc, ds, 9, graph=True, out=out2)
    torch.cuda.synchronize()
    for g, r in zip(_host(H, out2, out2["m"]), _ref(seqs, 9)):
        assert (g == r).all()
    ctx.close()


@pytest.mark.parametrize("route", ["intra", "pack16", "inter"])
def test_graph_replays_in_chunks(H, route, monkeypatch):
    """A workspace cap that splits the batch into chunks, captured into one
    graph: every chunk keeps its own plan region, so every replay (with eager
    work and synchronisations in between) equals the oracle."""
    import torch
    if route == "pack16":
        monkeypatch.setenv("HALIGN_STREAM_LANES", "16")
        monkeypatch.setenv("HALIGN_STREAM_PACK", "1")
    ctx = H.Context(0, workspace_cap=1_000_000)
    sc = H.Scoring()
    seqs = synth.generate("plain64", n_seqs=300, seed=32)
    ds = H.DeviceSeqs(seqs)
    ref = _ref(seqs, 0)
    rt = H.HALIGN_ROUTE_INTER if route == "inter" else H.HALIGN_ROUTE_INTRA
    out = H.sw_batch(ctx, sc, ds, 0, graph=True, route=rt)
    torch.cuda.synchronize()
    assert ctx.last_stats()["chunks"] >= 2
    for g, r in zip(_host(H, out, out["m"]), ref):
        assert (g == r).all()
    for rep in range(3):
        for k in out:
            if hasattr(out[k], "fill_"):
                out[k].fill_(-7)
        torch.cuda.synchronize()
        H.sw_batch(ctx, sc, ds, 0, graph=True, route=rt, out=out)
        torch.cuda.synchronize()
        for g, r in zip(_host(H, out, out["m"]), ref):
            assert (g == r).all(), rep
        other = H.sw_batch(ctx, sc, ds, 7, route=rt)   # eager call in between
        torch.cuda.synchronize()
        assert (other["score"].cpu().numpy() == _ref(seqs, 7)[0]).all()
    assert ctx.graph_launches() == 3
    # the end-to-end MSA with graph replay on the same capped ctx
    ctx.set_graph(True)
    mref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, 0)
    for _ in range(3):
        msa, _c = H.halign_msa(ctx, sc, ds, 0)
        torch.cuda.synchronize()
        assert (msa.cpu().numpy() == mref["msa"]).all()
    ctx.close()


def test_msa_with_graph(H):
    import torch
    ctx = H.Context(0)
    ctx.set_graph(True)
    sc = H.Scoring()
    seqs = synth.generate("plain64")
    ds = H.DeviceSeqs(seqs)
    ref = oracle.msa(synth.BLOSUM62, 11, 1, seqs.residues, seqs.offsets, 0)
    for _ in range(3):
        msa, _c = H.halign_msa(ctx, sc, ds, 0)
        torch.cuda.synchronize()
        assert (msa.cpu().numpy() == ref["msa"]).all()
    ctx.close()


def test_autotune_is_exact(H, tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "tune.txt"
    cache.write_text("garbage line\nm1_n1 9 9 9\n\n")      # corrupt entries are ignored
    monkeypatch.setenv("HALIGN_TUNE_CACHE", str(cache))
    ctx = H.Context(0)
    ctx.set_autotune(True)
    sc = H.Scoring()
    seqs = synth.generate("batch20k", n_seqs=3000, seed=5)
    ds = H.DeviceSeqs(seqs)
    out = H.sw_batch(ctx, sc, ds, 0)
    torch.cuda.synchronize()
    plan = ctx.last_plan()
    assert plan["route"] in (0, 1)
    ref = _ref(seqs, 0)
    for g, r in zip(_host(H, out, out["m"]), ref):
        assert (g == r).all()
    assert len(cache.read_text().strip().splitlines()) == 4   # one tuned bucket appended
    # a second context reads the cache and picks the same plan without timing
    ctx2 = H.Context(0)
    ctx2.set_autotune(True)
    out2 = H.sw_batch(ctx2, sc, ds, 0)
    torch.cuda.synchronize()
    assert ctx2.last_plan() == plan
    assert (out2["score"].cpu().numpy() == ref[0]).all()
    ctx.close()
    ctx2.close()


def test_encode(H):
    """Every byte value, and a long text spanning several workgroups, against
    the oracle's encoding."""
    import torch
    rng = np.random.default_rng(4)
    for raw in (bytes(range(256)) + b"ARNDCQEGHILKMFPSTWYVBZX*arndUOJ-",
                bytes(rng.integers(0, 256, 1_000_003, dtype=np.uint8))):
        a = torch.tensor(list(raw), dtype=torch.uint8, device="cuda")
        c = torch.empty_like(a)
        H.halign_encode(a, c)
        torch.cuda.synchronize()
        assert (c.cpu().numpy() == oracle.encode(raw)).all()
