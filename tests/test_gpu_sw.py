"""GPU parity: SW scores, end/start cells and center-star vectors, bit-exact
against the oracle, through the C ABI.  Both kernels (one pair per lane, one
pair per wavefront stream of 64, 32 or 16 lanes) are checked on every case."""
import os

import numpy as np
import pytest

import oracle
from golden_cases import load
from paper_1704_00878_amd import synth

pytestmark = pytest.mark.gpu

# intra32/intra16: 32- and 16-lane streams; pack32/pack16: the packed 16-bit
# wavefront kernel (two streams per lane group) on 32- and 16-lane streams
ROUTES = ["intra", "intra32", "intra16", "pack32", "pack16", "inter"]


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


def _route(H, name):
    return H.HALIGN_ROUTE_INTER if name == "inter" else H.HALIGN_ROUTE_INTRA


def _run(H, ctx, sc, seqs, center_codes, route, traceback=True):
    import torch
    ds = H.DeviceSeqs(seqs)
    cen = torch.from_numpy(np.ascontiguousarray(center_codes, dtype=np.uint8)).cuda()
    lanes = {"intra32": "32", "intra16": "16", "pack32": "32", "pack16": "16"}.get(route)
    if lanes:
        os.environ["HALIGN_STREAM_LANES"] = lanes
    if route.startswith("pack"):
        os.environ["HALIGN_STREAM_PACK"] = "1"
    try:
        out = H.sw_batch(ctx, sc, ds, 0, traceback=traceback, route=_route(H, route), center_seq=cen)
        torch.cuda.synchronize()
    finally:
        os.environ.pop("HALIGN_STREAM_LANES", None)
        os.environ.pop("HALIGN_STREAM_PACK", None)
    m = len(center_codes)
    res = dict(score=out["score"].cpu().numpy(), cells=out["cells"].cpu().numpy())
    if traceback:
        res["ins"] = out["ins"].cpu().numpy().view(np.uint16)
        res["aligned"] = H.aligned_to_bool(out["aligned"].cpu().numpy(), m)
    return res


def _compare(got, S, go, ge, center, seqs, traceback=True):
    score, cells, ins, al = oracle.sw_batch(S, go, ge, center, seqs.residues, seqs.offsets)
    bad = np.nonzero(got["score"] != score)[0]
    assert len(bad) == 0, f"score mismatch at {bad[:10]}: {got['score'][bad[:10]]} vs {score[bad[:10]]}"
    if traceback:
        bad = np.nonzero((got["cells"] != cells).any(axis=1))[0]
        assert len(bad) == 0, f"cells mismatch at {bad[:5]}: {got['cells'][bad[:5]]} vs {cells[bad[:5]]}"
        bad = np.nonzero((got["ins"] != ins).any(axis=1))[0]
        assert len(bad) == 0, f"ins mismatch at {bad[:5]}"
        bad = np.nonzero((got["aligned"] != al).any(axis=1))[0]
        assert len(bad) == 0, f"aligned mismatch at {bad[:5]}"
    else:
        # score-only reports the end cell as (0, 0, i1, j1)
        assert (got["cells"][:, 2:] == cells[:, 2:]).all()


@pytest.mark.parametrize("route", ROUTES)
def test_plain64_center0(H, ctx, route):
    seqs = synth.generate("plain64")
    sc = H.Scoring()
    got = _run(H, ctx, sc, seqs, seqs.seq(0), route)
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, seqs.seq(0), seqs)


@pytest.mark.parametrize("route", ROUTES)
def test_hand_cases(H, ctx, route):
    for case in [c for c in load() if c["kind"] == "case"]:
        sc = H.Scoring(gap_open=case["go"], gap_extend=case["ge"])
        seqs = synth.SeqSet.from_list([case["seq"]])
        got = _run(H, ctx, sc, seqs, case["center"], route)
        assert got["score"][0] == case["score"], case["name"]
        assert tuple(got["cells"][0]) == case["cells"], case["name"]
        assert (got["ins"][0] == case["ins"]).all(), case["name"]
        assert (got["aligned"][0] == case["aligned"]).all(), case["name"]


# centers spanning every rows-per-lane template, multi-pass layouts and the
# fallback to the strip kernel when the profile exceeds LDS (101 and 112 give
# 7 rows per lane on 16-lane packed streams, the plan of the long-tail
# workload)
@pytest.mark.parametrize("m", [1, 7, 64, 101, 112, 128, 129, 200, 256, 300, 384, 385, 512, 513, 700, 1100])
@pytest.mark.parametrize("route", ROUTES)
def test_center_lengths(H, ctx, m, route):
    rng = np.random.default_rng(1000 + m)
    base = synth.generate("plain64", n_seqs=24, seed=77 + m)
    center = rng.integers(0, 20, size=m).astype(np.uint8)
    # sequences related to the center plus unrelated ones and edge lengths
    seqs = [center[rng.integers(0, max(1, m // 3)):][: rng.integers(1, m + 1)].copy() for _ in range(8)]
    seqs += [base.seq(k) for k in range(8)]
    seqs += [np.zeros(0, np.uint8), center[:1].copy(), center.copy(),
             rng.integers(0, 24, size=int(rng.integers(1, 400))).astype(np.uint8)]
    for k in range(4):
        s = center.copy()
        for _ in range(max(1, m // 40)):
            p = int(rng.integers(0, len(s) + 1))
            s = np.insert(s, p, rng.integers(0, 20, size=int(rng.integers(1, 4))).astype(np.uint8))
        seqs.append(s)
    ss = synth.SeqSet.from_list(seqs)
    sc = H.Scoring()
    got = _run(H, ctx, sc, ss, center, route)
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, ss)


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("gaps", [(11, 1), (10, 1), (0, 1), (3, 2), (1, 1)])
def test_gap_params(H, ctx, route, gaps):
    seqs = synth.generate("plain64", n_seqs=40, seed=5)
    sc = H.Scoring(gap_open=gaps[0], gap_extend=gaps[1])
    got = _run(H, ctx, sc, seqs, seqs.seq(3), route)
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, seqs.seq(3), seqs)


@pytest.mark.parametrize("route", ROUTES)
def test_score_only(H, ctx, route):
    seqs = synth.generate("plain64")
    sc = H.Scoring()
    got = _run(H, ctx, sc, seqs, seqs.seq(5), route, traceback=False)
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, seqs.seq(5), seqs, traceback=False)


def test_small_alphabet_ties(H, ctx):
    """Tiny alphabet makes ties everywhere: every tie rule is exercised."""
    rng = np.random.default_rng(3)
    S = np.array([[2, -1], [-1, 2]], np.int8)
    for route in ROUTES:
        for go, ge in [(1, 1), (0, 1), (2, 1)]:
            center = rng.integers(0, 2, size=90).astype(np.uint8)
            seqs = synth.SeqSet.from_list([rng.integers(0, 2, size=int(rng.integers(0, 120))).astype(np.uint8)
                                           for _ in range(70)])
            sc = H.Scoring(S, go, ge)
            got = _run(H, ctx, sc, seqs, center, route)
            _compare(got, S, go, ge, center, seqs)


@pytest.mark.parametrize("route,m", [("pack32", 330), ("pack32", 420), ("pack16", 170), ("pack16", 420),
                                     ("intra32", 330), ("intra16", 420)])
@pytest.mark.parametrize("streams", [0, 3])
def test_small_alphabet_ties_long_centers(H, ctx, route, m, streams, monkeypatch):
    """Ties on centers that give 10 to 14 rows per lane (both end-cell
    trackings of the packed kernel, one and two passes), with one pair per
    stream and with many pairs per stream."""
    if streams:
        monkeypatch.setenv("HALIGN_MAX_STREAMS", str(streams))
    rng = np.random.default_rng(m + streams)
    S = np.array([[2, -1], [-1, 2]], np.int8)
    center = rng.integers(0, 2, size=m).astype(np.uint8)
    seqs = [rng.integers(0, 2, size=int(rng.integers(0, 300))).astype(np.uint8) for _ in range(60)]
    seqs += [center.copy(), center[m // 3:].copy(), np.zeros(0, np.uint8)]
    ss = synth.SeqSet.from_list(seqs)
    for go, ge in [(1, 1), (0, 1)]:
        sc = H.Scoring(S, go, ge)
        got = _run(H, ctx, sc, ss, center, route)
        if route.startswith("pack"):
            assert ctx.last_plan()["packed"] == 1
        _compare(got, S, go, ge, center, ss)


@pytest.mark.parametrize("route", ["pack32", "pack16"])
def test_packed_step_count_past_16_bits(H, ctx, route, monkeypatch):
    """One stream of about 80,000 columns: the packed kernel keeps the step of
    each end cell modulo 2^16, which must still give every column."""
    monkeypatch.setenv("HALIGN_MAX_STREAMS", "1")
    rng = np.random.default_rng(11)
    center = rng.integers(0, 20, size=150).astype(np.uint8)
    seqs = []
    for k in range(300):
        s = rng.integers(0, 20, size=int(rng.integers(200, 330))).astype(np.uint8)
        p = int(rng.integers(0, len(s) - 60))
        s[p:p + 60] = center[40:100]   # an end cell far into the pair
        seqs.append(s)
    ss = synth.SeqSet.from_list(seqs)
    assert int(ss.offsets[-1]) > 70000
    sc = H.Scoring()
    got = _run(H, ctx, sc, ss, center, route)
    assert ctx.last_plan()["packed"] == 1
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, ss)


@pytest.mark.parametrize("route", ["pack32", "pack16"])
@pytest.mark.parametrize("m", [1050, 1363, 1364])
def test_packed_scores_at_the_bound(H, ctx, route, m):
    """Scores up to the packed kernel's bound (max S x min(m, longest) <
    15000): a center of m tryptophans (S = 11) against itself and its parts
    reaches H = 11 m, 14,993 at m = 1363; at m = 1364 the bound fails and the
    32-bit kernel runs."""
    w = 17   # W in the NCBI order
    center = np.full(m, w, np.uint8)
    rng = np.random.default_rng(m)
    mixed = center.copy()
    mixed[rng.integers(0, m, m // 10)] = rng.integers(0, 20, m // 10).astype(np.uint8)
    ss = synth.SeqSet.from_list([center.copy(), center[m // 4:].copy(), mixed, np.zeros(0, np.uint8),
                                 rng.integers(0, 20, 200).astype(np.uint8)])
    sc = H.Scoring()
    got = _run(H, ctx, sc, ss, center, route)
    assert ctx.last_plan()["packed"] == (1 if 11 * m < 15000 else 0)
    assert got["score"][0] == 11 * m
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, ss)


@pytest.mark.parametrize("lanes", ["intra", "intra32", "intra16", "pack32", "pack16"])
@pytest.mark.parametrize("streams", [1, 2, 5])
def test_stream_packing(H, ctx, streams, lanes, monkeypatch):
    """Many pairs per wavefront: pair boundaries inside a stream reset the
    state exactly; empty and 1-residue sequences sit between long ones."""
    monkeypatch.setenv("HALIGN_MAX_STREAMS", str(streams))
    rng = np.random.default_rng(streams)
    base = synth.generate("plain64")
    seqs = [base.seq(k) for k in range(64)]
    for x in (3, 10, 11, 40):
        seqs[x] = np.zeros(0, np.uint8)
    for x in (5, 6, 7, 50):
        seqs[x] = rng.integers(0, 20, size=1).astype(np.uint8)
    ss = synth.SeqSet.from_list(seqs)
    sc = H.Scoring()
    for center in (base.seq(0), rng.integers(0, 20, size=700).astype(np.uint8)):
        got = _run(H, ctx, sc, ss, center, lanes)
        _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, ss)


@pytest.mark.parametrize("m", [90, 450, 1100])
def test_profile_int32_path(H, ctx, m, monkeypatch):
    """The int32-profile variant (used when scores may not fit 16 bits) agrees too."""
    monkeypatch.setenv("HALIGN_PROFILE32", "1")
    rng = np.random.default_rng(m)
    base = synth.generate("plain64", n_seqs=30, seed=m)
    center = rng.integers(0, 20, size=m).astype(np.uint8)
    seqs = synth.SeqSet.from_list([base.seq(k) for k in range(30)] + [center[5:m // 2].copy()])
    sc = H.Scoring()
    got = _run(H, ctx, sc, seqs, center, "intra")
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, seqs)


@pytest.mark.parametrize("traceback", [True, False])
def test_long_pairs_leave_the_strip_route(H, ctx, traceback, monkeypatch):
    """A batch on the one-pair-per-lane route (chosen here through the route
    knob; by default it is the route of batches of 262,144 pairs and more):
    its pairs longer than 1,000 residues run on the wavefront kernel in a
    launch of their own, the rest on the strip kernel, and every pair equals
    the oracle."""
    import torch
    monkeypatch.setenv("HALIGN_ROUTE", "inter")
    rng = np.random.default_rng(77)
    center = rng.integers(0, 20, size=300).astype(np.uint8)
    base = synth.generate("plain64", n_seqs=120, seed=78)
    seqs = [base.seq(k) for k in range(base.n)]
    for L in (1000, 1001, 1200, 2000):               # long pairs holding the center
        s = rng.integers(0, 20, size=L).astype(np.uint8)
        p = int(rng.integers(0, L - 300))
        s[p:p + 300] = center
        seqs.insert(int(rng.integers(0, len(seqs))), s)
    seqs.insert(7, rng.integers(0, 20, size=1500).astype(np.uint8))   # long and unrelated
    seqs.insert(9, np.zeros(0, np.uint8))
    ss = synth.SeqSet.from_list(seqs)
    ds = H.DeviceSeqs(ss)
    sc = H.Scoring()
    cen = torch.from_numpy(center).cuda()
    out = H.sw_batch(ctx, sc, ds, 0, traceback=traceback, center_seq=cen)
    torch.cuda.synchronize()
    st = ctx.last_stats()
    assert st["route"] == 1 and st["launches"] >= 2
    got = dict(score=out["score"].cpu().numpy(), cells=out["cells"].cpu().numpy())
    if traceback:
        got["ins"] = out["ins"].cpu().numpy().view(np.uint16)
        got["aligned"] = H.aligned_to_bool(out["aligned"].cpu().numpy(), len(center))
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, ss, traceback=traceback)
    assert (got["score"][[k for k in range(ss.n) if ss.lengths()[k] in (1001, 1200, 2000)]] >= 300 * 4).all()


def test_deterministic_repeat(H, ctx):
    seqs = synth.generate("plain64")
    sc = H.Scoring()
    a = _run(H, ctx, sc, seqs, seqs.seq(0), "intra")
    b = _run(H, ctx, sc, seqs, seqs.seq(0), "intra")
    for k in a:
        assert (a[k] == b[k]).all()


def test_workspace_cap_chunks(H):
    """A tiny workspace cap forces many chunks; results are identical."""
    seqs = synth.generate("plain64", n_seqs=300, seed=21)
    sc = H.Scoring()
    full = H.Context(0)
    small = H.Context(0, workspace_cap=1_000_000)
    for route in ROUTES:
        a = _run(H, full, sc, seqs, seqs.seq(0), route)
        b = _run(H, small, sc, seqs, seqs.seq(0), route)
        assert small.last_stats()["chunks"] > 1
        for k in a:
            assert (a[k] == b[k]).all()
    full.close()
    small.close()


def test_injected_chunk_failure_then_retry(H):
    """A chunk that fails is reported; re-running the call gives the same result."""
    seqs = synth.generate("plain64")
    sc = H.Scoring()
    ctx = H.Context(0, workspace_cap=200_000)
    ref = _run(H, ctx, sc, seqs, seqs.seq(0), "intra")
    ctx.fail_chunk(1)
    with pytest.raises(H.HalignError):
        _run(H, ctx, sc, seqs, seqs.seq(0), "intra")
    again = _run(H, ctx, sc, seqs, seqs.seq(0), "intra")
    for k in ref:
        assert (ref[k] == again[k]).all()
    ctx.close()


def test_invalid_arguments(H, ctx):
    import torch
    seqs = synth.generate("plain64", n_seqs=4)
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring()
    score = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(H.HalignError):
        H.halign_sw_batch(ctx, sc, ds.seq_ptr(0), 0, ds, 0, score)
    bad = H.Scoring(gap_open=-1)
    with pytest.raises(H.HalignError):
        H.halign_sw_batch(ctx, bad, ds.seq_ptr(0), ds.length(0), ds, 0, score)
    # residue codes at or above the alphabet size are rejected (after a safe run)
    res = seqs.residues.copy()
    res[5] = 30
    ds2 = H.DeviceSeqs(synth.SeqSet(res, seqs.offsets))
    with pytest.raises(H.HalignError) as ei:
        H.halign_sw_batch(ctx, sc, ds2.seq_ptr(0), ds2.length(0), ds2, H.HALIGN_TRACEBACK, score,
                          torch.empty((4, 4), dtype=torch.int32, device="cuda"),
                          torch.empty((4, ds2.length(0) + 1), dtype=torch.int16, device="cuda"),
                          torch.empty((4, (ds2.length(0) + 31) // 32), dtype=torch.int32, device="cuda"))
    assert ei.value.code == -1
    with pytest.raises(H.HalignError):
        H.halign_msa(ctx, sc, ds2, 1)
    # the context stays usable
    out = H.sw_batch(ctx, sc, ds, 0)
    torch.cuda.synchronize()


def test_packed_kernel_selected(H, ctx, monkeypatch):
    """The packed routes run the packed 16-bit kernel, not a silent fallback;
    above its bound (max S x length >= 15000) the 32-bit kernel takes over."""
    import torch
    monkeypatch.setenv("HALIGN_STREAM_LANES", "32")
    monkeypatch.setenv("HALIGN_STREAM_PACK", "1")
    sc = H.Scoring()
    seqs = synth.generate("plain64")
    for c in (0, int(np.argmax(seqs.lengths()))):
        got = _run(H, ctx, sc, seqs, seqs.seq(c), "pack32")
        assert ctx.last_plan()["packed"] == 1
        _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, seqs.seq(c), seqs)
    rng = np.random.default_rng(8)
    center = rng.integers(0, 20, 1500).astype(np.uint8)
    mut = center.copy()
    mut[rng.integers(0, 1500, 150)] = rng.integers(0, 20, 150).astype(np.uint8)
    ss = synth.SeqSet.from_list([mut, center[200:1400].copy(), rng.integers(0, 20, 300).astype(np.uint8)])
    got = _run(H, ctx, sc, ss, center, "pack32")
    assert ctx.last_plan()["packed"] == 0
    _compare(got, sc.matrix, sc.gap_open, sc.gap_extend, center, ss)
