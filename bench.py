"""Benchmark: batched center-star MSA on one MI355X.

One step = the whole hot path on the batch20k workload (20,000 synthetic
family-structured proteins, lengths 200-500, 8 roots, 25% substitution, 5%
indel; BLOSUM62, W_k = 11 + k; center = sequence 0): affine SW of every
sequence against the center with traceback, the gap merge, and row emission,
with the sequences already resident in HBM.  The metric is GCUPS = m * sum(n)
DP cells per second of the whole step.

Also reported: the dominant kernel's roofline (integer VALU), the same kernels
launched once per pair (no batching), and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "batched SW GCUPS vs per-pair launch; MSA s at SP ≥99% of exact center"
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12      # 39.32 T int32 lane-ops/s
PEAK_INT16X2_TOPS = 2 * PEAK_INT32_TOPS            # 78.64 T: packed 16-bit ops do two per lane
OPS_PER_CELL_TB = 14                               # fixed op model, traceback pass


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(seqs, center: int, budget_s: float = 20.0):
    """The oracle, unchanged, on a bounded sample of the same workload: SW with
    traceback of sequences against the center.  Timed on one thread (the
    oracle's own single-core rate) and on one thread per host core (up to 16,
    each running the single-threaded routine on its own slice)."""
    import oracle
    from paper_1704_00878_amd import synth
    host_cores = os.cpu_count() or 1
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else host_cores
    threads = max(1, min(usable, 16))
    c = seqs.seq(center)
    m = len(c)
    lens = seqs.lengths()
    cum = np.cumsum(lens) * m

    def run(sub):
        oracle.sw_batch(synth.BLOSUM62, synth.GAP_OPEN, synth.GAP_EXTEND, c, sub.residues, sub.offsets)

    # one core: whole passes over a prefix of the set for about 3 s
    probe = seqs.subset(range(min(40, seqs.n)))
    t = time.perf_counter()
    run(probe)
    rate1 = m * probe.residues.size / max(time.perf_counter() - t, 1e-6)
    n1 = int(min(seqs.n, max(1, np.searchsorted(cum, rate1 * 3.0))))
    one = seqs.subset(range(n1))
    t = time.perf_counter()
    run(one)
    dt1 = time.perf_counter() - t
    gcups1 = m * int(one.residues.size) / dt1 / 1e9
    # all threads: about budget_s of CPU work, whole passes until 2 s of wall time
    want_cells = rate1 * threads * budget_s
    nsamp = int(min(seqs.n, max(threads, np.searchsorted(cum, want_cells))))
    sample = seqs.subset(range(nsamp))
    slices = np.array_split(np.arange(nsamp), threads)
    parts = [sample.subset(sl) for sl in slices if len(sl)]
    err = []

    def work(p):
        try:
            run(p)
        except Exception as e:  # pragma: no cover
            err.append(e)

    reps = 0
    t = time.perf_counter()
    while True:
        ths = [threading.Thread(target=work, args=(p,)) for p in parts]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        reps += 1
        dt = time.perf_counter() - t
        if err:
            raise err[0]
        if dt >= 2.0 or nsamp < seqs.n:
            break
    cells = m * int(sample.residues.size) * reps
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": len(parts), "kind": "oracle",
            "host_cores": host_cores, "usable_cores": usable, "value_one_core": round(gcups1, 4),
            "sample": f"SW+traceback against the center: one thread on the first {n1} sequences "
                      f"({m * int(one.residues.size):.3e} cells, {dt1:.1f} s); {len(parts)} threads on the "
                      f"first {nsamp} of {seqs.n} sequences, {reps} pass(es) ({cells:.3e} cells, {dt:.1f} s)"}


# kernel -> the sources its counter records are tied to
KERNEL_SOURCES = {"sw_stream_kernel": ["sw_kernels.hpp"],
                  "sw_stream16_kernel": ["stream16_kernels.hpp", "sw_kernels.hpp", "pk16.hpp"]}


def kernel_source_sha(kernel: str):
    """sha256 over the kernel's source files (concatenated), or None."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES.get(kernel, []):
            h.update(open(os.path.join(ROOT, "paper_1704_00878_amd", "csrc", f), "rb").read())
    except OSError:
        return None
    return h.hexdigest() if kernel in KERNEL_SOURCES else None


def counter_record(kernel: str, workload: str, plan: dict):
    """HBM counters of the forward kernel taken with rocprofv3 --pmc on this
    workload and plan (rows per lane, lanes per stream), from the profiles/
    summaries; None unless they were taken on the kernel source as it is now
    (sha256 of its source files)."""
    import glob
    import re
    sha = kernel_source_sha(kernel)
    if sha is None:
        return None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for m in re.finditer(r"<!-- record (\{.*?\}) -->", open(path).read()):
            try:
                rec = json.loads(m.group(1))
            except ValueError:
                continue
            if (rec.get("kernel") == kernel and rec.get("workload") == workload and rec.get("source_sha256") == sha
                    and rec.get("R") == plan.get("R") and rec.get("lanes") == plan.get("lanes")):
                return rec
    return None


def learned_report(H, ctx, sc, workload: str, anchors: int, partners: int, epochs: int, ema: float,
                   nseqs: int = 0, exact: bool = True, prejudge=(256, 16384)):
    """Learned center on a family set: the exhaustive center (all pairs,
    score-only) against the trained proposer's judged top-16, with the MSA of
    each and its avg SP.  Also the untrained network, 16 random candidates and
    sequence 0 as centers.  Without the exhaustive center (a set too large for
    all pairs), each center's objective comes from the exact judge over that
    one candidate and is compared with the learned center's."""
    import torch
    from paper_1704_00878_amd import synth
    log(f"bench: learned center on {workload}")
    seqs = synth.generate(workload, n_seqs=nseqs) if nseqs > 0 else synth.generate(workload)
    ds = H.DeviceSeqs(seqs, "cuda:0")
    N = seqs.n
    L = seqs.lengths().astype(np.float64)
    pair_cells = (L.sum() ** 2 - (L * L).sum()) / 2
    npairs = N * (N - 1) // 2

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    S = None
    c_exact = t_exact = None
    if exact:
        sums = torch.empty(N, dtype=torch.int64, device="cuda")
        c_exact, t_exact = timed(lambda: H.halign_center_exact(ctx, sc, ds, sums))
        S = sums.cpu().numpy()
        log(f"bench: exact center {c_exact} in {t_exact:.2f} s ({pair_cells / t_exact / 1e9:.0f} GCUPS score-only)")

    def objective(c):
        if S is not None:
            return int(S[c])
        cand = torch.tensor([c], dtype=torch.int32, device="cuda")
        one = torch.empty(1, dtype=torch.int64, device="cuda")
        H.halign_center_judge(ctx, sc, ds, cand, one)
        return int(one.item())

    prop = H.Proposer(seed=1)
    losses, t_train = timed(lambda: H.halign_train_proposer(ctx, sc, ds, prop, anchors=anchors, batch=1024,
                                                            epochs=epochs, lr=1e-3, seed=7, ema=ema,
                                                            partners=partners))
    log(f"bench: trained on {anchors * partners} pairs x {epochs} epochs in {t_train:.2f} s, loss {losses[0]:.4f} -> "
        f"{losses[-1]:.4f}")
    ctx.set_prejudge(0, 0)
    c_plain, _ = H.halign_center_learned(ctx, sc, ds, prop, 16)   # top-16 by u judged directly
    ctx.set_prejudge(*prejudge)
    (c_learned, cand), t_prop = timed(lambda: H.halign_center_learned(ctx, sc, ds, prop, 16))
    log(f"bench: learned center {c_learned}: propose + pre-judge + judge {t_prop * 1e3:.1f} ms")
    c_untrained, _ = H.halign_center_learned(ctx, sc, ds, H.Proposer(seed=1), 16)
    rand = np.random.default_rng(0).choice(N, 16, replace=False)
    if S is not None:
        c_random = int(max(rand, key=lambda i: (S[i], -i)))
    else:
        rs = torch.empty(16, dtype=torch.int64, device="cuda")
        c_random = H.halign_center_judge(ctx, sc, ds, torch.tensor(rand, dtype=torch.int32, device="cuda"), rs)

    def msa_of(c):
        H.halign_msa(ctx, sc, ds, c)   # warm: plans (and tunes) this center length once
        (msa, _), dt = timed(lambda: H.halign_msa(ctx, sc, ds, c))
        sp = H.halign_sp_score(sc, msa)[0] / npairs
        return dt, sp, int(msa.shape[1])

    res = {}
    ref_name = "exact" if exact else "learned"
    centers = ((("exact", c_exact),) if exact else ()) + (
        ("learned", c_learned), ("learned_top16_only", c_plain), ("untrained", c_untrained), ("random16", c_random),
        ("seq0", 0))
    ref = objective(c_exact if exact else c_learned)
    for name, c in centers:
        dt, sp, w = msa_of(c)
        obj = objective(c)
        res[name] = {"center": int(c), "objective": obj, "objective_ratio": round(obj / ref, 5),
                     "avg_sp": round(sp, 3), "msa_s": round(dt, 5), "width": w}
        log(f"bench: {name:9s} center {c}: objective / {ref_name} {obj / ref:.4f}, avg SP {sp:.2f}, "
            f"MSA {dt * 1e3:.1f} ms")
    out = {
        "workload": f"{workload}: {N} seqs, len {int(L.min())}-{int(L.max())}",
        "objective_ratio_of": ref_name,
        "exact_center_s": round(t_exact, 3) if exact else None, "exact_pairs": npairs,
        "exact_cells": float(pair_cells),
        "exact_gcups": round(pair_cells / t_exact / 1e9, 1) if exact else None,
        "train_s": round(t_train, 3), "train_pairs": anchors * partners, "anchors": anchors, "epochs": epochs,
        "prejudge": {"candidates": prejudge[0], "partners": prejudge[1]},
        "ema": ema,
        "loss_first_last": [round(losses[0], 5), round(losses[-1], 5)],
        "propose_judge_s": round(t_prop, 4), "candidates": [int(x) for x in cand],
        "learned_msa_s": round(t_prop + res["learned"]["msa_s"], 4),
        "centers": res,
    }
    if exact:
        out["sp_ratio_exact_over_learned"] = round(res["exact"]["avg_sp"] / res["learned"]["avg_sp"], 5)
        out["exact_msa_s"] = round(t_exact + res["exact"]["msa_s"], 3)
    return out


def nucleotide_report(H, ctx, workload: str, reps: int, cpu_seqs: int):
    """The trie section's nucleotide center star on a DNA set: MSA time with
    the sequences resident; with cpu_seqs > 0 its CPU baseline, the oracle's
    pairwise routine on one host thread over the first cpu_seqs sequences."""
    import torch
    from paper_1704_00878_amd import synth
    seqs = synth.generate_dna(workload)
    ds = H.DeviceSeqs(seqs)
    sc = H.Scoring(synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND)
    k = synth.NUC_K
    log(f"bench: nucleotide center star on {workload} ({seqs.n} seqs)")
    msa, score = H.halign_nuc_msa(ctx, sc, ds, k)   # warm-up
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        msa, score = H.halign_nuc_msa(ctx, sc, ds, k, out=msa)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    ms = 1e3 * float(np.median(ts))
    sp = H.halign_sp_score(sc, msa)[0] / (seqs.n * (seqs.n - 1) / 2)
    log(f"bench: nucleotide MSA {ms:.2f} ms (width {msa.shape[1]})")
    cpu = None
    if cpu_seqs > 0:
        import oracle
        nc = min(cpu_seqs, seqs.n)
        c = seqs.seq(0)
        t = time.perf_counter()
        for x in range(nc):
            oracle.nuc_align(synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND, k, c, seqs.seq(x))
        dt = time.perf_counter() - t
        bases = float(seqs.offsets[nc])
        cpu = {"value": round(bases / dt, 1), "unit": "bases/s", "cores": 1, "kind": "oracle",
               "sample": f"pairwise vectors of the first {nc} of {seqs.n} sequences against sequence 0 "
                         f"({dt:.2f} s; no merge or rows)"}
    return {"workload": f"{workload}: {seqs.n} seqs, {int(seqs.offsets[-1])} bases, center seq 0, k {k}",
            "msa_ms": round(ms, 3), "width": int(msa.shape[1]), "avg_sp": round(sp, 4),
            "bases_per_s": round(float(seqs.offsets[-1]) / (ms / 1e3), 1), "cpu_baseline": cpu}


def phylogeny_report(H, ctx, workload: str, reps: int, cpu: bool):
    """The NJ section's tree on the nucleotide MSA of a DNA set: halign_nj_tree
    timed with the MSA resident; with cpu, its CPU baseline, the oracle's tree
    of the same MSA on one host thread."""
    import torch
    from paper_1704_00878_amd import synth
    seqs = synth.generate_dna(workload)
    sc = H.Scoring(synth.NUC_MATRIX, synth.NUC_GAP_OPEN, synth.NUC_GAP_EXTEND)
    msa, _ = H.halign_nuc_msa(ctx, sc, H.DeviceSeqs(seqs), synth.NUC_K)
    perm = synth.tree_permutation(seqs.n)
    log(f"bench: tree of the {workload} MSA ({seqs.n} x {msa.shape[1]}): warm-up call")
    H.halign_nj_tree(ctx, msa, perm)   # warm-up
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        parent, blen = H.halign_nj_tree(ctx, msa, perm)
        ts.append(time.perf_counter() - t)
    ms = 1e3 * float(np.median(ts))
    log(f"bench: tree {ms:.2f} ms")
    out = {"workload": f"{workload}: NJ tree of the {seqs.n} x {int(msa.shape[1])} nucleotide MSA, sample "
                       f"{(seqs.n + 9) // 10} rows", "tree_ms": round(ms, 3), "nodes": int(len(parent)),
           "rows_per_s": round(seqs.n / (ms / 1e3), 1), "cpu_baseline": None}
    if cpu:
        import oracle
        host = msa.cpu().numpy()
        t = time.perf_counter()
        wp, wb = oracle.nj_tree(host, perm)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(seqs.n / dt, 2), "unit": "rows/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole tree of the same MSA on one host thread ({dt:.2f} s)",
                               "equal": bool((wp == parent).all() and (wb == blen).all())}
    return out


PD_OPS_PER_PAIR_WORD = 3   # xor-add, three-input and, popcount-add per four columns of a pair
INT_PEAK_TOPS = 39.32      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz, int32 lane-ops


def distance_report(H, ctx, workload: str, reps: int, cpu_rows: int):
    """The NJ section's p-distances over every pair of rows of a protein MSA
    (halign_msa of the workload, center 0): halign_pdist timed with the MSA
    resident, in pair-columns per second, and its integer-ALU roofline; with
    cpu_rows > 0, the oracle on the first cpu_rows rows (one host thread) and a
    bit-for-bit check of that block."""
    import torch
    from paper_1704_00878_amd import synth
    seqs = synth.generate(workload)
    msa, _ = H.halign_msa(ctx, H.Scoring(), H.DeviceSeqs(seqs), 0)
    n, w = int(msa.shape[0]), int(msa.shape[1])
    log(f"bench: distances of the {workload} MSA ({n} x {w}): warm-up call")
    D = H.halign_pdist(ctx, msa)
    ts = []
    for _ in range(reps):
        del D
        torch.cuda.synchronize()
        t = time.perf_counter()
        D = H.halign_pdist(ctx, msa)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    ms = 1e3 * float(np.median(ts))
    pc = float(n) * n * w
    rate = pc / (ms / 1e3)
    log(f"bench: distances {ms:.2f} ms, {rate / 1e12:.2f} T pair-columns/s")
    achieved = rate * PD_OPS_PER_PAIR_WORD / 4 / 1e12
    out = {"workload": f"{workload}: p-distances of all {n} x {n} row pairs of the {n} x {w} protein MSA",
           "ms": round(ms, 3), "pair_columns_per_s": round(rate, 1),
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": INT_PEAK_TOPS, "unit": "TOP/s",
                        "frac": round(achieved / INT_PEAK_TOPS, 4), "kernel": "pdist_kernel",
                        "ops_per_pair_column": PD_OPS_PER_PAIR_WORD / 4},
           "cpu_baseline": None}
    if cpu_rows > 0:
        import oracle
        s = min(cpu_rows, n)
        host = msa[:s].cpu().numpy()
        t = time.perf_counter()
        want = oracle.pdist(host)
        dt = time.perf_counter() - t
        got = D[:s, :s].cpu().numpy()
        out["cpu_baseline"] = {"value": round(float(s) * s * w / dt, 1), "unit": "pair-columns/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"all pairs of the first {s} rows on one host thread ({dt:.2f} s)",
                               "equal": bool((got == want).all())}
    del D
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch20k")
    ap.add_argument("--route", default="auto", choices=["auto", "intra", "inter"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the hipGraph-replay measurement")
    ap.add_argument("--perpair", type=int, default=200, help="pairs for the per-pair-launch baseline")
    ap.add_argument("--calibrate-copy", action="store_true", help="also run a 256 MiB device copy")
    ap.add_argument("--learned", default="learned50k", help="family set for the learned-center report "
                    "('none' skips it)")
    ap.add_argument("--learned-n", type=int, default=0, help="first N sequences of the family set (0: all)")
    ap.add_argument("--no-exact", action="store_true", help="learned report without the exhaustive center")
    ap.add_argument("--nucleotide", default="dna672", help="DNA set for the nucleotide center-star report "
                    "(none: skip)")
    ap.add_argument("--nucleotide-only", action="store_true",
                    help="run only the nucleotide report and print it as one JSON line (profiling)")
    ap.add_argument("--tree", default="dna672", help="DNA set whose MSA the phylogeny report builds a tree of "
                    "(none: skip)")
    ap.add_argument("--tree-only", action="store_true",
                    help="run only the phylogeny report and print it as one JSON line (profiling)")
    ap.add_argument("--pdist", default="batch20k", help="protein set whose MSA the distance report takes all "
                    "row pairs of ('none': skip)")
    ap.add_argument("--pdist-only", action="store_true",
                    help="run only the distance report and print it as one JSON line (profiling)")
    ap.add_argument("--anchors", type=int, default=50000, help="training anchors")
    ap.add_argument("--partners", type=int, default=64, help="training partners per anchor")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--prejudge", type=int, nargs=2, default=(256, 16384), metavar=("CANDIDATES", "PARTNERS"),
                    help="pre-judge of the learned center (0 0: off)")
    ap.add_argument("--ema", type=float, default=0.0, help="parameter average decay (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU path (pairs would shard over GPUs; that is a design, not code).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1704_00878_amd as H
    from paper_1704_00878_amd import _build, synth
    if not os.path.exists(_build.LIB_PATH):
        _build.build()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    if args.nucleotide_only:
        nuc = nucleotide_report(H, H.Context(0), args.nucleotide, args.steps, 0 if args.no_cpu else 200)
        print(json.dumps({"nucleotide": nuc}), flush=True)
        return
    if args.tree_only:
        tree = phylogeny_report(H, H.Context(0), args.tree, args.steps, not args.no_cpu)
        print(json.dumps({"phylogeny": tree}), flush=True)
        return
    if args.pdist_only:
        dist = distance_report(H, H.Context(0), args.pdist, args.steps, 0 if args.no_cpu else 256)
        print(json.dumps({"distances": dist}), flush=True)
        return
    log(f"bench: generating {args.workload}")
    seqs = synth.generate(args.workload)
    center = 0
    m = len(seqs.seq(center))
    cells = m * int(seqs.residues.size)
    ds = H.DeviceSeqs(seqs, "cuda:0")
    sc = H.Scoring()
    ctx = H.Context(0)
    route = {"auto": H.HALIGN_ROUTE_AUTO, "intra": H.HALIGN_ROUTE_INTRA, "inter": H.HALIGN_ROUTE_INTER}[args.route]

    outbuf = {}

    def step():
        # the MSA buffer is reused from step to step once W is known
        msa_, c_ = H.halign_msa(ctx, sc, ds, center, out=outbuf.get("t"))
        outbuf.setdefault("t", msa_)
        return msa_, c_

    if route != H.HALIGN_ROUTE_AUTO:
        os.environ["HALIGN_ROUTE"] = args.route
    else:
        ctx.set_autotune(not args.no_autotune)   # the first warm-up call tunes the plan
    log(f"bench: N={seqs.n} m={m} cells={cells:.3e}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fwd, walk = [], []
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        msa, _c = step()
        tm = ctx.last_timings()      # HIP events on the stream of the kernels
        fwd.append(tm[0])
        walk.append(tm[1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    gcups = cells / (ms_step * 1e-3) / 1e9
    st = ctx.last_stats()
    fwd_ms = float(np.mean(fwd))
    walk_ms = float(np.mean(walk))
    width = int(msa.shape[1])
    plan = ctx.last_plan()
    log(f"bench: {ms_step:.3f} ms/step, {gcups:.1f} GCUPS; forward {fwd_ms:.3f} ms, walk {walk_ms:.3f} ms; "
        f"plan {plan}")

    # the same steps with the SW batch replayed from a captured hipGraph
    graph = None
    if not args.no_graph:
        msa_eager = msa.clone()
        msa.zero_()                  # every replayed step must write the MSA again
        ctx.set_graph(True)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        g0 = ctx.graph_launches()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gmsa, _c = step()
        torch.cuda.synchronize()
        gms = (time.perf_counter() - t0) * 1e3 / args.steps
        ctx.set_graph(False)
        same = bool(torch.equal(gmsa, msa_eager))
        graph = {"ms_per_step": round(gms, 4), "gcups": round(cells / (gms * 1e-3) / 1e9, 1),
                 "replays": ctx.graph_launches() - g0, "msa_equal_eager": same}
        log(f"bench: graph replay {gms:.3f} ms/step, msa equal to eager: {same}")
        del gmsa, msa_eager

    if args.calibrate_copy:
        # plain device copy of a known size: reference reading for HBM counters
        nb = 256 << 20
        xs = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ys = torch.empty_like(xs)
        xs.fill_(1)
        for _ in range(3):
            ys.copy_(xs)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {nb} bytes x3 done")

    # per-pair launches: same kernels, one pair per call, no batching (default
    # plan: tuning a one-pair batch would only add the tuner's own runs)
    ctx.set_autotune(False)
    rng = np.random.default_rng(0)
    pick = rng.choice(seqs.n, size=min(max(args.perpair, 1), seqs.n), replace=False)
    singles = [H.DeviceSeqs(seqs.subset([int(k)]), "cuda:0") for k in pick]
    cseq = ds.residues[int(ds.offsets_host[center]):int(ds.offsets_host[center + 1])]
    for d in singles[:5]:
        H.sw_batch(ctx, sc, d, 0, traceback=True, center_seq=cseq)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for d in singles:
        H.sw_batch(ctx, sc, d, 0, traceback=True, center_seq=cseq)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - tp
    pp_cells = m * int(seqs.lengths()[pick].sum())
    pp_gcups = pp_cells / dtp / 1e9
    log(f"bench: per-pair launches {pp_gcups:.2f} GCUPS over {len(pick)} pairs")

    # dominant kernel roofline: integer VALU, fixed op model
    achieved = cells * OPS_PER_CELL_TB / (fwd_ms * 1e-3) / 1e12
    kname = ("sw_stream16_kernel" if plan.get("packed") else "sw_stream_kernel") if st["route"] == 0 \
        else "sw_inter_kernel"
    packed = kname == "sw_stream16_kernel"
    peak = PEAK_INT16X2_TOPS if packed else PEAK_INT32_TOPS
    rec = counter_record(kname, args.workload, plan)
    traffic = clock = None
    if rec is not None:
        traffic = int(rec["fetch_kib"] * 1024 * rec["fetch_factor"] + rec["write_kib"] * 1024 * rec["write_factor"])
        clock = rec["clock_ghz"]
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2),
            "unit": "TOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel": kname, "ops_per_cell": OPS_PER_CELL_TB, "kernel_ms": round(fwd_ms, 4),
            "kernel_gcups": round(cells / (fwd_ms * 1e-3) / 1e9, 1),
            "measured_clock_ghz": clock,
            "frac_at_measured_clock": round(achieved / (peak * clock / 2.4), 4) if clock else None,
            "algorithmic_bytes": int(cells // 2 + seqs.residues.size)}

    # avg SP of the produced MSA (evaluation, untimed)
    sp, spb = H.halign_sp_score(sc, msa)
    npairs = seqs.n * (seqs.n - 1) // 2

    cpu = None
    if not args.no_cpu:
        log("bench: oracle on host cores")
        cpu = cpu_baseline(seqs, center)
        log(f"bench: oracle {cpu['value']:.3f} GCUPS on {cpu['cores']} threads")

    nuc = None
    if args.nucleotide != "none":
        nuc = nucleotide_report(H, ctx, args.nucleotide, 5, 0 if args.no_cpu else 200)
    tree = None
    if args.tree != "none":
        tree = phylogeny_report(H, ctx, args.tree, 3, not args.no_cpu)
    dist = None
    if args.pdist != "none":
        dist = distance_report(H, ctx, args.pdist, 3, 0 if args.no_cpu else 256)

    ctx.set_autotune(not args.no_autotune)
    learned = None
    if args.learned != "none":
        learned = learned_report(H, ctx, sc, args.learned, args.anchors, args.partners, args.epochs, args.ema,
                                 args.learned_n, not args.no_exact, tuple(args.prejudge))

    out = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int16x2" if packed else "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {seqs.n} seqs, len {int(seqs.lengths().min())}-"
                               f"{int(seqs.lengths().max())}, center seq 0 (m={m}), BLOSUM62, gap 11+k",
                   "cells_per_step": cells, "msa_width": width, "route": ["intra", "inter"][st["route"]],
                   "plan": plan},
        "roofline": roof,
        "cpu_baseline": cpu,
        "per_pair_launch": {"value": round(pp_gcups, 3), "unit": "GCUPS", "pairs": len(pick),
                            "batched_over_per_pair": round(gcups / pp_gcups, 1)},
        "stages_ms": {"forward": round(fwd_ms, 4), "walk": round(walk_ms, 4),
                      "merge_rows_other": round(ms_step - fwd_ms - walk_ms, 4)},
        "avg_sp": round(sp / npairs, 3), "msa_s": round(ms_step / 1e3, 6),
        "graph_replay": graph,
        "learned_center": learned,
        "nucleotide": nuc,
        "phylogeny": tree,
        "distances": dist,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
