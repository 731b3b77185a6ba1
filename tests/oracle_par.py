"""The oracle's pairwise routine run over slices of a sequence set in host
threads (the routine itself is unchanged and single-threaded; the ctypes call
releases the GIL), for parity checks of whole workloads."""
from __future__ import annotations

import os
import threading

import numpy as np

import oracle


def host_threads() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def sw_batch(S, go: int, ge: int, center, seqs, idx=None, threads: int | None = None):
    """oracle.sw_batch of the sequences idx (default: all) of `seqs` against
    center, split over threads; returns (score, cells, ins, aligned) in idx order."""
    idx = np.arange(seqs.n) if idx is None else np.asarray(idx)
    T = threads or host_threads()
    parts = [p for p in np.array_split(idx, T) if len(p)]
    out = [None] * len(parts)
    err = []

    def work(q):
        try:
            sub = seqs.subset(parts[q])
            out[q] = oracle.sw_batch(S, go, ge, center, sub.residues, sub.offsets)
        except Exception as e:  # pragma: no cover
            err.append(e)

    ths = [threading.Thread(target=work, args=(q,)) for q in range(len(parts))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    if err:
        raise err[0]
    m = len(center)
    if not parts:
        return (np.zeros(0, np.int32), np.zeros((0, 4), np.int32), np.zeros((0, m + 1), np.uint16),
                np.zeros((0, m), np.uint8))
    return tuple(np.concatenate([o[k] for o in out]) for k in range(4))


def msa(S, go: int, ge: int, seqs, center: int, threads: int | None = None):
    """The oracle's center-star MSA (as oracle.msa: pairwise vectors with the
    center's own row set to the identity, merge, rows), pairwise step threaded."""
    c = seqs.seq(center)
    score, cells, ins, al = sw_batch(S, go, ge, c, seqs, threads=threads)
    ins[center] = 0
    al[center] = 1
    G, col, W = oracle.merge(ins)
    rows = oracle.rows(seqs.residues, seqs.offsets, ins, al, G, W)
    return dict(score=score, cells=cells, ins=ins, aligned=al, G=G, col=col, width=W, msa=rows)


def sp_from_profile(P, S, ge: int):
    """(avg SP numerator, BLOSUM SP) from a column profile [W][alpha + 1]:
    residue pairs score +1 when different (or S), residue-gap pairs +2 (or
    -ge), gap-gap pairs 0."""
    alpha = P.shape[1] - 1
    res, gap = P[:, :alpha].astype(np.int64), P[:, alpha].astype(np.int64)
    r = res.sum(1)
    sp = int(((r * (r - 1) // 2) - (res * (res - 1) // 2).sum(1) + 2 * gap * r).sum())
    S64 = np.asarray(S, np.int64)[:alpha, :alpha]
    cross = np.einsum("xa,ab,xb->", res, S64, res)          # ordered pairs, self pairs included
    diag = (res * np.diag(S64)[None]).sum()                  # self pairs
    bl = int((cross - diag) // 2 - ge * (gap * r).sum())
    return sp, bl
