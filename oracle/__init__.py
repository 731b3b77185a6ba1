"""CPU oracle for the center-star protein MSA path (test infrastructure only).

The C source next to this file is the slow, plain definition that the HIP
library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  Nothing here imports the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "halign_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
GAP = 255

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single-threaded, no SIMD intrinsics, no
    fused multiply-add: every double operation rounds on its own)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L.orc_sw.argtypes = [P, I, I, I, P, I, P, I, P, P, P, P, P]
        L.orc_sw.restype = I
        L.orc_sw_score.argtypes = [P, I, I, I, P, I, P, I]
        L.orc_sw_score.restype = I
        L.orc_sw_eq2.argtypes = [P, I, P, P, I, P, I, P]
        L.orc_sw_eq2.restype = I
        L.orc_sw_eq2_path.argtypes = [P, I, P, P, I, P, I, P, P, P]
        L.orc_sw_eq2_path.restype = I
        L.orc_sw_batch.argtypes = [P, I, I, I, P, I, P, P, I, P, P, P, P]
        L.orc_sw_batch.restype = I
        L.orc_merge.argtypes = [P, I, I, P, P, P]
        L.orc_merge.restype = I
        L.orc_rows.argtypes = [P, P, I, I, P, P, P, ctypes.c_int64, P]
        L.orc_rows.restype = I
        L.orc_msa.argtypes = [P, I, I, I, P, P, I, I, P, P, P, P, P, P, P]
        L.orc_msa.restype = I
        L.orc_center_exact.argtypes = [P, I, I, I, P, P, I, P]
        L.orc_center_exact.restype = I
        L.orc_center_judge.argtypes = [P, I, I, I, P, P, I, P, I, P]
        L.orc_center_judge.restype = I
        for fn in ("orc_sp_pairs", "orc_sp_columns"):
            getattr(L, fn).argtypes = [P, I, ctypes.c_int64]
            getattr(L, fn).restype = ctypes.c_int64
        L.orc_encode.argtypes = [P, ctypes.c_int64, P]
        L.orc_encode.restype = None
        L.orc_nuc_matches.argtypes = [P, I, P, I, I, P, P, I]
        L.orc_nuc_matches.restype = I
        L.orc_nuc_chain.argtypes = [P, P, I, I, P]
        L.orc_nuc_chain.restype = I
        L.orc_nuc_align.argtypes = [P, I, I, I, I, P, I, P, I, P, P, P, P]
        L.orc_nuc_align.restype = I
        L.orc_nuc_msa.argtypes = [P, I, I, I, I, P, P, I, P, P, P, P, P, P]
        L.orc_nuc_msa.restype = I
        L.orc_column_profile.argtypes = [P, I, ctypes.c_int64, I, P]
        L.orc_column_profile.restype = I
        L.orc_sp_blosum.argtypes = [P, I, I, P, I, ctypes.c_int64]
        L.orc_sp_blosum.restype = ctypes.c_int64
        L.orc_pdist_counts.argtypes = [P, ctypes.c_int64, I, I, P, P]
        L.orc_pdist_counts.restype = None
        L.orc_pdist.argtypes = [P, ctypes.c_int64, I, I]
        L.orc_pdist.restype = ctypes.c_double
        L.orc_nj.argtypes = [P, I, P, P]
        L.orc_nj.restype = I
        L.orc_nj_clusters.argtypes = [P, I, ctypes.c_int64, P, P, P]
        L.orc_nj_clusters.restype = I
        L.orc_nj_tree.argtypes = [P, I, ctypes.c_int64, P, P, P]
        L.orc_nj_tree.restype = I
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def _mat(S) -> np.ndarray:
    S = np.ascontiguousarray(S, dtype=np.int8)
    assert S.ndim == 2 and S.shape[0] == S.shape[1]
    return S


def _check(r: int) -> int:
    if r < 0:
        raise ValueError(f"oracle error {r}")
    return r


def encode(text) -> np.ndarray:
    """Protein text (str or bytes) -> residue codes."""
    raw = np.frombuffer(text.encode() if isinstance(text, str) else bytes(text), dtype=np.uint8).copy()
    out = np.zeros(len(raw), np.uint8)
    if len(raw):
        lib().orc_encode(_p(raw), len(raw), _p(out))
    return out


def sw(S, go: int, ge: int, c, s, want_ops: bool = False):
    """Affine SW of s against center c.  Returns dict(score, cells, ins, aligned[, ops])."""
    S = _mat(S)
    c, s = _u8(c), _u8(s)
    m, n = len(c), len(s)
    cells = np.zeros(4, np.int32)
    ins = np.zeros(m + 1, np.uint16)
    al = np.zeros(max(m, 1), np.uint8)
    ops = ctypes.create_string_buffer(m + n + 1)
    nops = ctypes.c_int32(0)
    r = _check(lib().orc_sw(_p(S), S.shape[0], go, ge, _p(c), m, _p(s), n, _p(cells), _p(ins),
                            _p(al), ops, ctypes.byref(nops)))
    out = dict(score=r, cells=cells, ins=ins, aligned=al[:m].copy())
    if want_ops:
        out["ops"] = ops.raw[:nops.value].decode()
    return out


def sw_score(S, go: int, ge: int, a, b) -> int:
    S = _mat(S)
    a, b = _u8(a), _u8(b)
    return _check(lib().orc_sw_score(_p(S), S.shape[0], go, ge, _p(a), len(a), _p(b), len(b)))


def sw_eq2(S, W, c, s):
    """Literal eq. 2 with a general gap table W[k] (W[0] unused).  Returns (score, H, cells, ops)."""
    S = _mat(S)
    c, s = _u8(c), _u8(s)
    m, n = len(c), len(s)
    W = np.ascontiguousarray(W, dtype=np.int32)
    assert len(W) > max(m, n)
    H = np.zeros((m + 1, n + 1), np.int32)
    score = _check(lib().orc_sw_eq2(_p(S), S.shape[0], _p(W), _p(c), m, _p(s), n, _p(H)))
    cells = np.zeros(4, np.int32)
    ops = ctypes.create_string_buffer(m + n + 1)
    k = _check(lib().orc_sw_eq2_path(_p(S), S.shape[0], _p(W), _p(c), m, _p(s), n, _p(H),
                                     _p(cells), ops))
    return score, H, cells, ops.raw[:k].decode()


def sw_batch(S, go: int, ge: int, center, residues, offsets):
    """Every sequence against the center; returns (score, cells, ins, aligned)."""
    S = _mat(S)
    center = _u8(center)
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    N, m = len(off) - 1, len(center)
    score = np.zeros(N, np.int32)
    cells = np.zeros((N, 4), np.int32)
    ins = np.zeros((N, m + 1), np.uint16)
    al = np.zeros((N, max(m, 1)), np.uint8)
    _check(lib().orc_sw_batch(_p(S), S.shape[0], go, ge, _p(center), m, _p(res), _p(off), N,
                              _p(score), _p(cells), _p(ins), _p(al)))
    return score, cells, ins, al[:, :m].copy()


def merge(ins: np.ndarray):
    ins = np.ascontiguousarray(ins, dtype=np.uint16)
    N, m1 = ins.shape
    G = np.zeros(m1, np.int32)
    col = np.zeros(m1, np.int64)
    W = ctypes.c_int64(0)
    _check(lib().orc_merge(_p(ins), N, m1 - 1, _p(G), _p(col), ctypes.byref(W)))
    return G, col, int(W.value)


def rows(residues, offsets, ins, aligned, G, width: int) -> np.ndarray:
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ins = np.ascontiguousarray(ins, dtype=np.uint16)
    N, m1 = ins.shape
    m = m1 - 1
    al = np.zeros((N, max(m, 1)), np.uint8)
    al[:, :m] = aligned
    G = np.ascontiguousarray(G, dtype=np.int32)
    msa = np.zeros((N, max(width, 1)), np.uint8)
    _check(lib().orc_rows(_p(res), _p(off), N, m, _p(ins), _p(al), _p(G), width, _p(msa)))
    return msa[:, :width].copy()


def msa(S, go: int, ge: int, residues, offsets, center: int):
    """Full center-star MSA for a given center.  Returns a dict of every stage's output."""
    S = _mat(S)
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    N = len(off) - 1
    m = int(off[center + 1] - off[center])
    score = np.zeros(N, np.int32)
    cells = np.zeros((N, 4), np.int32)
    ins = np.zeros((N, m + 1), np.uint16)
    al = np.zeros((N, max(m, 1)), np.uint8)
    G = np.zeros(m + 1, np.int32)
    col = np.zeros(m + 1, np.int64)
    W = ctypes.c_int64(0)
    _check(lib().orc_msa(_p(S), S.shape[0], go, ge, _p(res), _p(off), N, center, _p(score),
                         _p(cells), _p(ins), _p(al), _p(G), _p(col), ctypes.byref(W)))
    aligned = al[:, :m].copy()
    width = int(W.value)
    return dict(score=score, cells=cells, ins=ins, aligned=aligned, G=G, col=col, width=width,
                msa=rows(res, off, ins, aligned, G, width))


def center_exact(S, go: int, ge: int, residues, offsets):
    S = _mat(S)
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    N = len(off) - 1
    sums = np.zeros(N, np.int64)
    best = _check(lib().orc_center_exact(_p(S), S.shape[0], go, ge, _p(res), _p(off), N, _p(sums)))
    return best, sums


def center_judge(S, go: int, ge: int, residues, offsets, cand):
    S = _mat(S)
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    sums = np.zeros(len(cand), np.int64)
    best = _check(lib().orc_center_judge(_p(S), S.shape[0], go, ge, _p(res), _p(off),
                                         len(off) - 1, _p(cand), len(cand), _p(sums)))
    return best, sums


def sp_pairs(msa_rows: np.ndarray) -> int:
    a = _u8(msa_rows)
    return int(lib().orc_sp_pairs(_p(a), a.shape[0], a.shape[1]))


def sp_columns(msa_rows: np.ndarray) -> int:
    a = _u8(msa_rows)
    return int(lib().orc_sp_columns(_p(a), a.shape[0], a.shape[1]))


def column_profile(msa_rows: np.ndarray, alpha: int) -> np.ndarray:
    """int32 [width][alpha + 1]: residue counts per column, gaps last."""
    a = _u8(msa_rows)
    out = np.zeros((a.shape[1], alpha + 1), np.int32)
    r = lib().orc_column_profile(_p(a), a.shape[0], a.shape[1], alpha, _p(out))
    if r != 0:
        raise ValueError("byte outside the alphabet and not a gap")
    return out


def avg_sp(msa_rows: np.ndarray) -> float:
    N = msa_rows.shape[0]
    return sp_columns(msa_rows) / (N * (N - 1) / 2) if N > 1 else 0.0


def sp_blosum(S, ge: int, msa_rows: np.ndarray) -> int:
    S = _mat(S)
    a = _u8(msa_rows)
    return int(lib().orc_sp_blosum(_p(S), S.shape[0], ge, _p(a), a.shape[0], a.shape[1]))


# ---------------------------------------------------------------------------
# Nucleotide center star (trie section): segments, matches, anchor chain,
# global alignment of the unmatched stretches
# ---------------------------------------------------------------------------
def nuc_matches(c, s, k: int):
    """(q, p) arrays: every match of an indexed center segment in s, by p."""
    c, s = _u8(c), _u8(s)
    cap = len(s) + 1
    mq = np.zeros(cap, np.int32)
    mp = np.zeros(cap, np.int32)
    a = _check(lib().orc_nuc_matches(_p(c), len(c), _p(s), len(s), k, _p(mq), _p(mp), cap))
    return mq[:a].copy(), mp[:a].copy()


def nuc_chain(mq, mp, k: int) -> np.ndarray:
    """Indices of the anchor chain among the matches (mq, mp)."""
    mq = np.ascontiguousarray(mq, np.int32)
    mp = np.ascontiguousarray(mp, np.int32)
    ch = np.zeros(max(1, len(mq)), np.int32)
    n = _check(lib().orc_nuc_chain(_p(mq), _p(mp), len(mq), k, _p(ch)))
    return ch[:n].copy()


def nuc_align(S, go: int, ge: int, k: int, c, s):
    """Pairwise nucleotide center-star alignment: dict(score, ins, aligned, anchors)."""
    S = _mat(S)
    c, s = _u8(c), _u8(s)
    m = len(c)
    ins = np.zeros(m + 1, np.uint16)
    al = np.zeros(max(m, 1), np.uint8)
    sc = ctypes.c_int32(0)
    na = ctypes.c_int32(0)
    _check(lib().orc_nuc_align(_p(S), S.shape[0], go, ge, k, _p(c), m, _p(s), len(s), ctypes.byref(sc), _p(ins),
                               _p(al), ctypes.byref(na)))
    return dict(score=int(sc.value), ins=ins, aligned=al[:m].copy(), anchors=int(na.value))


def nuc_msa(S, go: int, ge: int, k: int, residues, offsets):
    """Nucleotide MSA with sequence 0 as the center: dict of every stage's output."""
    S = _mat(S)
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    N = len(off) - 1
    m = int(off[1] - off[0])
    score = np.zeros(N, np.int32)
    ins = np.zeros((N, m + 1), np.uint16)
    al = np.zeros((N, max(m, 1)), np.uint8)
    G = np.zeros(m + 1, np.int32)
    col = np.zeros(m + 1, np.int64)
    W = ctypes.c_int64(0)
    _check(lib().orc_nuc_msa(_p(S), S.shape[0], go, ge, k, _p(res), _p(off), N, _p(score), _p(ins), _p(al), _p(G),
                             _p(col), ctypes.byref(W)))
    al = al[:, :m].copy()
    msa_rows = rows(res, off, ins, al, G, int(W.value))
    return dict(score=score, ins=ins, aligned=al, G=G, col=col, width=int(W.value), msa=msa_rows)


# ---------------------------------------------------------------------------
# Phylogeny from the MSA (NJ section, Fig. 4): p-distances, neighbour joining,
# the sampled clustering and the merged tree
# ---------------------------------------------------------------------------
def pdist_counts(msa_rows: np.ndarray):
    """(mism, comp) int64 N x N: mismatching and compared (both non-gap) columns."""
    a = _u8(msa_rows)
    n, w = a.shape
    mism = np.zeros((n, n), np.int64)
    comp = np.zeros((n, n), np.int64)
    mm, cc = ctypes.c_int64(0), ctypes.c_int64(0)
    for i in range(n):
        for j in range(n):
            lib().orc_pdist_counts(_p(a), w, i, j, ctypes.byref(mm), ctypes.byref(cc))
            mism[i, j], comp[i, j] = mm.value, cc.value
    return mism, comp


def pdist(msa_rows: np.ndarray) -> np.ndarray:
    """N x N p-distances (1 where two rows share no compared column)."""
    a = _u8(msa_rows)
    n, w = a.shape
    return np.array([[lib().orc_pdist(_p(a), w, i, j) for j in range(n)] for i in range(n)])


def nj(D: np.ndarray):
    """Neighbour joining over D: (parent, blen) per node, leaves 0..n-1 first."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    n = D.shape[0]
    parent = np.zeros(max(2 * n, 3), np.int32)
    blen = np.zeros(max(2 * n, 3), np.float64)
    nn = _check(lib().orc_nj(_p(D), n, _p(parent), _p(blen)))
    return parent[:nn].copy(), blen[:nn].copy()


def nj_clusters(msa_rows: np.ndarray, perm):
    """(label per row, seed row per cluster) of the sampled clustering."""
    a = _u8(msa_rows)
    n, w = a.shape
    perm = np.ascontiguousarray(perm, np.int32)
    label = np.zeros(n, np.int32)
    seed = np.zeros(n, np.int32)
    K = _check(lib().orc_nj_clusters(_p(a), n, w, _p(perm), _p(label), _p(seed)))
    return label, seed[:K].copy()


def nj_tree(msa_rows: np.ndarray, perm):
    """The merged tree: (parent, blen) per node, rows 0..N-1 first."""
    a = _u8(msa_rows)
    n, w = a.shape
    perm = np.ascontiguousarray(perm, np.int32)
    parent = np.zeros(2 * n + 2, np.int32)
    blen = np.zeros(2 * n + 2, np.float64)
    nn = _check(lib().orc_nj_tree(_p(a), n, w, _p(perm), _p(parent), _p(blen)))
    return parent[:nn].copy(), blen[:nn].copy()
