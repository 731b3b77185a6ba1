"""MI355X (gfx950) center-star protein MSA -- Python binding of libhalign.so.

The binding only marshals arguments: device memory comes from torch tensors
(``data_ptr()``), streams from ``torch.cuda.current_stream()``, and every step
of the path runs in the HIP kernels of ``csrc/``.  If the built library is
missing the import of this module still works, but every call raises.

Function names follow the C ABI in ``include/halign.h``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import synth
from ._build import LIB_PATH

GAP = 255
FEAT, HID, EMB = 8000, 256, 64

HALIGN_OK = 0
HALIGN_SCORE_ONLY = 0
HALIGN_TRACEBACK = 1
HALIGN_ROUTE_AUTO = 0
HALIGN_ROUTE_INTER = 1 << 4
HALIGN_ROUTE_INTRA = 2 << 4
HALIGN_GRAPH = 1 << 8
HALIGN_CENTER_EXACT = -1
HALIGN_CENTER_LEARNED = -2


class HalignError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"halign error {code}: {msg}")
        self.code = code


class _Scoring(ctypes.Structure):
    _fields_ = [("matrix_host", ctypes.c_void_p), ("alphabet", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class _Seqs(ctypes.Structure):
    _fields_ = [("residues", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("offsets_host", ctypes.c_void_p), ("n", ctypes.c_int32)]


class _Model(ctypes.Structure):
    _fields_ = [("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p),
                ("W2", ctypes.c_void_p), ("b2", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p), ("W2", ctypes.c_void_p),
                ("b2", ctypes.c_void_p), ("W1b", ctypes.c_void_p), ("W2b", ctypes.c_void_p)]


class _TrainOpts(ctypes.Structure):
    _fields_ = [("anchors", ctypes.c_int32), ("batch", ctypes.c_int32), ("epochs", ctypes.c_int32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint64), ("ema", ctypes.c_float),
                ("partners", ctypes.c_int32), ("group_weight", ctypes.c_float)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)

_lib = None


def lib():
    """Load libhalign.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "halign_ctx_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(P)], I),
        "halign_ctx_destroy": ([P], None),
        "halign_last_error": ([], ctypes.c_char_p),
        "halign_ctx_workspace_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], I),
        "halign_ctx_last_timings": ([P, P], I),
        "halign_ctx_last_stats": ([P, P], I),
        "halign_debug_fail_chunk": ([P, ctypes.c_int], I),
        "halign_ctx_set_autotune": ([P, ctypes.c_int], I),
        "halign_ctx_last_plan": ([P, P], I),
        "halign_ctx_set_graph": ([P, ctypes.c_int], I),
        "halign_ctx_graph_launches": ([P, P], I),
        "halign_encode": ([P, I64, P, P], I),
        "halign_sw_batch": ([P, P, P, I, P, U32, P, P, P, P, P], I),
        "halign_sw_score_noalloc": ([P, P, I, P, P, P, P], I),
        "halign_sw_pairs": ([P, P, P, P, I, P, P, P], I),
        "halign_merge": ([P, P, I, I, P, P, P, P], I),
        "halign_emit_rows": ([P, P, I, P, P, P, P, I64, P, P], I),
        "halign_center_exact": ([P, P, P, P, P, P], I),
        "halign_center_judge": ([P, P, P, P, I, P, P, P], I),
        "halign_center_judge_sample": ([P, P, P, P, I, P, I, P, P, P], I),
        "halign_ctx_set_prejudge": ([P, ctypes.c_int, ctypes.c_int], I),
        "halign_featurize": ([P, P, I, P, P], I),
        "halign_mlp_forward": ([P, P, P, I, P, P, P, P], I),
        "halign_pair_loss": ([P, P, P, I, P, P, P], I),
        "halign_pair_loss_grouped": ([P, P, P, I, I, ctypes.c_float, P, P, P], I),
        "halign_mlp_backward": ([P, P, P, I, P, P, P, P, P, P, P, P], I),
        "halign_f32_to_bf16": ([P, P, I64, P], I),
        "halign_exact_tiling": ([I64, I, I64, P, P, P], I),
        "halign_adam_step": ([P, P, P, P, P, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, I, P], I),
        "halign_topk_center": ([P, P, I, I, P, P, P], I),
        "halign_train_proposer": ([P, P, P, P, P, P, P], I),
        "halign_center_learned": ([P, P, P, P, I, P, P, P], I),
        "halign_msa": ([P, P, P, I, P, _ALLOC_FN, P, P, P, P, P], I),
        "halign_nuc_align": ([P, P, P, I, I, P, P, P, P, P], I),
        "halign_nuc_msa": ([P, P, P, I, I, P, _ALLOC_FN, P, P, P, P], I),
        "halign_sp_score": ([P, P, I, I64, P, P], I),
        "halign_column_profile": ([P, I, I64, I, P, P], I),
        "halign_pdist": ([P, P, I, I64, P, I, P, I, P, P, P, P], I),
        "halign_nj": ([P, P, I, P, P, P, P], I),
        "halign_nj_tree": ([P, P, I, I64, P, P, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        if not hasattr(L, name):
            continue
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != HALIGN_OK:
        msg = lib().halign_last_error()
        raise HalignError(rc, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
class Scoring:
    """s(a, b) and W_k = gap_open + k * gap_extend (host-side parameters)."""

    def __init__(self, matrix=None, gap_open: int = synth.GAP_OPEN, gap_extend: int = synth.GAP_EXTEND):
        mat = synth.BLOSUM62 if matrix is None else matrix
        self.matrix = np.ascontiguousarray(mat, dtype=np.int8)
        self.gap_open, self.gap_extend = int(gap_open), int(gap_extend)
        self._c = _Scoring(self.matrix.ctypes.data, self.matrix.shape[0], self.gap_open, self.gap_extend)

    @property
    def ref(self):
        return ctypes.byref(self._c)


class DeviceSeqs:
    """A packed sequence set resident on the GPU (residues + offsets) plus the
    host copy of the offsets the planner needs."""

    def __init__(self, seqs: synth.SeqSet, device: str = "cuda"):
        import torch
        self.host = seqs
        self.offsets_host = np.ascontiguousarray(seqs.offsets, dtype=np.int64)
        res = seqs.residues if len(seqs.residues) else np.zeros(1, np.uint8)
        self.residues = torch.from_numpy(np.ascontiguousarray(res)).to(device)
        self.offsets = torch.from_numpy(self.offsets_host.copy()).to(device)
        self.n = seqs.n
        self._c = _Seqs(self.residues.data_ptr(), self.offsets.data_ptr(),
                        self.offsets_host.ctypes.data, self.n)

    @property
    def ref(self):
        return ctypes.byref(self._c)

    def length(self, k: int) -> int:
        return int(self.offsets_host[k + 1] - self.offsets_host[k])

    def seq_ptr(self, k: int) -> int:
        return self.residues.data_ptr() + int(self.offsets_host[k])


class Context:
    """Owns a halign_ctx (device scratch for codes, plans)."""

    def __init__(self, device: int = 0, workspace_cap: int = 0):
        h = ctypes.c_void_p()
        _check(lib().halign_ctx_create(device, workspace_cap, ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().halign_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        v = ctypes.c_size_t(0)
        _check(lib().halign_ctx_workspace_bytes(self.h, ctypes.byref(v)))
        return int(v.value)

    def last_timings(self):
        a = (ctypes.c_float * 3)()
        _check(lib().halign_ctx_last_timings(self.h, a))
        return list(a)

    def last_stats(self):
        a = (ctypes.c_int64 * 4)()
        _check(lib().halign_ctx_last_stats(self.h, a))
        return dict(cells=a[0], launches=a[1], route=a[2], chunks=a[3])

    def set_autotune(self, on: bool):
        _check(lib().halign_ctx_set_autotune(self.h, 1 if on else 0))

    def last_plan(self):
        a = (ctypes.c_int32 * 5)()
        _check(lib().halign_ctx_last_plan(self.h, a))
        return dict(route=a[0], R=a[1], streams=a[2], lanes=a[3], packed=a[4])

    def set_graph(self, on: bool):
        _check(lib().halign_ctx_set_graph(self.h, 1 if on else 0))

    def graph_launches(self) -> int:
        v = ctypes.c_int64(0)
        _check(lib().halign_ctx_graph_launches(self.h, ctypes.byref(v)))
        return int(v.value)

    def set_prejudge(self, candidates: int, partners: int):
        _check(lib().halign_ctx_set_prejudge(self.h, candidates, partners))

    def fail_chunk(self, c: int):
        _check(lib().halign_debug_fail_chunk(self.h, c))


# ---------------------------------------------------------------------------
# Thin wrappers with the C names.  Tensors are torch CUDA tensors.
# ---------------------------------------------------------------------------
def halign_encode(ascii_t, codes_t, stream=None):
    _check(lib().halign_encode(_ptr(ascii_t), ascii_t.numel(), _ptr(codes_t), _stream(stream)))


def halign_sw_batch(ctx: Context, sc: Scoring, center_t, m: int, seqs: DeviceSeqs, flags: int,
                    score, cells=None, ins=None, aligned=None, stream=None):
    _check(lib().halign_sw_batch(ctx.h, sc.ref, ctypes.c_void_p(center_t if isinstance(center_t, int)
                                                                  else center_t.data_ptr()),
                                 m, seqs.ref, flags, _ptr(score), _ptr(cells), _ptr(ins), _ptr(aligned),
                                 _stream(stream)))


def halign_sw_score_noalloc(sc: Scoring, center_t, m: int, seqs: DeviceSeqs, score, cells=None, stream=None):
    _check(lib().halign_sw_score_noalloc(sc.ref, ctypes.c_void_p(center_t if isinstance(center_t, int)
                                                                 else center_t.data_ptr()),
                                         m, seqs.ref, _ptr(score), _ptr(cells), _stream(stream)))


def halign_sw_pairs(ctx: Context, sc: Scoring, seqs: DeviceSeqs, anchors: np.ndarray,
                    partners: np.ndarray, score, stream=None):
    a = np.ascontiguousarray(anchors, dtype=np.int32)
    b = np.ascontiguousarray(partners, dtype=np.int32)
    assert len(b) == 64 * len(a)
    _check(lib().halign_sw_pairs(ctx.h, sc.ref, seqs.ref, a.ctypes.data, len(a), b.ctypes.data,
                                 _ptr(score), _stream(stream)))


def halign_merge(ctx: Context, ins, n: int, m: int, G, col, stream=None) -> int:
    w = ctypes.c_int64(0)
    _check(lib().halign_merge(ctx.h, _ptr(ins), n, m, _ptr(G), _ptr(col), ctypes.byref(w), _stream(stream)))
    return int(w.value)


def halign_emit_rows(ctx: Context, seqs: DeviceSeqs, m: int, ins, aligned, G, col, width: int, msa,
                     stream=None):
    _check(lib().halign_emit_rows(ctx.h, seqs.ref, m, _ptr(ins), _ptr(aligned), _ptr(G), _ptr(col),
                                  width, _ptr(msa), _stream(stream)))


def halign_center_exact(ctx: Context, sc: Scoring, seqs: DeviceSeqs, sums, stream=None) -> int:
    c = ctypes.c_int32(-1)
    _check(lib().halign_center_exact(ctx.h, sc.ref, seqs.ref, _ptr(sums), ctypes.byref(c), _stream(stream)))
    return int(c.value)


def halign_center_judge(ctx: Context, sc: Scoring, seqs: DeviceSeqs, cand, sums, stream=None) -> int:
    c = ctypes.c_int32(-1)
    _check(lib().halign_center_judge(ctx.h, sc.ref, seqs.ref, _ptr(cand), cand.numel(), _ptr(sums),
                                     ctypes.byref(c), _stream(stream)))
    return int(c.value)


def halign_center_judge_sample(ctx: Context, sc: Scoring, seqs: DeviceSeqs, cand, partners: np.ndarray, sums,
                               stream=None) -> int:
    c = ctypes.c_int32(-1)
    pa = np.ascontiguousarray(partners, dtype=np.int32)
    _check(lib().halign_center_judge_sample(ctx.h, sc.ref, seqs.ref, _ptr(cand), cand.numel(), pa.ctypes.data,
                                            len(pa), _ptr(sums), ctypes.byref(c), _stream(stream)))
    return int(c.value)


def halign_sp_score(sc: Scoring, msa, stream=None):
    out = (ctypes.c_int64 * 2)()
    n, w = (msa.shape[0], msa.shape[1]) if msa.dim() == 2 else (0, 0)
    _check(lib().halign_sp_score(sc.ref, _ptr(msa), n, w, out, _stream(stream)))
    return int(out[0]), int(out[1])


def halign_column_profile(msa, alphabet: int = 24, out=None, stream=None):
    """int32 [W, alphabet + 1] device tensor: residue counts per MSA column, gaps last."""
    import torch
    n, w = (msa.shape[0], msa.shape[1]) if msa.dim() == 2 else (0, 0)
    if out is None:
        out = torch.empty((w, alphabet + 1), dtype=torch.int32, device=msa.device)
    _check(lib().halign_column_profile(_ptr(msa), n, w, alphabet, _ptr(out), _stream(stream)))
    return out


def halign_pdist(ctx: Context, msa, a_rows=None, b_rows=None, counts: bool = False, stream=None):
    """p-distances between MSA rows (device uint8 [N, W]): float64 [na, nb]
    device tensor (rows a_rows x b_rows, int32 device tensors; None: all
    rows); with counts=True also the int32 mismatch and compared-column counts."""
    import torch
    n, w = msa.shape[0], msa.shape[1]
    na = n if a_rows is None else a_rows.numel()
    nb = n if b_rows is None else b_rows.numel()
    dev = msa.device
    D = torch.empty((na, nb), dtype=torch.float64, device=dev)
    mm = torch.empty((na, nb), dtype=torch.int32, device=dev) if counts else None
    cc = torch.empty((na, nb), dtype=torch.int32, device=dev) if counts else None
    _check(lib().halign_pdist(ctx.h, _ptr(msa), n, w, _ptr(a_rows), na, _ptr(b_rows), nb, _ptr(D), _ptr(mm),
                              _ptr(cc), _stream(stream)))
    return (D, mm, cc) if counts else D


def halign_nj(ctx: Context, D, stream=None):
    """Neighbour joining over a float64 device distance matrix [n, n]:
    (parent int32, blen float64) numpy arrays per node, leaves 0..n-1 first."""
    n = D.shape[0]
    parent = np.zeros(2 * n + 1, np.int32)
    blen = np.zeros(2 * n + 1, np.float64)
    nodes = ctypes.c_int32(0)
    _check(lib().halign_nj(ctx.h, _ptr(D), n, parent.ctypes.data, blen.ctypes.data, ctypes.byref(nodes),
                           _stream(stream)))
    return parent[:nodes.value].copy(), blen[:nodes.value].copy()


def halign_nj_tree(ctx: Context, msa, perm, stream=None):
    """The tree of an MSA (device uint8 [N, W]) with the sample drawn by perm
    (a permutation of 0..N-1): (parent int32, blen float64) numpy arrays per
    node, rows 0..N-1 first."""
    n, w = msa.shape[0], msa.shape[1]
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    parent = np.zeros(2 * n + 2, np.int32)
    blen = np.zeros(2 * n + 2, np.float64)
    nodes = ctypes.c_int32(0)
    _check(lib().halign_nj_tree(ctx.h, _ptr(msa), n, w, perm.ctypes.data, parent.ctypes.data, blen.ctypes.data,
                                ctypes.byref(nodes), _stream(stream)))
    return parent[:nodes.value].copy(), blen[:nodes.value].copy()


def newick(parent, blen, names=None) -> str:
    """Newick text of a (parent, blen) tree (leaves named by index unless names given)."""
    nn = len(parent)
    kids = [[] for _ in range(nn)]
    root = -1
    for v in range(nn):
        if parent[v] < 0:
            root = v
        else:
            kids[parent[v]].append(v)
    out = []

    def walk(v):   # iterative: deep trees
        stack = [(v, 0)]
        while stack:
            x, k = stack.pop()
            if k == 0 and kids[x]:
                out.append("(")
            if k < len(kids[x]):
                if k > 0:
                    out.append(",")
                stack.append((x, k + 1))
                stack.append((kids[x][k], 0))
                continue
            if kids[x]:
                out.append(")")
            else:
                out.append(str(names[x]) if names is not None else str(x))
            if parent[x] >= 0:
                out.append(f":{blen[x]:.6g}")
    walk(root)
    return "".join(out) + ";"


def halign_msa(ctx: Context, sc: Scoring, seqs: DeviceSeqs, center: int, model=None, stream=None, out=None):
    """End-to-end MSA.  Returns (msa uint8 tensor [N, W], center index).
    `out`: an optional uint8 device tensor that the MSA is written into when it
    holds N * W bytes (the result is then a view of it); otherwise a new
    tensor is allocated once W is known."""
    import torch
    keep = {}

    def _alloc(nbytes, user):
        if out is not None and out.dtype == torch.uint8 and out.is_contiguous() and out.numel() >= nbytes:
            keep["t"] = out.view(-1)
        else:
            keep["t"] = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{ctx.device}")
        return keep["t"].data_ptr()

    cb = _ALLOC_FN(_alloc)
    out_ptr = ctypes.c_void_p()
    width = ctypes.c_int64(0)
    cout = ctypes.c_int32(-1)
    mref = ctypes.byref(model._c) if model is not None else None
    _check(lib().halign_msa(ctx.h, sc.ref, seqs.ref, center, mref, cb, None, ctypes.byref(out_ptr),
                            ctypes.byref(width), ctypes.byref(cout), _stream(stream)))
    W = int(width.value)
    t = keep["t"][: seqs.n * W].view(seqs.n, W)
    return t, int(cout.value)


def halign_nuc_align(ctx: Context, sc: Scoring, seqs: DeviceSeqs, center: int, k: int, score, ins, aligned, G=None,
                     stream=None):
    _check(lib().halign_nuc_align(ctx.h, sc.ref, seqs.ref, center, k, _ptr(score), _ptr(ins), _ptr(aligned), _ptr(G),
                                  _stream(stream)))


def halign_nuc_msa(ctx: Context, sc: Scoring, seqs: DeviceSeqs, k: int, center: int = 0, stream=None, out=None):
    """Nucleotide center-star MSA (trie section).  Returns (msa uint8 [N, W], score int32 [N])."""
    import torch
    keep = {}

    def _alloc(nbytes, user):
        if out is not None and out.dtype == torch.uint8 and out.is_contiguous() and out.numel() >= nbytes:
            keep["t"] = out.view(-1)
        else:
            keep["t"] = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{ctx.device}")
        return keep["t"].data_ptr()

    cb = _ALLOC_FN(_alloc)
    score = torch.empty(seqs.n, dtype=torch.int32, device=f"cuda:{ctx.device}")
    out_ptr = ctypes.c_void_p()
    width = ctypes.c_int64(0)
    _check(lib().halign_nuc_msa(ctx.h, sc.ref, seqs.ref, center, k, _ptr(score), cb, None, ctypes.byref(out_ptr),
                                ctypes.byref(width), _stream(stream)))
    W = int(width.value)
    return keep["t"][: seqs.n * W].view(seqs.n, W), score


# ---------------------------------------------------------------------------
# Convenience layer (allocation of outputs)
# ---------------------------------------------------------------------------
def sw_batch(ctx: Context, sc: Scoring, seqs: DeviceSeqs, center: int, traceback: bool = True,
             route: int = HALIGN_ROUTE_AUTO, center_seq=None, graph: bool = False, out=None):
    """SW of every sequence against sequence `center` (or `center_seq`, a
    uint8 CUDA tensor).  Returns dict of CUDA tensors."""
    import torch
    dev = seqs.residues.device
    N = seqs.n
    if center_seq is None:
        m = seqs.length(center)
        cptr = seqs.seq_ptr(center)
    else:
        m = int(center_seq.numel())
        cptr = center_seq.data_ptr()
    if out is not None:   # reuse output tensors (graph replays need the same pointers)
        score, cells, ins, aligned = out["score"], out["cells"], out["ins"], out["aligned"]
    else:
        score = torch.empty(N, dtype=torch.int32, device=dev)
        cells = torch.empty((N, 4), dtype=torch.int32, device=dev)
        ins = aligned = None
        if traceback:
            ins = torch.empty((N, m + 1), dtype=torch.int16, device=dev)
            aligned = torch.empty((N, (m + 31) // 32), dtype=torch.int32, device=dev)
    flags = (HALIGN_TRACEBACK if traceback else HALIGN_SCORE_ONLY) | route | (HALIGN_GRAPH if graph else 0)
    halign_sw_batch(ctx, sc, cptr, m, seqs, flags, score, cells, ins, aligned)
    return dict(score=score, cells=cells, ins=ins, aligned=aligned, m=m)


def aligned_to_bool(aligned_words: np.ndarray, m: int) -> np.ndarray:
    """uint32 bit rows -> uint8 [N, m] (host helper for comparisons)."""
    w = np.ascontiguousarray(aligned_words).view(np.uint32)
    bits = (w[:, :, None] >> np.arange(32, dtype=np.uint32)[None, None, :]) & 1
    return bits.reshape(w.shape[0], -1)[:, :m].astype(np.uint8)


# ---------------------------------------------------------------------------
# Learned center proposer
# ---------------------------------------------------------------------------
class Proposer:
    """MLP parameters on the GPU: fp32 masters and the bf16 copies the
    forward reads.  Initialised He-uniform from a seed (host numpy)."""

    def __init__(self, seed: int = 1, device: str = "cuda", params=None):
        import torch
        if params is None:
            rng = np.random.default_rng(seed)
            l1, l2 = np.sqrt(6.0 / FEAT), np.sqrt(6.0 / HID)
            params = (rng.uniform(-l1, l1, size=(FEAT, HID)).astype(np.float32), np.zeros(HID, np.float32),
                      rng.uniform(-l2, l2, size=(HID, EMB)).astype(np.float32), np.zeros(EMB, np.float32))
        W1, b1, W2, b2 = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device) for x in params]
        self.W1, self.b1, self.W2, self.b2 = W1, b1, W2, b2
        self.W1b = torch.empty(W1.shape, dtype=torch.int16, device=device)
        self.W2b = torch.empty(W2.shape, dtype=torch.int16, device=device)
        self.refresh_bf16()

    def refresh_bf16(self):
        for src, dst in ((self.W1, self.W1b), (self.W2, self.W2b)):
            halign_f32_to_bf16(src, dst)

    def model(self):
        m = _Model(self.W1b.data_ptr(), self.b1.data_ptr(), self.W2b.data_ptr(), self.b2.data_ptr())
        self._c = m
        return m

    def params(self):
        return _Params(self.W1.data_ptr(), self.b1.data_ptr(), self.W2.data_ptr(), self.b2.data_ptr(),
                       self.W1b.data_ptr(), self.W2b.data_ptr())


def halign_featurize(seqs: DeviceSeqs, X, rows=None, nrows=None, stream=None):
    n = seqs.n if rows is None else rows.numel()
    _check(lib().halign_featurize(seqs.ref, _ptr(rows), n if nrows is None else nrows, _ptr(X), _stream(stream)))


def halign_mlp_forward(ctx: Context, prop: Proposer, X, nrows: int, Z, Hb, E, stream=None):
    m = prop.model()
    _check(lib().halign_mlp_forward(ctx.h, ctypes.byref(m), _ptr(X), nrows, _ptr(Z), _ptr(Hb), _ptr(E),
                                    _stream(stream)))


def halign_pair_loss(ctx: Context, E, target, npairs: int, dE, loss, stream=None):
    _check(lib().halign_pair_loss(ctx.h, _ptr(E), _ptr(target), npairs, _ptr(dE), _ptr(loss), _stream(stream)))


def halign_pair_loss_grouped(ctx: Context, E, target, npairs: int, group: int, lam: float, dE, loss, stream=None):
    _check(lib().halign_pair_loss_grouped(ctx.h, _ptr(E), _ptr(target), npairs, group, lam, _ptr(dE), _ptr(loss),
                                          _stream(stream)))


def halign_mlp_backward(ctx: Context, prop: Proposer, X, nrows: int, Z, Hb, dE, dW1, db1, dW2, db2, stream=None):
    m = prop.model()
    _check(lib().halign_mlp_backward(ctx.h, ctypes.byref(m), _ptr(X), nrows, _ptr(Z), _ptr(Hb), _ptr(dE),
                                     _ptr(dW1), _ptr(db1), _ptr(dW2), _ptr(db2), _stream(stream)))


def halign_f32_to_bf16(src, dst, stream=None):
    assert src.is_contiguous() and dst.is_contiguous() and src.numel() == dst.numel()
    _check(lib().halign_f32_to_bf16(_ptr(src), _ptr(dst), src.numel(), _stream(stream)))


def halign_exact_tiling(n: int, step: int, g: int = -1):
    """Group count of the exhaustive center's tiling and, for g >= 0, the
    (center position, first partner position) of group g (host only)."""
    ng, a, b0 = ctypes.c_int64(0), ctypes.c_int64(-1), ctypes.c_int64(-1)
    _check(lib().halign_exact_tiling(n, step, g, ctypes.byref(ng), ctypes.byref(a), ctypes.byref(b0)))
    return (int(ng.value), int(a.value), int(b0.value)) if g >= 0 else int(ng.value)


def halign_adam_step(p, g, m, v, pb, lr, b1, b2, eps, t, stream=None):
    _check(lib().halign_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(pb), p.numel(), lr, b1, b2, eps, t,
                                  _stream(stream)))


def halign_topk_center(ctx: Context, E, nrows: int, k: int, u, top, stream=None):
    _check(lib().halign_topk_center(ctx.h, _ptr(E), nrows, k, _ptr(u), _ptr(top), _stream(stream)))


def halign_train_proposer(ctx: Context, sc: Scoring, seqs: DeviceSeqs, prop: Proposer, anchors: int,
                          batch: int = 1024, epochs: int = 4, lr: float = 1e-3, seed: int = 7, ema: float = 0.0,
                          partners: int = 64, group_weight: float = 0.0, stream=None):
    opts = _TrainOpts(anchors, batch, epochs, lr, seed, ema, partners, group_weight)
    pr = prop.params()
    losses = (ctypes.c_float * epochs)()
    _check(lib().halign_train_proposer(ctx.h, sc.ref, seqs.ref, ctypes.byref(opts), ctypes.byref(pr), losses,
                                       _stream(stream)))
    return list(losses)


def halign_center_learned(ctx: Context, sc: Scoring, seqs: DeviceSeqs, prop: Proposer, k: int = 16, stream=None):
    cand = (ctypes.c_int32 * k)()
    c = ctypes.c_int32(-1)
    m = prop.model()
    _check(lib().halign_center_learned(ctx.h, sc.ref, seqs.ref, ctypes.byref(m), k, cand, ctypes.byref(c),
                                       _stream(stream)))
    return int(c.value), list(cand)[: min(k, seqs.n)]
