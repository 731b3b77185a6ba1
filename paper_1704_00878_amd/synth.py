"""Seeded synthetic protein families and the scoring tables they are scored with.

This module holds inputs only: the substitution matrix s(a, b) and the gap
scheme W_k that the method takes as parameters (Methods, "Smith-Waterman
algorithm for protein sequences with Spark", eq. 2 and the sentence before
eq. 1), the residue alphabet, and a deterministic generator of
family-structured protein sets.  It contains none of the method's arithmetic,
so the CPU oracle and the HIP path can both be fed from it.

The real protein benchmark the paper uses (BAliBASE 4 R10, Table 1) is not
available; the generator produces stand-ins with the same kind of structure:
sequences descended from a few random roots by substitution and indels, with
configurable length distributions.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import os
from typing import Callable, Sequence

import numpy as np

# NCBI 24-letter protein order; codes 0..23.  Codes 0..19 are the 20 standard
# amino acids, 20..22 the ambiguity letters B, Z, X and 23 the stop '*'.
ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"
N_STANDARD = 20
GAP_CODE = 255

# BLOSUM62 (Henikoff & Henikoff, PNAS 1992), half-bit units, NCBI layout.
_BLOSUM62_TEXT = """
   A  R  N  D  C  Q  E  G  H  I  L  K  M  F  P  S  T  W  Y  V  B  Z  X  *
A  4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0 -2 -1  0 -4
R -1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3 -1  0 -1 -4
N -2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3  3  0 -1 -4
D -2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3  4  1 -1 -4
C  0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1 -3 -3 -2 -4
Q -1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2  0  3 -1 -4
E -1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
G  0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3 -1 -2 -1 -4
H -2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3  0  0 -1 -4
I -1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3 -3 -3 -1 -4
L -1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1 -4 -3 -1 -4
K -1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2  0  1 -1 -4
M -1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1 -3 -1 -1 -4
F -2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1 -3 -3 -1 -4
P -1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2 -2 -1 -2 -4
S  1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2  0  0  0 -4
T  0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0 -1 -1  0 -4
W -3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3 -4 -3 -2 -4
Y -2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1 -3 -2 -1 -4
V  0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4 -3 -2 -1 -4
B -2 -1  3  4 -3  0  1 -1  0 -3 -4  0 -3 -3 -2  0 -1 -4 -3 -3  4  1 -1 -4
Z -1  0  0  1 -3  3  4 -2  0 -3 -3  1 -1 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
X  0 -1 -1 -1 -2 -1 -1 -1 -1 -1 -1 -1 -1 -1 -2  0  0 -2 -1 -1 -1 -1 -1 -4
* -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4  1
"""


def _parse_matrix(text: str) -> np.ndarray:
    lines = [ln.split() for ln in text.strip().splitlines()]
    header = lines[0]
    assert "".join(header) == ALPHABET
    mat = np.zeros((24, 24), dtype=np.int8)
    for r, row in enumerate(lines[1:]):
        assert row[0] == ALPHABET[r]
        mat[r] = [int(v) for v in row[1:]]
    return mat


BLOSUM62 = _parse_matrix(_BLOSUM62_TEXT)
BLOSUM62.setflags(write=False)

# Background amino-acid frequencies that BLOSUM62 was derived with
# (Henikoff & Henikoff 1992), three decimals, order ARNDCQEGHILKMFPSTWYV.
BACKGROUND = np.array(
    [0.074, 0.052, 0.045, 0.054, 0.025, 0.034, 0.054, 0.074, 0.026, 0.068,
     0.099, 0.058, 0.025, 0.047, 0.039, 0.057, 0.051, 0.013, 0.032, 0.073],
    dtype=np.float64)

# Default gap scheme: W_k = GAP_OPEN + GAP_EXTEND * k (a 1-residue gap costs 12).
GAP_OPEN = 11
GAP_EXTEND = 1

_ENCODE = np.full(256, 22, dtype=np.uint8)  # unknown letters -> X
for _i, _ch in enumerate(ALPHABET):
    _ENCODE[ord(_ch)] = _i
    _ENCODE[ord(_ch.lower())] = _i
_ENCODE[ord("U")] = _ENCODE[ord("u")] = ALPHABET.index("C")  # selenocysteine
_ENCODE[ord("O")] = _ENCODE[ord("o")] = ALPHABET.index("K")  # pyrrolysine
ENCODE_TABLE = _ENCODE
ENCODE_TABLE.setflags(write=False)


def encode(text: str) -> np.ndarray:
    """ASCII protein string -> uint8 codes (host-side convenience)."""
    return ENCODE_TABLE[np.frombuffer(text.encode("ascii"), dtype=np.uint8)]


def decode(codes: Sequence[int]) -> str:
    return "".join("-" if int(x) == GAP_CODE else ALPHABET[int(x)] for x in codes)


# ---------------------------------------------------------------------------
# Packed sequence sets
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class SeqSet:
    """N sequences as one concatenated uint8 code array plus int64 offsets."""
    residues: np.ndarray  # uint8[sum n]
    offsets: np.ndarray   # int64[N+1]

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def seq(self, k: int) -> np.ndarray:
        return self.residues[self.offsets[k]:self.offsets[k + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    @staticmethod
    def from_list(seqs: Sequence[np.ndarray]) -> "SeqSet":
        lens = np.array([len(s) for s in seqs], dtype=np.int64)
        offs = np.zeros(len(seqs) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        res = (np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs])
               if len(seqs) and offs[-1] > 0 else np.zeros(0, np.uint8))
        return SeqSet(res.astype(np.uint8), offs)

    def subset(self, idx: Sequence[int]) -> "SeqSet":
        """The sequences idx, in that order (one gather)."""
        idx = np.asarray(idx, dtype=np.int64).reshape(-1)
        lens = self.offsets[idx + 1] - self.offsets[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        pos = np.arange(offs[-1], dtype=np.int64) + np.repeat(self.offsets[idx] - offs[:-1], lens)
        return SeqSet(self.residues[pos].astype(np.uint8), offs)


# ---------------------------------------------------------------------------
# Family generator
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class FamilyConfig:
    name: str
    n_seqs: int
    n_roots: int
    p_sub: float
    p_indel: float
    length: Callable[[np.random.Generator, int], np.ndarray]
    seed: int


def _uniform(lo: int, hi: int):
    def draw(rng: np.random.Generator, k: int) -> np.ndarray:
        return rng.integers(lo, hi + 1, size=k)
    return draw


def _lognormal(mu: float, sigma: float, lo: int, hi: int):
    def draw(rng: np.random.Generator, k: int) -> np.ndarray:
        x = np.round(np.exp(rng.normal(mu, sigma, size=k)))
        return np.clip(x, lo, hi).astype(np.int64)
    return draw


SEED_BASE = 20170403

# The five workloads (sizes, length laws, family structure, mutation rates).
CONFIGS = {
    "plain64": FamilyConfig("plain64", 64, 1, 0.20, 0.05, _uniform(80, 160), SEED_BASE + 1),
    "batch20k": FamilyConfig("batch20k", 20_000, 8, 0.25, 0.05, _uniform(200, 500), SEED_BASE + 2),
    "longtail200k": FamilyConfig("longtail200k", 200_000, 32, 0.30, 0.08,
                                 _lognormal(5.8, 0.5, 50, 2000), SEED_BASE + 3),
    "learned50k": FamilyConfig("learned50k", 50_000, 32, 0.25, 0.05, _uniform(150, 600), SEED_BASE + 4),
    "ultra1m": FamilyConfig("ultra1m", 1_000_000, 128, 0.30, 0.06, _uniform(50, 1000), SEED_BASE + 5),
}


_BG_CDF = np.cumsum(BACKGROUND)
_BG_CDF[-1] = 1.0


def _background_draw(rng: np.random.Generator, k: int) -> np.ndarray:
    return np.searchsorted(_BG_CDF, rng.random(k), side="right").astype(np.uint8)


_CHUNK = 65536   # sequences generated per chunk (fixed: part of the recipe)


def _generate_chunk(rng, cfg, n, roots, root_off, root_lens):
    which = rng.integers(0, cfg.n_roots, size=n)
    L = cfg.length(rng, n).astype(np.int64)
    Lr = root_lens[which]
    take = np.minimum(L, Lr)
    start = (rng.random(n) * (Lr - take + 1)).astype(np.int64)
    left = (rng.random(n) * (L - take + 1)).astype(np.int64)
    off = np.zeros(n + 1, np.int64)
    np.cumsum(L, out=off[1:])
    T = int(off[-1])
    # base sequences: background, with the root window laid over it
    base = _background_draw(rng, T)
    k = np.repeat(np.arange(n, dtype=np.int32), L)
    q = np.arange(T, dtype=np.int64) - off[k]
    inroot = (q >= left[k]) & (q < left[k] + take[k])
    idx = np.nonzero(inroot)[0]
    kk = k[idx]
    base[idx] = roots[root_off[which[kk]] + start[kk] + (q[idx] - left[kk])]
    del q, inroot, idx, kk
    # substitutions: redraw from the background, conditioned on differing
    hit = np.nonzero(rng.random(T) < cfg.p_sub)[0]
    new = _background_draw(rng, len(hit))
    same = new == base[hit]
    while same.any():
        new[same] = _background_draw(rng, int(same.sum()))
        same = new == base[hit]
    base[hit] = new
    del hit, new, same
    # indels: deletions remove the union of their intervals (clipped at the
    # sequence end); an insertion goes before its position if that survives
    ev = np.nonzero(rng.random(T) < cfg.p_indel)[0]
    is_ins = rng.random(len(ev)) < 0.5
    elen = rng.geometric(0.5, size=len(ev)).astype(np.int64)
    dpos = ev[~is_ins]
    dend = np.minimum(dpos + elen[~is_ins], off[k[dpos].astype(np.int64) + 1])
    diff = np.bincount(dpos, minlength=T + 1)[:T + 1] - np.bincount(dend, minlength=T + 1)[:T + 1]
    keep = np.cumsum(diff[:T]) == 0
    insl = np.zeros(T, np.int64)
    ipos = ev[is_ins]
    ok = keep[ipos]
    insl[ipos[ok]] = elen[is_ins][ok]
    out_end = np.cumsum(keep.astype(np.int64) + insl)
    out = _background_draw(rng, int(out_end[-1]) if T else 0)
    kept = np.nonzero(keep)[0]
    out[out_end[kept] - 1] = base[kept]
    new_off = np.zeros(n + 1, np.int64)
    ends = off[1:] - 1
    new_off[1:] = np.where(L > 0, out_end[np.maximum(ends, 0)] if T else 0, 0)
    new_off[1:] = np.maximum.accumulate(new_off[1:])   # empty sequences keep the offset
    return out, new_off


def generate(cfg: FamilyConfig | str, n_seqs: int | None = None, seed: int | None = None) -> SeqSet:
    """Deterministic family-structured protein set (vectorised, in chunks).

    R roots are drawn from the BLOSUM62 background.  Each sequence picks a root
    uniformly and a target length L from the config's length law; it takes a
    uniform window of the root, or the whole root padded on both ends (random
    split) with background residues when L exceeds the root.  Every residue is
    then substituted with probability p_sub (redrawn from the background,
    conditioned on being different).  Finally indels start at each position
    with probability p_indel, half insertions and half deletions, of
    geometric(0.5) length: deletions remove the union of their intervals
    (clipped at the sequence end); an insertion places its residues before its
    position when that position survives.  Chunks of 65,536 sequences draw
    from their own seed streams.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    n_seqs = cfg.n_seqs if n_seqs is None else n_seqs
    ss = np.random.SeedSequence(cfg.seed if seed is None else seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    root_lens = cfg.length(rng, cfg.n_roots).astype(np.int64)
    roots = _background_draw(rng, int(root_lens.sum()))
    root_off = np.zeros(cfg.n_roots + 1, np.int64)
    np.cumsum(root_lens, out=root_off[1:])
    nchunks = max(1, (n_seqs + _CHUNK - 1) // _CHUNK)
    kids = ss.spawn(nchunks)

    def chunk(c):
        n = min(_CHUNK, n_seqs - c * _CHUNK)
        return _generate_chunk(np.random.Generator(np.random.PCG64(kids[c])), cfg, n, roots, root_off, root_lens)

    # chunks draw from their own seed streams, so they are generated in
    # parallel (numpy releases the GIL) and concatenated in order
    workers = max(1, min(nchunks, 8, os.cpu_count() or 1))
    if workers > 1:
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            results = list(ex.map(chunk, range(nchunks)))
    else:
        results = [chunk(c) for c in range(nchunks)]
    parts, offs, base = [], [np.zeros(1, np.int64)], 0
    for out, off in results:
        parts.append(out)
        offs.append(off[1:] + base)
        base += int(off[-1])
    res = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return SeqSet(res.astype(np.uint8), np.concatenate(offs))


def random_set(rng: np.random.Generator, n_seqs: int, lo: int, hi: int,
               alphabet: int = N_STANDARD) -> SeqSet:
    """Unrelated iid sequences with uniform lengths (edge-case tests)."""
    lens = rng.integers(lo, hi + 1, size=n_seqs)
    return SeqSet.from_list([rng.integers(0, alphabet, size=int(L)).astype(np.uint8) for L in lens])


# ---------------------------------------------------------------------------
# Nucleotide sets (the trie section's workload: similar genomes)
# ---------------------------------------------------------------------------
NUC_ALPHABET = "ACGTN"            # codes 0..4; N is never part of an anchor
# BLASTN-style scores (the paper names none): +2 match, -3 mismatch, -1 for
# any pair with N; gaps W_k = 5 + 2k
NUC_MATRIX = np.array([[2 if (a == b and a < 4) else (-1 if (a == 4 or b == 4) else -3) for b in range(5)]
                       for a in range(5)], dtype=np.int8)
NUC_MATRIX.setflags(write=False)
NUC_GAP_OPEN = 5
NUC_GAP_EXTEND = 2
NUC_K = 16                        # center segment length of the trie


@dataclasses.dataclass(frozen=True)
class DnaConfig:
    name: str
    n_seqs: int
    root_len: int
    p_sub: float
    p_indel: float
    p_n: float
    seed: int


DNA_CONFIGS = {
    # 672 human mitochondrial genomes (Table 1: lengths 16,556-16,579) and the
    # 100x replication; stand-ins: one random root, low divergence
    "dna672": DnaConfig("dna672", 672, 16569, 0.003, 0.0002, 0.0, SEED_BASE + 10),
    "dna67k": DnaConfig("dna67k", 67_200, 16569, 0.003, 0.0002, 0.0, SEED_BASE + 11),
    # small, more divergent set with a few N codes (tests)
    "dna_small": DnaConfig("dna_small", 48, 1500, 0.02, 0.004, 0.001, SEED_BASE + 12),
}


def generate_dna(cfg: DnaConfig | str, n_seqs: int | None = None, seed: int | None = None) -> SeqSet:
    """Similar nucleotide sequences: one uniform ACGT root; each sequence
    copies it with substitutions (probability p_sub, to a different base),
    then indels starting at each position with probability p_indel (half
    insertions of uniform bases before the position, half deletions),
    geometric(0.5) lengths, then N codes at rate p_n.  Sequence 0 is a copy
    like the others (it becomes the center)."""
    if isinstance(cfg, str):
        cfg = DNA_CONFIGS[cfg]
    n_seqs = cfg.n_seqs if n_seqs is None else n_seqs
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(cfg.seed if seed is None else seed)))
    root = rng.integers(0, 4, cfg.root_len).astype(np.uint8)
    L = cfg.root_len
    seqs = []
    for _ in range(n_seqs):
        b = root.copy()
        hit = np.nonzero(rng.random(L) < cfg.p_sub)[0]
        b[hit] = (b[hit] + rng.integers(1, 4, len(hit))) % 4
        ev = np.nonzero(rng.random(L) < cfg.p_indel)[0]
        is_ins = rng.random(len(ev)) < 0.5
        elen = rng.geometric(0.5, size=len(ev))
        keep = np.ones(L, bool)
        for pos, ln in zip(ev[~is_ins], elen[~is_ins]):
            keep[pos:pos + ln] = False
        parts, last = [], 0
        for pos, ln in zip(ev[is_ins], elen[is_ins]):
            parts.append(b[last:pos][keep[last:pos]])
            if keep[pos]:
                parts.append(rng.integers(0, 4, int(ln)).astype(np.uint8))
            last = pos
        parts.append(b[last:][keep[last:]])
        x = np.concatenate(parts).astype(np.uint8)
        if cfg.p_n > 0:
            x[rng.random(len(x)) < cfg.p_n] = 4
        seqs.append(x)
    return SeqSet.from_list(seqs)


def tree_permutation(n: int, seed: int | None = None) -> np.ndarray:
    """The random draw of the tree stage: a seeded permutation of 0..n-1 (its
    first ceil(n / 10) rows are the sample)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + 20 if seed is None else seed)))
    return rng.permutation(n).astype(np.int32)
