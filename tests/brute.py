"""Brute-force local alignment enumerator for tiny inputs (test-only).

Enumerates every local alignment of every pair of substrings of c and s as a
path of columns M (c_i with s_j), I (s_j against a gap) and D (c_i against a
gap).  Its score is the sum of S over M columns minus W_k = go + ge*k for
every maximal run of k I columns or k D columns.  An optimal local alignment
can always be taken to start and end with an M column (trimming a leading or
trailing gap run only raises the score), so only those are enumerated; the
best local score is max(0, best path).

This shares nothing with the oracle: it never builds a DP matrix.
"""
from __future__ import annotations

from typing import List, Tuple


def enumerate_alignments(S, go: int, ge: int, c, s):
    """Yield (score, i0, j0, i1, j1, ops) for every M-bounded local alignment."""
    m, n = len(c), len(s)
    out = []

    def rec(i, j, score, ops, last, run, i0, j0):
        # (i, j) = residues consumed so far (0-based next positions)
        if last == "M":
            out.append((score, i0, j0, i, j, "".join(ops)))
        if i < m and j < n:
            ops.append("M")
            rec(i + 1, j + 1, score + int(S[c[i]][s[j]]), ops, "M", 0, i0, j0)
            ops.pop()
        if j < n:
            cost = ge if last == "I" else go + ge
            ops.append("I")
            rec(i, j + 1, score - cost, ops, "I", run + 1, i0, j0)
            ops.pop()
        if i < m:
            cost = ge if last == "D" else go + ge
            ops.append("D")
            rec(i + 1, j, score - cost, ops, "D", run + 1, i0, j0)
            ops.pop()

    for a in range(m):
        for b in range(n):
            rec(a + 1, b + 1, int(S[c[a]][s[b]]), ["M"], "M", 0, a, b)
    return out


def best_local(S, go: int, ge: int, c, s) -> Tuple[int, List[tuple]]:
    """(best score, all optimal alignments) with best >= 0."""
    allal = enumerate_alignments(S, go, ge, c, s)
    best = max([0] + [a[0] for a in allal])
    return best, [a for a in allal if a[0] == best and best > 0]


def rescore(S, go: int, ge: int, c, s, i0: int, j0: int, ops: str) -> int:
    """Score of an alignment given as a start cell and M/I/D ops."""
    i, j, tot, prev = i0, j0, 0, ""
    for op in ops:
        if op == "M":
            tot += int(S[c[i]][s[j]])
            i += 1
            j += 1
        elif op == "I":
            tot -= ge if prev == "I" else go + ge
            j += 1
        else:
            tot -= ge if prev == "D" else go + ge
            i += 1
        prev = op
    return tot
