"""The phylogeny oracle (NJ section, Fig. 4) pinned against what does not
come from it: hand-counted p-distances, neighbour joining's recovery of every
additive tree metric (with its branch lengths), a hand-derived tie case,
hand-built clusterings, and the merged tree's structure."""
import numpy as np
import pytest

import oracle

G = oracle.GAP


def _rows(*txt):
    """MSA rows from strings over 'ACGT-' (codes 0..3, gap byte)."""
    code = {"A": 0, "C": 1, "G": 2, "T": 3, "-": G}
    return np.array([[code[ch] for ch in t] for t in txt], np.uint8)


def test_pdist_hand_counts():
    m = _rows("ACGT-A", "ACTT-C", "--GTAA", "------")
    mism, comp = oracle.pdist_counts(m)
    # rows 0, 1: columns 0-3 and 5 compared (4 is gap in both), mismatches at 2 and 5
    assert (mism[0, 1], comp[0, 1]) == (2, 5)
    # rows 0, 2: columns 2, 3, 5 compared (2 has G/G, 3 T/T, 5 A/A): no mismatch
    assert (mism[0, 2], comp[0, 2]) == (0, 3)
    # rows 1, 2: columns 2 (T/G), 3 (T/T), 5 (C/A)
    assert (mism[1, 2], comp[1, 2]) == (2, 3)
    # an all-gap row compares nothing: distance 1 by the reading
    assert comp[3].sum() == 0
    D = oracle.pdist(m)
    assert D[0, 1] == 2 / 5 and D[0, 2] == 0.0 and D[1, 2] == 2 / 3 and D[0, 3] == 1.0 and D[3, 3] == 1.0
    assert (D == D.T).all()


def _random_tree(rng, n, integral=True):
    """A random unrooted binary tree on n leaves: edges (u, v, length)."""
    # grow by inserting leaf t on a random edge
    edges = [(0, 1, 0)] if n >= 2 else []
    nxt = n
    for t in range(2, n):
        k = int(rng.integers(len(edges)))
        u, v, _ = edges.pop(k)
        w = nxt
        nxt += 1
        edges += [(u, w, 0), (w, v, 0), (w, t, 0)]
    out = []
    for (u, v, _) in edges:
        ln = float(rng.integers(1, 20)) if integral else float(rng.uniform(0.05, 2.0))
        out.append((u, v, ln))
    return out, nxt


def _path_lengths(edges, nnodes, leaves):
    adj = [[] for _ in range(nnodes)]
    for u, v, ln in edges:
        adj[u].append((v, ln))
        adj[v].append((u, ln))
    D = np.zeros((leaves, leaves))
    for s in range(leaves):
        dist = {s: 0.0}
        stack = [s]
        while stack:
            x = stack.pop()
            for y, ln in adj[x]:
                if y not in dist:
                    dist[y] = dist[x] + ln
                    stack.append(y)
        for t in range(leaves):
            D[s, t] = dist[t]
    return D


def _splits(parent, blen, n):
    """Leaf set below each non-root edge (as the smaller side, canonical) with its length."""
    nn = len(parent)
    below = [set() for _ in range(nn)]
    for v in range(n):
        x = v
        while x >= 0:
            below[x].add(v)
            x = parent[x]
    allv = frozenset(range(n))
    out = {}
    for v in range(nn):
        if parent[v] < 0:
            continue
        s = frozenset(below[v])
        c = min(s, allv - s, key=lambda z: (len(z), sorted(z)))
        out[c] = out.get(c, 0.0) + blen[v]   # edges through a degree-2 root add up
    return {k: v for k, v in out.items() if 0 < len(k) < n}


def _tree_metric(parent, blen, n):
    nn = len(parent)
    adj = [[] for _ in range(nn)]
    for v in range(nn):
        if parent[v] >= 0:
            adj[v].append((parent[v], blen[v]))
            adj[parent[v]].append((v, blen[v]))
    return _path_lengths([(v, parent[v], blen[v]) for v in range(nn) if parent[v] >= 0], nn, n)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 9, 17, 30])
def test_nj_recovers_additive_trees(n):
    """Neighbour joining is exact on tree metrics: same splits, same lengths."""
    rng = np.random.default_rng(100 + n)
    for rep in range(6):
        edges, nnodes = _random_tree(rng, n, integral=rep % 2 == 0)
        D = _path_lengths(edges, nnodes, n)
        parent, blen = oracle.nj(D)
        assert len(parent) == 2 * n - 2 and (parent == -1).sum() == 1
        # the tree metric of the answer is D
        assert np.allclose(_tree_metric(parent, blen, n), D, atol=1e-9)
        # and the splits with their lengths are the true tree's
        truth = {}
        below = {}
        # true splits from the generating tree
        adj = [[] for _ in range(nnodes)]
        for u, v, ln in edges:
            adj[u].append((v, ln))
            adj[v].append((u, ln))
        for u, v, ln in edges:
            seen = {u}
            side = set()
            stack = [v]
            seen.add(v)
            while stack:
                x = stack.pop()
                if x < n:
                    side.add(x)
                for y, _ in adj[x]:
                    if y not in seen:
                        seen.add(y)
                        stack.append(y)
            s = frozenset(side)
            c = min(s, frozenset(range(n)) - s, key=lambda z: (len(z), sorted(z)))
            if 0 < len(c) < n:
                truth[c] = truth.get(c, 0.0) + ln
        got = _splits(parent, blen, n)
        assert set(got) == set(truth)
        for k in truth:
            assert abs(got[k] - truth[k]) < 1e-9


def test_nj_hand_cases():
    # four taxa ((0:2, 1:3):3, (2:4, 3:4)): the first join is (0, 1)
    D = np.array([[0, 5, 9, 9], [5, 0, 10, 10], [9, 10, 0, 8], [9, 10, 8, 0]], float)
    parent, blen = oracle.nj(D)
    assert list(parent) == [4, 4, 5, 5, 5, -1]
    assert list(blen) == [2.0, 3.0, 4.0, 4.0, 3.0, 0.0]
    # all distances equal: every Q ties, the tie rule joins (0, 1) first (by
    # hand: r = 3d, Q = -4d everywhere; lengths d/2; then the centre of u, 2,
    # 3 gets u at 0 and the others at d/2)
    d = 3.0
    D = np.full((4, 4), d) - d * np.eye(4)
    parent, blen = oracle.nj(D)
    assert list(parent) == [4, 4, 5, 5, 5, -1]
    assert list(blen) == [d / 2, d / 2, d / 2, d / 2, 0.0, 0.0]
    # one, two and three leaves
    p, b = oracle.nj(np.zeros((1, 1)))
    assert list(p) == [-1]
    p, b = oracle.nj(np.array([[0, 4.0], [4.0, 0]]))
    assert list(p) == [2, 2, -1] and list(b) == [2.0, 2.0, 0.0]
    p, b = oracle.nj(np.array([[0, 3.0, 5.0], [3.0, 0, 6.0], [5.0, 6.0, 0]]))
    assert list(p) == [3, 3, 3, -1] and list(b) == [1.0, 2.0, 4.0, 0.0]


def _families(rng, fam_sizes, width=120, p=0.05):
    """Rows in families: each family mutates its own random root at rate p;
    roots differ at about 3/4 of the columns."""
    rows = []
    for s in fam_sizes:
        root = rng.integers(0, 4, width)
        for _ in range(s):
            r = root.copy()
            hit = rng.random(width) < p
            r[hit] = (r[hit] + rng.integers(1, 4, hit.sum())) % 4
            rows.append(r)
    return np.array(rows, np.uint8)


def _clusters(label, seed):
    return [sorted(np.nonzero(label == c)[0].tolist()) for c in range(len(seed))]


def test_clusters_hand_built():
    rng = np.random.default_rng(3)
    # 30 rows in three families of 10; N = 30 -> 3 seeds (one per family) and
    # clusters of at most 3 rows.  Each family's cluster (10 rows) gets one
    # new seed, its first row in permutation order, which takes every row:
    # no split, so the family is cut into runs of 3 in permutation order.
    m = _families(rng, [10, 10, 10])
    perm = np.array([4, 15, 27] + [x for x in range(30) if x not in (4, 15, 27)], np.int32)
    label, seed = oracle.nj_clusters(m, perm)
    assert list(seed) == [4, 2, 6, 9, 15, 12, 16, 19, 27, 22, 25, 29]
    assert _clusters(label, seed) == [[0, 1, 4], [2, 3, 5], [6, 7, 8], [9], [10, 11, 15], [12, 13, 14],
                                      [16, 17, 18], [19], [20, 21, 27], [22, 23, 24], [25, 26, 28], [29]]
    # a cluster of fewer than 3 rows is merged into the cluster of the
    # nearest seed, then the divide passes (clusters over ceil(22/10) = 3
    # rows) reseed from the rows in permutation order (0, 12, 14, 1, 2, ...)
    m3 = _families(rng, [12, 2, 8])    # N = 22 -> 3 seeds: rows 0 (A), 12 (B), 14 (C)
    perm3 = np.array([0, 12, 14] + [x for x in range(22) if x not in (0, 12, 14)], np.int32)
    label3, seed3 = oracle.nj_clusters(m3, perm3)
    D3 = oracle.pdist(m3)
    assert D3[12, 0] < D3[12, 14]   # B joins A: A+B (14 rows, seed 0), C (8 rows, seed 14)
    cl = _clusters(label3, seed3)
    # A+B is divided between rows 0 and 12 (the first two in permutation
    # order): B comes back out as its own cluster; C (one seed, 14, takes
    # all) is cut into runs 14-16, 17-19, 20-21; A keeps dividing (its first
    # rows in permutation order are 0, 1, 2, ...) until no part exceeds 3
    assert [12, 13] in cl and [14, 15, 16] in cl and [17, 18, 19] in cl and [20, 21] in cl
    a_parts = [c for c in cl if c[0] < 12]
    assert sorted(x for c in a_parts for x in c) == list(range(12))
    assert all(len(c) <= 3 for c in cl)
    # seeds come in cluster order, each labelled with its own cluster
    assert all(label3[s] == c for c, s in enumerate(seed3))


def test_clusters_properties():
    """On families with sub-families (where divisions split by nearness):
    every cluster is non-empty and at most ceil(N / 10) rows, each seed is in
    its own cluster, and the partition refines the first labelling (rows of
    different nearest sample rows never share a cluster, merges aside)."""
    rng = np.random.default_rng(12)
    m = np.concatenate([_families(rng, [20, 20], p=0.02), _families(rng, [25, 15, 20], p=0.02)])
    N = m.shape[0]
    S = (N + 9) // 10
    for rep in range(3):
        perm = rng.permutation(N).astype(np.int32)
        label, seed = oracle.nj_clusters(m, perm)
        cl = _clusters(label, seed)
        assert all(0 < len(c) <= S for c in cl)
        assert all(label[s] == c for c, s in enumerate(seed))
        D = oracle.pdist(m)
        first = np.argmin(D[:, perm[:S]], axis=1)   # nearest sample row, ties to the earlier
        sizes = np.bincount(first, minlength=S)
        if (sizes[sizes > 0] >= 3).all():           # no merge happened: a refinement
            for c in cl:
                assert len(set(first[c].tolist())) == 1


def test_nj_tree_small_is_plain_nj():
    """N <= 10: clusters hold at most ceil(N / 10) = 1 row, so every row is a
    cluster, in permutation order (the one sample row takes every row, which
    is then cut into runs of one); the tree is neighbour joining over the rows
    taken in permutation order, its leaves mapped back to the rows."""
    rng = np.random.default_rng(8)
    for n in (1, 2, 3, 5, 10):
        m = _families(rng, [n])
        perm = rng.permutation(n).astype(np.int32)
        p, b = oracle.nj_tree(m, perm)
        D = oracle.pdist(m)
        p2, b2 = oracle.nj(D[np.ix_(perm, perm)] * (1 - np.eye(n)))
        node = lambda v: int(perm[v]) if v < n else v
        want_p = np.zeros(len(p2), np.int32)
        want_b = np.zeros(len(p2))
        for v in range(len(p2)):
            want_p[node(v)] = -1 if p2[v] < 0 else node(p2[v])
            want_b[node(v)] = b2[v]
        assert (p == want_p).all() and (b == want_b).all()


def test_nj_tree_families_are_clades():
    """Well separated families come out as clades of the merged tree, and the
    result is one tree over all rows."""
    rng = np.random.default_rng(11)
    sizes = [12, 9, 15, 7, 11]
    m = _families(rng, sizes, width=200, p=0.03)
    N = m.shape[0]
    perm = rng.permutation(N).astype(np.int32)
    parent, blen = oracle.nj_tree(m, perm)
    assert (parent == -1).sum() == 1
    # every node reaches the root
    for v in range(len(parent)):
        x, steps = v, 0
        while parent[x] >= 0:
            x = parent[x]
            steps += 1
            assert steps <= len(parent)
    # clades: for each family, some edge splits it off exactly
    sp = _splits(parent, blen, N)
    off = 0
    for s in sizes:
        fam = frozenset(range(off, off + s))
        c = min(fam, frozenset(range(N)) - fam, key=lambda z: (len(z), sorted(z)))
        assert c in sp, f"family at {off} is not a clade"
        off += s
