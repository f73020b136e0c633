"""Pins of the oracle's minimum spanning forest (no GPU).

The forest is over the stored edges taken as undirected, with edge keys
(weight, edge index) so that it is unique.  Pinned by exhaustive search on
tiny graphs, by scipy's minimum spanning tree weight, by the certificate
(forest + spanning + cycle property) with planted mistakes it must reject,
and by closed forms.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import minimum_spanning_tree

import oracle
from helpers import path_graph, random_graph, star
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.timeout(300)


def keys(g):
    return g.w.astype(np.int64) * (1 << 32) + np.arange(g.m, dtype=np.int64)


def scipy_msf_weight(g):
    """Weight of the minimum spanning forest by scipy: the undirected simple
    graph keeps the lightest of parallel edges; self-loops dropped."""
    src, dst, w = g.edge_list()
    keep = src != dst
    a, b, w = np.minimum(src, dst)[keep], np.maximum(src, dst)[keep], w[keep]
    best = {}
    for x, y, z in zip(a.tolist(), b.tolist(), w.tolist()):
        if (x, y) not in best or z < best[(x, y)]:
            best[(x, y)] = z
    if not best:
        return 0
    xs, ys = zip(*best.keys())
    mat = sp.csr_matrix((list(best.values()), (xs, ys)), shape=(g.n, g.n))
    return int(round(minimum_spanning_tree(mat).sum()))


def forest_path(n, src, dst, chosen, a, b):
    """Edge indices on the path a..b of the forest (breadth-first search)."""
    adj = [[] for _ in range(n)]
    for e in chosen:
        adj[src[e]].append((dst[e], e))
        adj[dst[e]].append((src[e], e))
    prev = {a: None}
    queue = [a]
    for u in queue:
        for v, e in adj[u]:
            if v not in prev:
                prev[v] = (u, e)
                queue.append(v)
    assert b in prev
    out, x = [], b
    while prev[x] is not None:
        x, e = prev[x]
        out.append(e)
    return out


def test_matches_exhaustive_search_on_tiny_graphs():
    rng = np.random.default_rng(41)
    for i in range(400):
        n = int(rng.integers(1, 9))
        m = int(rng.integers(0, 15))
        # narrow weights: many ties, settled by the edge index
        g = random_graph(rng, n, m, 0 if i % 3 == 0 else 1, int(rng.integers(1, 5)))
        sel, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
        want = oracle.msf_brute(g.n, g.row_ptr, g.col, g.w)
        np.testing.assert_array_equal(sel, want, err_msg=f"case {i}")
        assert total == int(g.w[sel == 1].sum())


def test_weight_matches_scipy():
    rng = np.random.default_rng(42)
    for i in range(120):
        n = int(rng.integers(1, 300))
        g = random_graph(rng, n, int(rng.integers(0, 5 * n + 1)), 1, int(rng.integers(1, 1000)))
        _, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
        assert total == scipy_msf_weight(g), f"case {i}"


def test_certificate_accepts_the_forest_and_rejects_planted_mistakes():
    rng = np.random.default_rng(43)
    graphs = [random_graph(rng, 2000, 8000, 1, 50), random_graph(rng, 500, 400, 1, 3),
              gen.workload("rmat12"), gen.workload("grid96")]
    for g in graphs:
        sel, _ = oracle.msf(g.n, g.row_ptr, g.col, g.w)
        assert oracle.check_msf(g.n, g.row_ptr, g.col, g.w, sel) == 0, g.name
        src, dst, _ = g.edge_list()
        chosen = np.flatnonzero(sel)
        left = np.flatnonzero((sel == 0) & (src != dst))
        # a forest edge dropped: no longer spanning
        bad = sel.copy()
        bad[chosen[len(chosen) // 2]] = 0
        assert oracle.check_msf(g.n, g.row_ptr, g.col, g.w, bad) == 2, g.name
        # an extra edge: a cycle
        if len(left):
            bad = sel.copy()
            bad[left[0]] = 1
            assert oracle.check_msf(g.n, g.row_ptr, g.col, g.w, bad) == 1, g.name
        # a self-loop selected
        loops = np.flatnonzero(src == dst)
        if len(loops):
            bad = sel.copy()
            bad[loops[0]] = 1
            assert oracle.check_msf(g.n, g.row_ptr, g.col, g.w, bad) == 1, g.name
        # a forest edge swapped for a heavier edge that reconnects its ends:
        # still a spanning forest, but the cycle property fails
        if len(left):
            f = left[len(left) // 2]
            path = forest_path(g.n, src, dst, chosen, src[f], dst[f])
            e = max(path, key=lambda x: keys(g)[x])
            assert keys(g)[e] < keys(g)[f]
            bad = sel.copy()
            bad[e], bad[f] = 0, 1
            assert oracle.check_msf(g.n, g.row_ptr, g.col, g.w, bad) == 3, g.name


def test_closed_forms():
    # a path is its own forest
    g = path_graph(50, np.arange(1, 50))
    sel, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
    assert sel.all() and total == sum(range(1, 50))
    # a cycle with distinct weights drops its heaviest edge
    n = 40
    rng = np.random.default_rng(7)
    w = rng.permutation(np.arange(1, n + 1)).astype(np.int32)
    src = np.arange(n, dtype=np.int32)
    g = gen.from_edges(n, src, (src + 1) % n, w)
    sel, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
    assert sel.sum() == n - 1 and total == w.sum() - n and g.w[sel == 0][0] == n
    # parallel edges of equal weight: the lowest index wins
    g = star(5, [[3, 3, 3]] * 5)
    sel, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
    assert total == 15 and list(np.flatnonzero(sel)) == [0, 3, 6, 9, 12]
    # no edges; one vertex; self-loops only
    for g in (gen.from_edges(7, [], [], []), gen.from_edges(1, [0, 0], [0, 0], [1, 2])):
        sel, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
        assert sel.sum() == 0 and total == 0
    # unit-weight grid without shortcuts: connected, n - 1 edges of weight 1
    g = gen.grid(30, 20, 0, 8, 1, 1)
    sel, total = oracle.msf(g.n, g.row_ptr, g.col, g.w)
    assert sel.sum() == g.n - 1 and total == g.n - 1
    # disjoint blocks: n - (number of blocks) edges
    rng = np.random.default_rng(8)
    s, d = [], []
    for b in range(6):
        base = 10 * b
        s += [base + i for i in range(9)]
        d += [base + i + 1 for i in range(9)]
        s += list(base + rng.integers(0, 10, 20))
        d += list(base + rng.integers(0, 10, 20))
    g = gen.from_edges(60, s, d, rng.integers(1, 9, len(s)))
    sel, _ = oracle.msf(g.n, g.row_ptr, g.col, g.w)
    assert sel.sum() == 60 - 6
