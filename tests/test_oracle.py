"""Pins for the CPU oracle (no GPU).

The oracle's routines are checked against things other than themselves:
scipy.sparse.csgraph (an independent library), closed forms, hand-derived
fixtures, brute force on tiny inputs, and certificates that are themselves
pinned by planted mistakes in oracle outputs.
"""
import numpy as np
import pytest
from scipy.sparse import csgraph, csr_matrix

import oracle
from paper_1903_01665_amd import gen
from helpers import (INF, complete_digraph, golden_files, path_graph, random_graph,
                     read_golden, star)


def scipy_sssp(g, source, unit=False):
    """Shortest paths by scipy's Dijkstra over a dense matrix holding the
    lightest parallel edge (self-loops dropped); inf = no edge."""
    D = np.full((g.n, g.n), np.inf)
    src, dst, w = g.edge_list()
    for u, v, x in zip(src, dst, w if not unit else np.ones(len(src))):
        if u != v and x < D[u, v]:
            D[u, v] = x
    G = csgraph.csgraph_from_dense(D, null_value=np.inf)
    d = csgraph.dijkstra(G, directed=True, indices=source)
    out = np.where(np.isinf(d), INF, d).astype(np.int64)
    return np.minimum(out, INF).astype(np.int32)


def scipy_cc(g):
    src, dst, _ = g.edge_list()
    A = csr_matrix((np.ones(len(src)), (src, dst)), shape=(g.n, g.n))
    _, comp = csgraph.connected_components(A, directed=True, connection="weak")
    first = {}
    for v, c in enumerate(comp):
        first.setdefault(c, v)
    return np.array([first[c] for c in comp], np.int32)


def _rand_cases(count, seed, nmax=40, wlo=1, whi=9):
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(rng.integers(1, nmax + 1))
        m = int(rng.integers(0, 4 * n + 1))
        g = random_graph(rng, n, m, wlo, whi, name=f"r{i}")
        s = int(rng.integers(0, n))
        yield g, s


# --------------------------------------------------------------- SSSP -----

@pytest.mark.parametrize("wlo,whi", [(1, 9), (0, 3), (1, 1000)])
def test_sssp_matches_scipy_and_brute_force(wlo, whi):
    for g, s in _rand_cases(150, 1000 + whi, wlo=wlo, whi=whi):
        d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        np.testing.assert_array_equal(d, scipy_sssp(g, s), err_msg=g.name)
        np.testing.assert_array_equal(d, oracle.sssp_floyd_warshall(g.n, g.row_ptr, g.col, g.w, s))
        np.testing.assert_array_equal(d, oracle.sssp_bellman_ford(g.n, g.row_ptr, g.col, g.w, s))
        assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, d) == 0


def test_sssp_direction_matters():
    # 0 -> 1 only: from 1 nothing is reachable (a transposed operand would
    # make 0 reachable from 1)
    g = gen.from_edges(2, [0], [1], [5])
    np.testing.assert_array_equal(oracle.sssp(2, g.row_ptr, g.col, g.w, 0), [0, 5])
    np.testing.assert_array_equal(oracle.sssp(2, g.row_ptr, g.col, g.w, 1), [INF, 0])


def test_sssp_path_prefix_sums():
    w = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.int32)
    g = path_graph(9, w)
    want = np.concatenate([[0], np.cumsum(w)]).astype(np.int32)
    np.testing.assert_array_equal(oracle.sssp(9, g.row_ptr, g.col, g.w, 0), want)
    # from the middle: everything before is unreachable
    d = oracle.sssp(9, g.row_ptr, g.col, g.w, 4)
    np.testing.assert_array_equal(d[:4], [INF] * 4)
    np.testing.assert_array_equal(d[4:], np.concatenate([[0], np.cumsum(w[4:])]))


def test_sssp_star_takes_lightest_parallel_edge():
    ws = [[5, 2, 9], [7], [4, 4], [100, 1]]
    g = star(4, ws)
    np.testing.assert_array_equal(oracle.sssp(5, g.row_ptr, g.col, g.w, 0),
                                  [0] + [min(x) for x in ws])


def test_sssp_unit_weight_grid_is_manhattan():
    W, H = 13, 9
    g = gen.grid(W, H, 0, 8, 1, 1, stream=77)
    for s in [0, W * H - 1, 4 * W + 6]:
        d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        sx, sy = s % W, s // W
        x, y = np.arange(g.n) % W, np.arange(g.n) // W
        np.testing.assert_array_equal(d, np.abs(x - sx) + np.abs(y - sy))


def test_sssp_no_edges_and_single_vertex():
    g = gen.from_edges(5, [], [], [])
    np.testing.assert_array_equal(oracle.sssp(5, g.row_ptr, g.col, g.w, 2), [INF, INF, 0, INF, INF])
    g1 = gen.from_edges(1, [0], [0], [3])
    np.testing.assert_array_equal(oracle.sssp(1, g1.row_ptr, g1.col, g1.w, 0), [0])


def test_sssp_clamps_at_inf():
    # a path whose length passes 2^31-1 is reported as INF (output is
    # min(distance, INF)); a shorter one just below stays exact
    big = 2**30
    g = gen.from_edges(4, [0, 1, 2], [1, 2, 3], [big, big - 1, 1])
    np.testing.assert_array_equal(oracle.sssp(4, g.row_ptr, g.col, g.w, 0),
                                  [0, big, 2 * big - 1, INF])


def test_sssp_clamp_against_brute_force_with_huge_weights():
    # weights near 2^30 and 2^31: many shortest paths pass INF.  Floyd-
    # Warshall and Bellman-Ford in int64 (clamped only when written out)
    # and scipy's float Dijkstra (exact below 2^53) agree with the heap
    # Dijkstra on which vertices stay finite and on every finite value
    rng = np.random.default_rng(2**31 - 1)
    for i in range(40):
        n = int(rng.integers(2, 60))
        m = int(rng.integers(0, 5 * n + 1))
        lo = [1, 2**29, INF - 50][i % 3]
        g = random_graph(rng, n, m, lo, INF, name=f"huge{i}")
        s = int(rng.integers(0, n))
        d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        np.testing.assert_array_equal(d, oracle.sssp_floyd_warshall(g.n, g.row_ptr, g.col, g.w, s))
        np.testing.assert_array_equal(d, oracle.sssp_bellman_ford(g.n, g.row_ptr, g.col, g.w, s))
        ref = csgraph.dijkstra(_scipy_min_matrix(g), directed=True, indices=s)
        ref = np.where(np.isinf(ref) | (ref >= INF), INF, ref).astype(np.int64)
        np.testing.assert_array_equal(d.astype(np.int64), ref)
        clamped = (oracle.bfs(g.n, g.row_ptr, g.col, s) != INF) & (d == INF)
        if not clamped.any():
            assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, d) == 0


def _scipy_min_matrix(g):
    # parallel edges keep their smallest weight (csr_matrix would sum them)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    best = {}
    for u, v, w in zip(src.tolist(), g.col.tolist(), g.w.tolist()):
        if (u, v) not in best or w < best[(u, v)]:
            best[(u, v)] = w
    if not best:
        return csr_matrix((g.n, g.n))
    keys = list(best)
    # a stored zero weight would read as "no edge": add a tiny offset and
    # round it away (all other weights are integers >= 1)
    vals = [best[k] if best[k] > 0 else 1e-9 for k in keys]
    return csr_matrix((vals, ([k[0] for k in keys], [k[1] for k in keys])), shape=(g.n, g.n))


def test_sssp_rejects_bad_input():
    g = gen.from_edges(3, [0, 1], [1, 2], [1, 1])
    with pytest.raises(ValueError):
        oracle.sssp(3, g.row_ptr, g.col, g.w, 3)
    with pytest.raises(ValueError):
        oracle.sssp(3, g.row_ptr, g.col, np.array([1, -1], np.int32), 0)
    with pytest.raises(ValueError):
        oracle.sssp(3, g.row_ptr, np.array([1, 5], np.int32), g.w, 0)


# ---------------------------------------------------------------- BFS -----

def test_bfs_matches_scipy_and_unit_sssp():
    for g, s in _rand_cases(200, 2024):
        d = oracle.bfs(g.n, g.row_ptr, g.col, s)
        np.testing.assert_array_equal(d, scipy_sssp(g, s, unit=True), err_msg=g.name)
        ones = np.ones(max(g.m, 1), np.int32)[: g.m]
        np.testing.assert_array_equal(d, oracle.sssp(g.n, g.row_ptr, g.col, ones, s))
        assert oracle.check_bfs(g.n, g.row_ptr, g.col, s, d) == 0


def test_bfs_complete_digraph_and_grid():
    g = complete_digraph(9)
    d = oracle.bfs(9, g.row_ptr, g.col, 3)
    np.testing.assert_array_equal(d, [1, 1, 1, 0, 1, 1, 1, 1, 1])
    W, H = 17, 6
    g = gen.grid(W, H, 0, 8, 1, 1000, stream=78)
    d = oracle.bfs(g.n, g.row_ptr, g.col, 0)
    np.testing.assert_array_equal(d, np.arange(g.n) % W + np.arange(g.n) // W)


def test_bfs_path_levels():
    g = path_graph(12, np.full(11, 7))
    np.testing.assert_array_equal(oracle.bfs(12, g.row_ptr, g.col, 0), np.arange(12))


# ----------------------------------------------------------------- CC -----

def test_cc_matches_scipy_and_warshall():
    for g, _ in _rand_cases(200, 7, nmax=60):
        lab = oracle.cc(g.n, g.row_ptr, g.col)
        np.testing.assert_array_equal(lab, scipy_cc(g), err_msg=g.name)
        np.testing.assert_array_equal(lab, oracle.cc_warshall(g.n, g.row_ptr, g.col))
        assert oracle.check_cc(g.n, g.row_ptr, g.col, lab) == 0


def test_cc_closed_forms():
    g = gen.from_edges(6, [], [], [])
    np.testing.assert_array_equal(oracle.cc(6, g.row_ptr, g.col), np.arange(6))
    W = 11
    g = gen.grid(W, W, 0, 8, 1, 9, stream=79)
    np.testing.assert_array_equal(oracle.cc(g.n, g.row_ptr, g.col), np.zeros(g.n))
    # disjoint blocks, each a directed cycle entered from its largest id
    blocks = [[9, 4, 7], [2, 8], [0, 5, 6, 1], [3]]
    src, dst = [], []
    for b in blocks:
        for i in range(len(b)):
            if len(b) > 1:
                src.append(b[i])
                dst.append(b[(i + 1) % len(b)])
    g = gen.from_edges(10, src, dst, [1] * len(src))
    want = np.zeros(10, np.int32)
    for b in blocks:
        want[b] = min(b)
    np.testing.assert_array_equal(oracle.cc(10, g.row_ptr, g.col), want)


# ------------------------------------------------------------- golden -----

@pytest.mark.parametrize("fname", golden_files())
def test_golden_fixtures(fname):
    g, s, want = read_golden(fname)
    np.testing.assert_array_equal(oracle.sssp(g.n, g.row_ptr, g.col, g.w, s), want["sssp"])
    np.testing.assert_array_equal(oracle.bfs(g.n, g.row_ptr, g.col, s), want["bfs"])
    np.testing.assert_array_equal(oracle.cc(g.n, g.row_ptr, g.col), want["cc"])


# ------------------------------------------------------- certificates -----

def test_certificates_reject_planted_mistakes():
    rng = np.random.default_rng(99)
    caught = {"sssp": 0, "bfs": 0, "cc": 0}
    for g, s in _rand_cases(150, 4242, nmax=30):
        d = oracle.sssp(g.n, g.row_ptr, g.col, g.w, s)
        b = oracle.bfs(g.n, g.row_ptr, g.col, s)
        lab = oracle.cc(g.n, g.row_ptr, g.col)
        v = int(rng.integers(0, g.n))
        # distances: off by one either way, or reach flipped
        for bad in (d[v] + 1 if d[v] < INF else 5, d[v] - 1 if d[v] > 0 else INF):
            dd = d.copy()
            dd[v] = bad
            if not np.array_equal(dd, d):
                assert oracle.check_sssp(g.n, g.row_ptr, g.col, g.w, s, dd) != 0
                caught["sssp"] += 1
        for bad in (b[v] + 1 if b[v] < INF else 3, INF):
            bb = b.copy()
            bb[v] = bad
            if not np.array_equal(bb, b):
                assert oracle.check_bfs(g.n, g.row_ptr, g.col, s, bb) != 0
                caught["bfs"] += 1
        # labels: any other label for one vertex is wrong
        ll = lab.copy()
        ll[v] = (lab[v] + 1) % g.n if g.n > 1 else lab[v]
        if not np.array_equal(ll, lab):
            assert oracle.check_cc(g.n, g.row_ptr, g.col, ll) != 0
            caught["cc"] += 1
    assert min(caught.values()) > 50


def test_certificate_rejects_zero_cycle_fake():
    # dist values that are feasible and locally tight on a zero-weight cycle
    # but not connected to the source by tight edges
    g = gen.from_edges(3, [1, 2], [2, 1], [0, 0])
    fake = np.array([0, 5, 5], np.int32)
    assert oracle.check_sssp(3, g.row_ptr, g.col, g.w, 0, fake) != 0
    assert oracle.check_sssp(3, g.row_ptr, g.col, g.w, 0, np.array([0, INF, INF], np.int32)) == 0


def test_certificate_rejects_merged_components():
    g = gen.from_edges(4, [0, 2], [1, 3], [1, 1])
    assert oracle.check_cc(4, g.row_ptr, g.col, np.array([0, 0, 2, 2], np.int32)) == 0
    assert oracle.check_cc(4, g.row_ptr, g.col, np.array([0, 0, 0, 0], np.int32)) != 0
    assert oracle.check_cc(4, g.row_ptr, g.col, np.array([1, 1, 2, 2], np.int32)) != 0
