"""Input generator checks (no GPU): shapes, distributions, determinism."""
import os
import subprocess
import sys

import numpy as np

from paper_1903_01665_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_uniform_shape_and_ranges():
    g = gen.uniform(1000, 20000, 1, 100, stream=3)
    assert g.n == 1000 and g.m == 20000 and len(g.row_ptr) == 1001
    assert np.all(np.diff(g.row_ptr) >= 0)
    src, dst, w = g.edge_list()
    assert np.all(src != dst)  # self-loops are redrawn
    assert w.min() >= 1 and w.max() <= 100
    assert abs(w.mean() - 50.5) < 1.5
    # endpoints roughly uniform
    deg = g.degrees()
    assert abs(deg.mean() - 20) < 1e-9 and deg.std() < 8


def test_deterministic_and_stream_separated():
    a = gen.uniform(500, 4000, 1, 100, stream=9)
    b = gen.uniform(500, 4000, 1, 100, stream=9)
    c = gen.uniform(500, 4000, 1, 100, stream=10)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)
    assert not np.array_equal(a.col, c.col)


def test_thread_count_does_not_change_output():
    code = ("import sys; sys.path.insert(0, %r); from paper_1903_01665_amd import gen; "
            "g = gen.rmat(14, 16 << 14, stream=5); print(gen.fnv1a(g.col), gen.fnv1a(g.w), "
            "gen.fnv1a(g.row_ptr))" % ROOT)
    outs = set()
    for t in ("1", "3", "8"):
        env = dict(os.environ, GGEN_THREADS=t)
        outs.add(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                capture_output=True, text=True).stdout)
    assert len(outs) == 1


def test_rmat_skew_and_quadrants():
    s = 14
    g = gen.rmat(s, 16 << s, stream=11)
    assert g.n == 1 << s and g.m == 16 << s
    src, dst, _ = g.edge_list()
    # top bit of src set with probability c + d = .24, of dst with b + d = .24
    top = 1 << (s - 1)
    assert abs(np.mean(src >= top) - 0.24) < 0.01
    assert abs(np.mean(dst >= top) - 0.24) < 0.01
    # without permutation vertex 0 is the hub: expected degree m (a+b)^s
    expect = g.m * 0.76 ** s
    assert 0.8 * expect < g.degrees()[0] < 1.2 * expect


def test_grid_structure():
    W, H = 20, 15
    g = gen.grid(W, H, 0, 8, 1, 1000, stream=4)
    und = H * (W - 1) + W * (H - 1)
    assert g.m == 2 * und
    deg = g.degrees()
    assert deg.min() == 2 and deg.max() == 4
    src, dst, w = g.edge_list()
    # symmetric with one weight per undirected edge
    fwd = {(int(u), int(v)): int(x) for u, v, x in zip(src, dst, w)}
    assert all(fwd[(v, u)] == x for (u, v), x in fwd.items())
    assert np.all(np.abs(src - dst) > 0)
    assert set(np.abs(src - dst).tolist()) == {1, W}


def test_grid_shortcuts():
    W = 64
    k = (2 * W * (W - 1)) // 100
    g = gen.grid(W, W, k, 8, 1, 1000, stream=6)
    assert g.m == 2 * (2 * W * (W - 1) + k)
    src, dst, _ = g.edge_list()
    dx = np.abs(src % W - dst % W)
    dy = np.abs(src // W - dst // W)
    short = (dx + dy) >= 2
    assert short.sum() == 2 * k
    assert dx.max() <= 8 and dy.max() <= 8


def test_full_size_grid_counts():
    assert gen.GRID_SHORTCUTS == 335462
    lib = gen._load()
    assert lib.ggen_grid_edges(4096, 4096, gen.GRID_SHORTCUTS) == 67763404


def test_pick_sources_have_out_edges():
    g = gen.rmat(12, 16 << 12, stream=12)
    s = gen.pick_sources(g, 50, stream=1)
    assert np.all(g.degrees()[s] > 0)


def test_from_edges_is_stable():
    g = gen.from_edges(3, [2, 0, 2, 0], [1, 2, 0, 1], [5, 6, 7, 8])
    np.testing.assert_array_equal(g.row_ptr, [0, 2, 2, 4])
    np.testing.assert_array_equal(g.col, [2, 1, 1, 0])
    np.testing.assert_array_equal(g.w, [6, 8, 5, 7])
