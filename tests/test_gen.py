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


# ------------------------------------------------------------ pinned values --
_M64 = (1 << 64) - 1


def _rotl(x, k):
    return ((x << k) | (x >> (64 - k))) & _M64


def _splitmix64(x):
    """One SplitMix64 step (Steele, Lea & Flood 2014): (new state, output)."""
    x = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return x, z ^ (z >> 31)


def _xoshiro256ss(s):
    """One xoshiro256** step (Blackman & Vigna 2018) on the list s."""
    r = (_rotl((s[1] * 5) & _M64, 7) * 9) & _M64
    t = (s[1] << 17) & _M64
    s[2] ^= s[0]
    s[3] ^= s[1]
    s[1] ^= s[2]
    s[0] ^= s[3]
    s[2] ^= t
    s[3] = _rotl(s[3], 45)
    return r


def test_reference_generators_reproduce_published_outputs():
    # SplitMix64 from state 0 and xoshiro256** from state {1, 2, 3, 4}: the
    # first outputs of the authors' reference code
    x, a = _splitmix64(0)
    x, b = _splitmix64(x)
    assert (a, b) == (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4)
    s = [1, 2, 3, 4]
    assert [_xoshiro256ss(s) for _ in range(4)] == [11520, 0, 1509978240, 1215971899390074240]


def test_generator_stream_matches_the_reference_generators():
    # each (seed, stream, chunk) folds the three words through SplitMix64,
    # then four more SplitMix64 outputs seed xoshiro256**
    for seed, stream, chunk in [(gen.MASTER_SEED, 0, 0), (gen.MASTER_SEED, 7, 3), (1, 2**40, 5)]:
        x, h = _splitmix64(seed)
        x, h = _splitmix64(h ^ stream)
        x, h = _splitmix64(h ^ chunk)
        x, st = h, []
        for _ in range(4):
            x, o = _splitmix64(x)
            st.append(o)
        want = [_xoshiro256ss(st) for _ in range(64)]
        got = [int(v) for v in gen.raw(seed, stream, chunk, 64)]
        assert got == want, (seed, stream, chunk)


def test_fnv1a_is_the_64_bit_fnv1a_of_the_bytes():
    a = np.array([0, 1, -1, 2**31 - 1, 123456789], np.int32)
    h = 0xCBF29CE484222325
    for byte in a.tobytes():
        h = ((h ^ byte) * 0x100000001B3) & _M64
    assert gen.fnv1a(a) == h


# Edge count, weight sum and FNV-1a of the CSR arrays of three workloads,
# recorded from this generator.  Every number measured on these workloads
# depends on them: a change here must be deliberate.
PINNED = {
    "er16k": (16384, 131072, 6628609, 15350851502895587387, 2798882199098992367,
              1518096853049179888),
    "rmat14": (16384, 262144, 13213434, 16872330375340597956, 18306333071721251876,
               14554040412407950779),
    "grid96": (9216, 36844, 18304316, 7844583345317226537, 8516709398010831331,
               5409390177751042377),
}


def test_workloads_are_pinned():
    for name, (n, m, wsum, hrow, hcol, hw) in PINNED.items():
        g = gen.workload(name)
        got = (g.n, g.m, int(g.w.astype(np.int64).sum()), gen.fnv1a(g.row_ptr),
               gen.fnv1a(g.col), gen.fnv1a(g.w))
        assert got == (n, m, wsum, hrow, hcol, hw), name
