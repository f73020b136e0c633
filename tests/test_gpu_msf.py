"""GPU parity of the minimum spanning forest against the oracle's Kruskal:
the same edge set (keys (weight, edge index) make it unique), weight and
size, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
from helpers import golden_files, path_graph, random_graph, read_golden, star
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_01665_amd import gg as _gg
    _gg.lib()
    return _gg


def check(gg, hg, reps=2, ws=False, stream=None):
    want, total = oracle.msf(hg.n, hg.row_ptr, hg.col, hg.w)
    g = gg.Graph.from_host(hg)
    w = gg.Workspace(g) if ws else None
    try:
        for _ in range(reps):
            say(f"[gpu] msf {hg.name} n={hg.n} m={hg.m}")
            sel, tw, ne = g.msf(ws=w, stream=stream)
            got = sel.cpu().numpy()
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, (f"{hg.name}: {bad.size} mismatches, first e={bad[0]} "
                                   f"got={got[bad[0]]} want={want[bad[0]]}")
            assert tw == total and ne == int(want.sum()), (hg.name, tw, total, ne)
    finally:
        if w is not None:
            w.free()
        g.free()


@pytest.mark.parametrize("fname", golden_files())
def test_golden(gg, fname):
    hg, _, _ = read_golden(fname)
    if hg.w is not None:
        check(gg, hg)


def test_random_tiny_graphs_with_ties(gg):
    rng = np.random.default_rng(91)
    for i in range(40):
        n = int(rng.integers(1, 300))
        hg = random_graph(rng, n, int(rng.integers(0, 6 * n + 1)), 0 if i % 4 == 0 else 1,
                          int(rng.integers(1, 6)), name=f"t{i}")
        check(gg, hg, reps=1)


def test_shapes(gg):
    # a path whose weights grow along it: every component picks the edge to
    # its left, so one round links a chain of all vertices
    check(gg, path_graph(5000, np.arange(1, 5000)))
    check(gg, path_graph(5000, np.arange(5000, 1, -1)))
    check(gg, star(40, [[5, 3, 3]] * 40))
    check(gg, gen.from_edges(1, [0, 0], [0, 0], [4, 1], name="loops"))
    check(gg, gen.from_edges(9, [], [], [], name="empty"))
    check(gg, gen.workload("grid96"), ws=True)


def test_workloads(gg):
    for name in ("er16k", "rmat14", "rmat16", "grid724"):
        check(gg, gen.workload(name))


def test_streams_and_errors(gg):
    import torch
    hg = gen.workload("rmat12")
    check(gg, hg, reps=3, ws=True, stream=torch.cuda.Stream())
    g = gg.Graph(hg.n, hg.row_ptr, hg.col)  # unweighted
    try:
        with pytest.raises(gg.GGError):
            g.msf()
    finally:
        g.free()
