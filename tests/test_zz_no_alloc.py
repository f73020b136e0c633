"""BFS through the entry point that allocates nothing (gg_bfs_noalloc, for
callers that cannot allocate): its scratch memory is a fixed device array of
the library.  Two calls in a row, the second on a smaller graph, each
element by element equal to gg_bfs_ex (the same traversal with a workspace)
and to the oracle; a graph above the array's vertex limit is refused."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
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


def noalloc(gg, g, source, opts, out):
    import torch
    stream = torch.cuda.current_stream()
    return gg.lib().gg_bfs_noalloc(g.handle, int(source), ctypes.byref(opts),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_bfs_matches_the_workspace_form(gg):
    import torch
    big = gen.workload("rmat16")
    small = gen.workload("grid96")
    variants = [gg.make_opts(), gg.make_opts(gg.VERTEX, gg.ASYNC, gg.MAP_BALANCED),
                gg.make_opts(gg.VERTEX, gg.SYNC, gg.MAP_THREAD),
                gg.make_opts(gg.EDGE, gg.ASYNC), gg.make_opts(gg.VERTEX, gg.DIROPT)]
    for k, o in enumerate(variants):
        for hg in (big, small):  # the second call of each pair is smaller
            s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
            g = gg.Graph.from_host(hg, symmetrize=True)
            try:
                say(f"[gpu] noalloc bfs {hg.name} n={hg.n} variant {k}")
                want = g.bfs(s, opts=o).cpu().numpy()
                out = torch.full((hg.n,), -3, dtype=torch.int32, device="cuda")
                assert noalloc(gg, g, s, o, out) == 0
                got = out.cpu().numpy()
                np.testing.assert_array_equal(got, want)
                np.testing.assert_array_equal(got, oracle.bfs(hg.n, hg.row_ptr, hg.col, s))
            finally:
                g.free()


def test_noalloc_refuses_graphs_above_its_limit(gg):
    import torch
    n = (1 << 22) + 1
    hg = gen.from_edges(n, [0], [1], [1])
    g = gg.Graph.from_host(hg)
    try:
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        assert noalloc(gg, g, 0, gg.make_opts(), out) == -1
    finally:
        g.free()
