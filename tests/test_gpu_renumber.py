"""GPU parity on graphs stored in the library's own vertex order (hottest
vertex first, GG_RENUMBER): every id at the interface stays the caller's, so
every variant must still equal the oracle element by element -- distances,
levels, CC labels (the smallest caller id of each component) and the forest
flags of gg_msf (by caller edge index) -- through the blocking, the
host-asynchronous, the serving and the allocation-free entry points.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from helpers import random_graph, star
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu

# (name, mode, sched, mapping, hops, delta)
VARIANTS = [("vertex-sync-thread", 0, 0, 1, 0, 0), ("vertex-sync-balanced", 0, 0, 3, 0, 0),
            ("vertex-async-wave", 0, 1, 2, 0, 0), ("vertex-async-balanced", 0, 1, 3, 0, 0),
            ("vertex-async-local8", 0, 1, 3, 8, 0), ("edge-sync", 1, 0, 0, 0, 0),
            ("edge-async", 1, 1, 0, 0, 0), ("nearfar-local4", 0, 3, 3, 4, 20),
            ("vertex-diropt", 0, 4, 3, 0, 0), ("edge-diropt", 1, 4, 0, 0, 0),
            ("unionfind", 0, 5, 3, 0, 0)]


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


def graphs():
    rng = np.random.default_rng(1903_01665)
    out = [gen.workload("rmat12"), gen.workload("grid48"),
           # many components and isolated vertices: CC's minimum of caller ids
           random_graph(rng, 3000, 1500, 1, 9, name="sparse3000"),
           star(40, [[5, 2]] * 40),
           random_graph(rng, 257, 4000, 0, 3, name="dense257")]
    return out


def applies(algo, v):
    name, mode, sched = v[0], v[1], v[2]
    if sched == 3 and algo != "sssp":
        return False
    if sched == 4 and mode == 1 and algo != "cc":
        return False
    if sched == 5 and algo != "cc":
        return False
    return True


def test_every_variant_in_the_caller_ids(gg):
    for hg in graphs():
        s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
        want = {"sssp": oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s),
                "bfs": oracle.bfs(hg.n, hg.row_ptr, hg.col, s),
                "cc": oracle.cc(hg.n, hg.row_ptr, hg.col)}
        g = gg.Graph.from_host(hg, symmetrize=True, transpose=True, renumber=True)
        try:
            assert g.renumbered()
            for v in VARIANTS:
                o = gg.make_opts(v[1], v[2], v[3], hops=v[4], delta=v[5])
                for algo in ("sssp", "bfs", "cc"):
                    if not applies(algo, v):
                        continue
                    say(f"[gpu] renumbered {hg.name} n={hg.n} {algo} {v[0]}")
                    out = g.cc(opts=o) if algo == "cc" else getattr(g, algo)(s, opts=o)
                    got = out.cpu().numpy()
                    assert g.stats()["rc"] == 0
                    bad = np.flatnonzero(got != want[algo])
                    assert bad.size == 0, (hg.name, algo, v[0], bad.size, int(bad[0]),
                                           int(got[bad[0]]), int(want[algo][bad[0]]))
            # every source of a small graph, AUTO variant
            if hg.n <= 300:
                for src in range(hg.n):
                    np.testing.assert_array_equal(
                        g.sssp(src).cpu().numpy(),
                        oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, src))
        finally:
            g.free()


def test_order_choice(gg):
    """Skewed graphs of >= 2^20 edges are renumbered unless the caller keeps
    the order; uniform ones and small ones are not."""
    big = gen.workload("rmat16")
    small = gen.workload("rmat12")
    uni = gen.workload("er16k")
    for hg, kw, want in ((big, {}, True), (big, {"renumber": False}, False),
                         (small, {}, False), (small, {"renumber": True}, True),
                         (uni, {}, False)):
        g = gg.Graph.from_host(hg, **kw)
        try:
            assert g.renumbered() == want, (hg.name, kw)
            s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
            np.testing.assert_array_equal(g.bfs(s).cpu().numpy(),
                                          oracle.bfs(hg.n, hg.row_ptr, hg.col, s))
        finally:
            g.free()


def test_forest_in_caller_edge_order(gg):
    rng = np.random.default_rng(77)
    for hg in (gen.workload("rmat12"), random_graph(rng, 500, 3000, 0, 4, name="ties500")):
        want, total = oracle.msf(hg.n, hg.row_ptr, hg.col, hg.w)
        g = gg.Graph.from_host(hg, renumber=True)
        try:
            assert g.renumbered()
            sel, tw, ne = g.msf()
            got = sel.cpu().numpy()
            assert np.array_equal(got, want), (hg.name, int((got != want).sum()))
            assert tw == total and ne == int(want.sum())
        finally:
            g.free()


def test_async_serve_and_noalloc(gg):
    import torch
    hg = gen.workload("rmat14")
    srcs = [int(x) for x in gen.pick_sources(hg, 6, stream=gen.STREAM["sources"])]
    g = gg.Graph.from_host(hg, symmetrize=True, renumber=True)
    try:
        assert g.renumbered()
        ws = [gg.Workspace(g) for _ in range(3)]
        tickets = [g.sssp_async(srcs[0], ws=ws[0]), g.bfs_async(srcs[1], ws=ws[1]),
                   g.cc_async(ws=ws[2])]
        d, b, c = [t.wait() for t in tickets]
        for t in tickets:
            t.free()
        for w in ws:
            w.free()
        np.testing.assert_array_equal(d.cpu().numpy(),
                                      oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, srcs[0]))
        np.testing.assert_array_equal(b.cpu().numpy(),
                                      oracle.bfs(hg.n, hg.row_ptr, hg.col, srcs[1]))
        np.testing.assert_array_equal(c.cpu().numpy(), oracle.cc(hg.n, hg.row_ptr, hg.col))
        # allocation-free BFS on the renumbered graph
        out = torch.full((hg.n,), -3, dtype=torch.int32, device="cuda")
        o = gg.make_opts()
        stream = torch.cuda.current_stream()
        rc = gg.lib().gg_bfs_noalloc(g.handle, srcs[2], ctypes.byref(o),
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0
        np.testing.assert_array_equal(out.cpu().numpy(),
                                      oracle.bfs(hg.n, hg.row_ptr, hg.col, srcs[2]))
    finally:
        g.free()
    # served queries on a renumbered graph
    srv = gg.Server(slots=4)
    try:
        gid = srv.add_graph(gg.Graph.from_host(hg, symmetrize=True, renumber=True))
        outs = [torch.full((hg.n,), -5, dtype=torch.int32, device="cuda") for _ in srcs]
        ids = {srv.submit(gid, i % 2, s, o): i for i, (s, o) in enumerate(zip(srcs, outs))}
        done = 0
        while done < len(srcs):
            for qid, st, rounds, ts, ta, td in srv.poll():
                assert st == 0
                i = ids[qid]
                # readable once reported done
                got = outs[i].cpu().numpy()
                want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, srcs[i]) if i % 2 == 0 \
                    else oracle.bfs(hg.n, hg.row_ptr, hg.col, srcs[i])
                np.testing.assert_array_equal(got, want)
                done += 1
    finally:
        srv.free()
