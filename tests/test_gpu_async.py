"""Host-asynchronous traversals (gg_*_async): one host thread keeps several
traversals in flight together (the paper's barrier-free independent kernels,
Sec. 3.2); every result is bit-exact against the oracle; the workspace, the
caller's stream order and the time limit behave as gg.h states."""
import sys

import numpy as np
import pytest

import oracle
from helpers import path_graph
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu

VERTEX, EDGE, SYNC, ASYNC = 0, 1, 0, 1
EBUSY, ETIMEOUT = -4, -6


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


def want_of(hg, s):
    return {"sssp": oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s),
            "bfs": oracle.bfs(hg.n, hg.row_ptr, hg.col, s),
            "cc": oracle.cc(hg.n, hg.row_ptr, hg.col)}


def test_async_every_variant_matches_the_oracle(gg):
    variants = [(VERTEX, SYNC, 1), (VERTEX, SYNC, 3), (VERTEX, ASYNC, 2), (VERTEX, ASYNC, 3),
                (EDGE, SYNC, 0), (EDGE, ASYNC, 0)]
    for name in ("rmat13", "grid96", "er16k"):
        hg = gen.workload(name)
        s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
        want = want_of(hg, s)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            opts = [gg.make_opts(*v) for v in variants]
            opts += [gg.make_opts(), gg.make_opts(VERTEX, gg.NEARFAR, 3, hops=4, far_degree=8)]
            for k, o in enumerate(opts):
                say(f"[gpu] async {name} variant {k}")
                for algo in ("sssp", "bfs", "cc"):
                    if algo != "sssp" and o.sched == gg.NEARFAR:
                        continue
                    t = (g.cc_async(opts=o) if algo == "cc"
                         else getattr(g, algo + "_async")(s, opts=o))
                    got = t.wait().cpu().numpy()
                    t.free()
                    assert g.stats()["rc"] == 0
                    np.testing.assert_array_equal(got, want[algo], err_msg=f"{name} {algo} {k}")
            for o in (gg.make_opts(VERTEX, gg.DIROPT, 3), gg.make_opts(EDGE, gg.DIROPT, 0)):
                algo = "bfs" if o.mode == VERTEX else "cc"
                t = g.bfs_async(s, opts=o) if algo == "bfs" else g.cc_async(opts=o)
                np.testing.assert_array_equal(t.wait().cpu().numpy(), want[algo])
                t.free()
        finally:
            g.free()


def test_one_host_thread_overlaps_sssp_bfs_and_cc(gg):
    """SSSP, BFS and CC issued back to back from this thread, each on its own
    workspace: the later ones begin on the device before the first ends, and
    all three results are exact."""
    import torch
    hg = gen.workload("grid256")
    s = 0
    want = want_of(hg, s)
    g = gg.Graph.from_host(hg, symmetrize=True)
    ws = [gg.Workspace(g) for _ in range(3)]
    outs = [torch.full((hg.n,), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    # vertex-synchronous sweeps over a 256 x 256 grid from a corner take
    # hundreds of rounds, milliseconds, far longer than issuing a call
    o = gg.make_opts(VERTEX, SYNC, 3)
    try:
        for rep in range(3):
            say(f"[gpu] async overlap grid256 rep={rep}")
            t0 = g.sssp_async(s, out=outs[0], ws=ws[0], opts=o)
            t1 = g.bfs_async(s, out=outs[1], ws=ws[1], opts=o)
            t2 = g.cc_async(out=outs[2], ws=ws[2], opts=o)
            for t in (t0, t1, t2):
                t.wait()
            b0, e0, r0 = t0.times()
            b1, e1, _ = t1.times(t0)
            b2, e2, _ = t2.times(t0)
            say(f"[gpu]   sssp [{b0:.3f}, {e0:.3f}] ms ({r0} rounds), bfs [{b1:.3f}, {e1:.3f}], "
                f"cc [{b2:.3f}, {e2:.3f}]")
            assert b1 < e0 and b2 < e0, (b0, e0, b1, e1, b2, e2)
            np.testing.assert_array_equal(outs[0].cpu().numpy(), want["sssp"])
            np.testing.assert_array_equal(outs[1].cpu().numpy(), want["bfs"])
            np.testing.assert_array_equal(outs[2].cpu().numpy(), want["cc"])
            for t in (t0, t1, t2):
                t.free()
            for x in outs:
                x.fill_(-1)
    finally:
        for w in ws:
            w.free()
        g.free()


def test_workspace_stays_taken_while_in_flight(gg):
    """A long traversal (a path: one level per round) holds its workspace:
    calls on it, its statistics, freeing it and freeing the graph are
    refused until the ticket reports the end; then all work again."""
    import torch
    n = 40000
    hg = path_graph(n, np.ones(n - 1, np.int32))
    want = oracle.bfs(hg.n, hg.row_ptr, hg.col, 0)
    g = gg.Graph.from_host(hg)
    ws = gg.Workspace(g)
    o = gg.make_opts(VERTEX, SYNC, 1)
    try:
        say("[gpu] async busy path40000")
        t = g.bfs_async(0, ws=ws, opts=o)
        t_def = g.bfs_async(0, opts=o)  # the default workspace is another one
        assert not t.query()
        with pytest.raises(gg.GGError) as e:
            g.bfs(0, ws=ws, opts=o)
        assert e.value.code == EBUSY
        with pytest.raises(gg.GGError) as e:
            g.bfs_async(0, ws=ws, opts=o)
        assert e.value.code == EBUSY
        assert g.stats(ws)["rc"] == EBUSY
        with pytest.raises(gg.GGError) as e:
            ws.free()
        assert e.value.code == EBUSY
        h = g.handle
        assert gg.lib().gg_graph_free(h) == EBUSY
        got = t.wait().cpu().numpy()
        np.testing.assert_array_equal(got, want)
        assert t.query()
        np.testing.assert_array_equal(t_def.wait().cpu().numpy(), want)
        st = g.stats(ws)
        assert st["rc"] == 0 and st["iterations"] >= n - 1, st
        t.free()
        t_def.free()
        # the workspace serves a plain call on another stream afterwards
        s2 = torch.cuda.Stream()
        got = g.bfs(5, ws=ws, opts=gg.make_opts(VERTEX, ASYNC, 3), stream=s2)
        s2.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(),
                                      oracle.bfs(hg.n, hg.row_ptr, hg.col, 5))
    finally:
        ws.free()
        g.free()


def test_async_follows_the_callers_stream(gg):
    """The traversal starts after the work enqueued on the caller's stream
    before the call (a spin kernel, then a fill of the output), and a second
    stream made to wait on the ticket sees the final values."""
    import torch
    hg = gen.workload("rmat14")
    s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
    want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
    g = gg.Graph.from_host(hg)
    st, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    out = torch.empty(hg.n, dtype=torch.int32, device="cuda")
    try:
        for rep in range(3):
            say(f"[gpu] async stream order rep={rep}")
            torch.cuda.synchronize()
            with torch.cuda.stream(st):
                torch.cuda._sleep(20_000_000)  # ~10 ms on the caller's stream
                out.fill_(-5)
            t = g.sssp_async(s, out=out, stream=st)
            t.stream_wait(st2)
            with torch.cuda.stream(st2):
                copy = out.clone()
            st2.synchronize()
            np.testing.assert_array_equal(copy.cpu().numpy(), want)
            assert t.wait() is out
            t.free()
    finally:
        g.free()


def test_async_time_limit_reports_timeout(gg):
    """A traversal that runs out of time stops with GG_ETIMEOUT (the driver
    does not wait for it while serving others), and the workspace is usable
    afterwards."""
    n = 200000
    hg = path_graph(n, np.ones(n - 1, np.int32))
    g = gg.Graph.from_host(hg)
    try:
        say("[gpu] async time limit path200000")
        t_long = g.bfs_async(0, opts=gg.make_opts(VERTEX, SYNC, 1, time_limit_ms=5))
        ws = gg.Workspace(g)
        t_short = g.sssp_async(n - 10, ws=ws, opts=gg.make_opts(VERTEX, ASYNC, 3))
        with pytest.raises(gg.GGError) as e:
            t_long.wait()
        assert e.value.code == ETIMEOUT
        np.testing.assert_array_equal(t_short.wait().cpu().numpy(),
                                      oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, n - 10))
        t_long.free()
        t_short.free()
        ws.free()
        got = g.bfs(n - 100, opts=gg.make_opts(VERTEX, ASYNC, 3)).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.bfs(hg.n, hg.row_ptr, hg.col, n - 100))
    finally:
        g.free()
