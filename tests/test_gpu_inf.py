"""SSSP with weights near 2^30: paths whose length reaches 2^31-1 are
reported as INF, paths just below it stay exact, in every variant.

The relaxation of Algorithms 1-2 adds a weight to the tail's distance; with
int32 values that sum can pass 2^31-1.  The library's reading is that the
result is min(shortest distance, INF), INF = 2^31-1, and the oracle clamps
its int64 Dijkstra distances the same way.  These graphs put many shortest
paths on both sides of that line, so a kernel that wraps the sum, saturates
it wrongly or drops a candidate too early fails element by element.
"""
import sys

import numpy as np
import pytest

import oracle
from helpers import INF, path_graph, random_graph
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu

VERTEX, EDGE, SYNC, ASYNC = 0, 1, 0, 1
THREAD, WAVE, BALANCED = 1, 2, 3
PLAIN = [(VERTEX, SYNC, THREAD), (VERTEX, SYNC, WAVE), (VERTEX, SYNC, BALANCED),
         (VERTEX, ASYNC, THREAD), (VERTEX, ASYNC, WAVE), (VERTEX, ASYNC, BALANCED),
         (EDGE, SYNC, 0), (EDGE, ASYNC, 0)]


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


def huge(hg, lo, hi, seed, name):
    """The same topology with weights drawn uniformly from [lo, hi]."""
    rng = np.random.default_rng(seed)
    w = rng.integers(lo, hi + 1, size=hg.m, dtype=np.int64).astype(np.int32)
    src = np.repeat(np.arange(hg.n, dtype=np.int32), np.diff(hg.row_ptr))
    return gen.from_edges(hg.n, src, hg.col, w, name=name)


def mixed(hg, seed, name):
    """Weights that are mostly small with some near 2^30 and a few near
    2^31: distances land on both sides of INF and exactly on it."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 10, size=hg.m)
    w = rng.integers(1, 10, size=hg.m, dtype=np.int64)
    big = rng.integers(2**30 - 8, 2**30 + 8, size=hg.m, dtype=np.int64)
    top = rng.integers(INF - 12, INF + 1, size=hg.m, dtype=np.int64)
    w = np.where(k < 6, w, np.where(k < 9, big, top)).astype(np.int32)
    src = np.repeat(np.arange(hg.n, dtype=np.int32), np.diff(hg.row_ptr))
    return gen.from_edges(hg.n, src, hg.col, w, name=name)


def cases():
    rng = np.random.default_rng(2**30)
    out = []
    # the edges of the INF line: a sum equal to INF is INF, one below is exact
    out.append((path_graph(4, [INF - 1, 1, 1]), 0, [0, INF - 1, INF, INF]))
    out.append((path_graph(4, [INF - 2, 1, 1]), 0, [0, INF - 2, INF - 1, INF]))
    out.append((path_graph(3, [INF, 0]), 0, [0, INF, INF]))
    out.append((path_graph(5, [2**30, 2**30 - 1, 0, 1]), 0, [0, 2**30, INF, INF, INF]))
    out.append((path_graph(5, [2**30 - 1, 2**30 - 1, 0, 1]), 0,
                [0, 2**30 - 1, INF - 1, INF - 1, INF]))
    for i in range(6):
        n = int(rng.integers(2, 300))
        hg = random_graph(rng, n, int(rng.integers(n, 6 * n + 1)), 2**29, INF, name=f"big{i}")
        out.append((hg, int(rng.integers(0, n)), None))
    for i in range(4):
        n = int(rng.integers(2, 400))
        hg = random_graph(rng, n, int(rng.integers(n, 8 * n + 1)), 1, 9, name=f"mix{i}")
        out.append((mixed(hg, 100 + i, f"mix{i}"), int(rng.integers(0, n)), None))
    hub = gen.workload("rmat14")  # heavy rows go through the chunk kernel
    s = int(gen.pick_sources(hub, 1, stream=gen.STREAM["sources"])[0])
    out.append((huge(hub, 2**28, 2**30, 7, "rmat14-big"), s, None))
    out.append((mixed(hub, 8, "rmat14-mix"), s, None))
    grid = gen.workload("grid96")  # deep: many rounds, local expansion
    out.append((huge(grid, 2**24, 2**25, 9, "grid96-big"), 0, None))
    return out


def near_far_opts(gg):
    out = []
    # (a width of 1 would take about 2^31 rounds to cross these distances:
    # the bound grows by one width per round that pushes nothing near)
    for delta in (0, 2**20, 2**29, INF):
        for hops, far in ((0, 0), (3, 0), (0, 4), (3, 4)):
            out.append((f"nearfar-d{delta}-h{hops}-f{far}",
                        gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED, delta=delta,
                                     hops=hops, far_degree=far)))
    for hops in (1, 3, 64):
        out.append((f"async-h{hops}", gg.make_opts(gg.VERTEX, gg.ASYNC, gg.MAP_BALANCED,
                                                   hops=hops)))
    return out


def test_inf_line_every_variant(gg):
    extra = near_far_opts(gg)
    for hg, s, fixed in cases():
        want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
        if fixed is not None:
            # the closed form of the path cases pins the oracle too
            np.testing.assert_array_equal(want, np.array(fixed, np.int32), err_msg=hg.name)
        reach = int(np.sum(want != INF))
        g = gg.Graph.from_host(hg)
        try:
            variants = [(f"{m}-{sc}-{mp}", gg.make_opts(m, sc, mp)) for m, sc, mp in PLAIN]
            variants += extra + [("auto", None)]
            for name, o in variants:
                say(f"[gpu] inf {hg.name} n={hg.n} m={hg.m} s={s} reached={reach} {name}")
                got = g.sssp(s, opts=o).cpu().numpy()
                st = g.stats()
                assert st["rc"] == 0, (hg.name, name, st)
                bad = np.flatnonzero(got != want)
                assert bad.size == 0, (f"{hg.name} {name}: {bad.size} mismatches, first "
                                       f"v={bad[0]} got={got[bad[0]]} want={want[bad[0]]}")
        finally:
            g.free()


def test_inf_line_auto_width_resolves(gg):
    """With a mean weight near 2^31 the default near-far width stays in range
    (it is capped at 2^30) and the traversal ends with exact distances."""
    rng = np.random.default_rng(31)
    hg = random_graph(rng, 500, 4000, INF - 1000, INF, name="top")
    g = gg.Graph.from_host(hg)
    try:
        o = g.resolve(gg.ALGO_SSSP, gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED))
        assert 1 <= o.delta <= 2**30, o.delta
        for s in (0, 17, 499):
            say(f"[gpu] inf top-weights nearfar auto width s={s}")
            got = g.sssp(s, opts=gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED)).cpu()
            assert g.stats()["rc"] == 0
            np.testing.assert_array_equal(got.numpy(),
                                          oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s))
    finally:
        g.free()


def test_inf_line_batched_and_served(gg):
    """The batched and the served paths concatenate or pool graphs; the
    clamp must hold there too."""
    import torch
    rng = np.random.default_rng(230)
    inst = []
    for i in range(12):
        n = int(rng.integers(2, 600))
        hg = random_graph(rng, n, int(rng.integers(n, 6 * n + 1)), 1, 9, name=f"b{i}")
        hg = mixed(hg, 300 + i, f"b{i}") if i % 2 else huge(hg, 2**29, INF, 400 + i, f"b{i}")
        inst.append((0, hg, int(rng.integers(0, n))))
    want = [oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s) for _, hg, s in inst]
    for flags in (0, gg.BATCH_NO_GRAPH):
        b = gg.Batch(inst, flags=flags)
        try:
            out = torch.full((b.total_n,), -7, dtype=torch.int32, device="cuda")
            for rep in range(2):
                say(f"[gpu] inf batch flags={flags} rep={rep}")
                out.fill_(-7)
                b.run(out)
                torch.cuda.synchronize()
                got, off = out.cpu().numpy(), b.offsets()
                for i, (_, hg, _) in enumerate(inst):
                    np.testing.assert_array_equal(got[off[i]: off[i] + hg.n], want[i],
                                                  err_msg=f"batch instance {i}")
        finally:
            b.free()
    srv = gg.Server(slots=4, mem_budget_bytes=0)
    try:
        gids = [srv.add_graph(gg.Graph.from_host(hg)) for _, hg, _ in inst]
        outs = [torch.full((hg.n,), -1, dtype=torch.int32, device="cuda") for _, hg, _ in inst]
        torch.cuda.synchronize()
        ids = {srv.submit(gids[i], gg.ALGO_SSSP, s, outs[i]): i
               for i, (_, _, s) in enumerate(inst)}
        done = {}
        while len(done) < len(ids):
            for qid, st, *_ in srv.poll():
                assert st == 0
                done[qid] = ids[qid]
        torch.cuda.synchronize()
        say("[gpu] inf served")
        for i in range(len(inst)):
            np.testing.assert_array_equal(outs[i].cpu().numpy(), want[i],
                                          err_msg=f"served query {i}")
    finally:
        srv.free()
