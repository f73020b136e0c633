"""GPU parity: every variant of the HIP path against the CPU oracle, bit-exact.

All calls go through the C ABI (libgg.so) via the ctypes binding.  Values are
int32 and exact, so the bar is element-by-element equality.
"""
import sys

import numpy as np
import pytest

import oracle
from helpers import golden_files, path_graph, random_graph, read_golden, star
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu

VERTEX, EDGE, SYNC, ASYNC = 0, 1, 0, 1
THREAD, WAVE, BALANCED = 1, 2, 3
VARIANTS = [(VERTEX, SYNC, THREAD), (VERTEX, SYNC, WAVE), (VERTEX, SYNC, BALANCED),
            (VERTEX, ASYNC, THREAD), (VERTEX, ASYNC, WAVE), (VERTEX, ASYNC, BALANCED),
            (EDGE, SYNC, 0), (EDGE, ASYNC, 0)]
VNAME = {v: f"{'vertex' if v[0] == 0 else 'edge'}-{'sync' if v[1] == 0 else 'async'}"
            f"{['', '-thread', '-wave', '-balanced'][v[2]]}" for v in VARIANTS}


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


def expected(hg, source):
    out = {"bfs": oracle.bfs(hg.n, hg.row_ptr, hg.col, source),
           "cc": oracle.cc(hg.n, hg.row_ptr, hg.col)}
    if hg.w is not None:
        out["sssp"] = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, source)
    return out


def check_graph(gg, hg, source, name, variants=VARIANTS, algos=("sssp", "bfs", "cc"),
                want=None):
    want = want or expected(hg, source)
    g = gg.Graph.from_host(hg, symmetrize=True)
    try:
        for v in variants:
            for algo in algos:
                if algo == "sssp" and hg.w is None:
                    continue
                say(f"[gpu] {name} n={hg.n} m={hg.m} {algo} {VNAME[v]}")
                if algo == "cc":
                    got = g.cc(*v)
                else:
                    got = getattr(g, algo)(source, *v)
                got = got.cpu().numpy()[: hg.n]
                st = g.stats()
                assert st["rc"] == 0, (name, algo, VNAME[v], st)
                assert st["iterations"] >= 1
                bad = np.flatnonzero(got != want[algo])
                assert bad.size == 0, (f"{name} {algo} {VNAME[v]}: {bad.size} mismatches, first "
                                       f"v={bad[0]} got={got[bad[0]]} want={want[algo][bad[0]]}")
    finally:
        g.free()


@pytest.mark.parametrize("fname", golden_files())
def test_golden(gg, fname):
    hg, s, want = read_golden(fname)
    check_graph(gg, hg, s, fname, want=want)


def test_random_tiny_graphs(gg):
    rng = np.random.default_rng(20190304)
    for i in range(24):
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 6 * n + 1))
        hg = random_graph(rng, n, m, 0, 9, name=f"tiny{i}")
        check_graph(gg, hg, int(rng.integers(0, n)), hg.name)


def test_no_edges_and_single_vertex(gg):
    check_graph(gg, gen.from_edges(1, [], [], []), 0, "n1")
    check_graph(gg, gen.from_edges(1, [0], [0], [4]), 0, "n1-loop")
    check_graph(gg, gen.from_edges(130, [], [], []), 77, "m0")


def test_heavy_rows_are_chunked(gg):
    # hubs far above the heavy-row threshold (64 edges), plus a tail
    rng = np.random.default_rng(5)
    src, dst = [], []
    for hub, deg in [(0, 3000), (1, 700), (65, 1500)]:
        src += [hub] * deg
        dst += list(rng.integers(0, 4000, size=deg))
    src += list(rng.integers(0, 4000, size=6000))
    dst += list(rng.integers(0, 4000, size=6000))
    w = rng.integers(1, 50, size=len(src))
    hg = gen.from_edges(4000, src, dst, w, name="hubs")
    check_graph(gg, hg, 0, "hubs")
    check_graph(gg, hg, 3999, "hubs-s3999")
    hg = star(600, [[5, 3], [1]] + [[7]] * 598)
    check_graph(gg, hg, 0, "star600")


def test_long_path(gg):
    hg = path_graph(1500, np.arange(1, 1500) % 7 + 1)
    check_graph(gg, hg, 0, "path1500")


def test_er16k(gg):
    hg = gen.workload("er16k")
    check_graph(gg, hg, 0, "er16k")


def test_rmat14(gg):
    hg = gen.workload("rmat14")
    s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
    check_graph(gg, hg, s, "rmat14")


def test_grid96(gg):
    hg = gen.workload("grid96")
    check_graph(gg, hg, 0, "grid96")


def test_repeat_and_launch_shapes(gg):
    """Same answer over repeats, workspaces and grid caps (race check)."""
    hg = gen.workload("rmat13")
    s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
    want = expected(hg, s)
    g = gg.Graph.from_host(hg, symmetrize=True)
    ws = gg.Workspace(g)
    try:
        for rep in range(3):
            for cap in (1, 7, 64, 0):
                for v in VARIANTS:
                    o = gg.make_opts(*v, max_blocks=cap)
                    say(f"[gpu] rmat13 rep={rep} cap={cap} {VNAME[v]}")
                    use = ws if rep % 2 else None
                    np.testing.assert_array_equal(
                        g.sssp(s, opts=o, ws=use).cpu().numpy(), want["sssp"])
                    np.testing.assert_array_equal(
                        g.bfs(s, opts=o, ws=use).cpu().numpy(), want["bfs"])
                    np.testing.assert_array_equal(
                        g.cc(opts=o, ws=use).cpu().numpy(), want["cc"])
    finally:
        ws.free()
        g.free()


def test_cc_without_shortcut(gg):
    hg = gen.workload("grid48")
    want = oracle.cc(hg.n, hg.row_ptr, hg.col)
    g = gg.Graph.from_host(hg)
    try:
        for v in VARIANTS:
            say(f"[gpu] grid48 cc no-jump {VNAME[v]}")
            o = gg.make_opts(*v, flags=gg.OPT_CC_NO_JUMP)
            np.testing.assert_array_equal(g.cc(opts=o).cpu().numpy(), want)
    finally:
        g.free()


def test_cc_needs_symmetric_arrays_except_edge_sync(gg):
    hg = gen.workload("er300x900")
    g = gg.Graph(hg.n, hg.row_ptr, hg.col, hg.w)  # no GG_SYMMETRIZE
    try:
        want = oracle.cc(hg.n, hg.row_ptr, hg.col)
        np.testing.assert_array_equal(g.cc().cpu().numpy(), want)  # AUTO -> edge sync
        np.testing.assert_array_equal(g.cc(EDGE, SYNC).cpu().numpy(), want)
        for mode, sched in [(VERTEX, SYNC), (VERTEX, ASYNC), (EDGE, ASYNC)]:
            with pytest.raises(gg.GGError) as e:
                g.cc(mode, sched)
            assert e.value.code == -5
    finally:
        g.free()


def test_bad_calls(gg):
    import torch
    hg = gen.workload("er300x900")
    g = gg.Graph(hg.n, hg.row_ptr, hg.col, None)  # unweighted
    try:
        with pytest.raises(gg.GGError) as e:
            g.sssp(0)
        assert e.value.code == -1
        for s in (-1, hg.n):
            with pytest.raises(gg.GGError):
                g.bfs(s)
        with pytest.raises(ValueError):
            g.bfs(0, out=torch.empty(hg.n - 1, dtype=torch.int32, device="cuda"))
    finally:
        g.free()


def test_two_streams_two_workspaces(gg):
    """SSSP and BFS issued at the same moment from two host threads, each on
    its own stream and workspace: their device time lines overlap (profile
    events on one time line), and both results are exact."""
    import threading

    import torch
    hg = gen.workload("grid256")  # hundreds of rounds: milliseconds each
    want = expected(hg, 0)
    g = gg.Graph.from_host(hg, symmetrize=True)
    ws = [gg.Workspace(g), gg.Workspace(g)]
    st = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.full((hg.n,), -1, dtype=torch.int32, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    o = gg.make_opts(VERTEX, SYNC, BALANCED, flags=gg.OPT_PROFILE)
    try:
        for rep in range(3):
            say(f"[gpu] two host threads, two streams: grid256 rep={rep}")
            gate = threading.Barrier(2)
            errs = []

            def run(i):
                try:
                    gate.wait()
                    fn = g.sssp if i == 0 else g.bfs
                    fn(0, out=outs[i], ws=ws[i], stream=st[i], opts=o)
                except Exception as e:  # reported below
                    errs.append(e)

            th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
            for t in th:
                t.start()
            for t in th:
                t.join()
            assert not errs, errs
            torch.cuda.synchronize()
            p0, p1 = g.profile(ws[0]), g.profile(ws[1])
            say(f"[gpu]   sssp [{p0['begin_ms']:.3f}, {p0['end_ms']:.3f}] ms, "
                f"bfs [{p1['begin_ms']:.3f}, {p1['end_ms']:.3f}] ms")
            assert p0["begin_ms"] < p1["end_ms"] and p1["begin_ms"] < p0["end_ms"], (p0, p1)
            np.testing.assert_array_equal(outs[0].cpu().numpy(), want["sssp"])
            np.testing.assert_array_equal(outs[1].cpu().numpy(), want["bfs"])
            for x in outs:
                x.fill_(-1)
    finally:
        for w in ws:
            w.free()
        g.free()


def test_nearfar_sssp(gg):
    """The near-far schedule (buckets of width delta) gives the same distances."""
    rng = np.random.default_rng(1903)
    graphs = [read_golden(f)[:2] for f in golden_files()]
    for i in range(8):
        n = int(rng.integers(1, 300))
        graphs.append((random_graph(rng, n, int(rng.integers(0, 6 * n + 1)), 0, 9,
                                    name=f"nf{i}"), int(rng.integers(0, n))))
    hub = gen.workload("rmat14")
    graphs += [(gen.workload("er16k"), 0), (gen.workload("grid96"), 0),
               (hub, int(gen.pick_sources(hub, 1, stream=gen.STREAM["sources"])[0])),
               (path_graph(700, np.arange(1, 700) % 5 + 1), 0)]
    for hg, s in graphs:
        want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
        g = gg.Graph.from_host(hg)
        try:
            for delta in (1, 5, 0, 10**6):
                say(f"[gpu] nearfar {hg.name} n={hg.n} delta={delta}")
                o = gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED, delta=delta)
                got = g.sssp(s, opts=o).cpu().numpy()
                assert g.stats()["rc"] == 0
                np.testing.assert_array_equal(got, want, err_msg=f"{hg.name} delta={delta}")
            with pytest.raises(gg.GGError):
                g.bfs(s, opts=gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED))
            with pytest.raises(gg.GGError):
                g.sssp(s, opts=gg.make_opts(gg.EDGE, gg.NEARFAR))
        finally:
            g.free()


def test_nearfar_long_rows_only(gg):
    """Near-far with only rows longer than far_degree held back (short rows
    served at once), plain and with local expansion: the same distances."""
    rng = np.random.default_rng(7)
    graphs = [read_golden(f)[:2] for f in golden_files()]
    for i in range(5):
        n = int(rng.integers(1, 300))
        graphs.append((random_graph(rng, n, int(rng.integers(0, 8 * n + 1)), 1, 50,
                                    name=f"far{i}"), int(rng.integers(0, n))))
    hub = gen.workload("rmat14")
    graphs += [(hub, int(gen.pick_sources(hub, 1, stream=gen.STREAM["sources"])[0])),
               (gen.workload("er16k"), 0), (path_graph(500, np.arange(1, 500) % 7 + 1), 0),
               (star(300, [[4, 9, 2]] * 300), 0)]
    for hg, s in graphs:
        want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
        g = gg.Graph.from_host(hg)
        try:
            for far in (1, 4, 64):
                for delta in (1, 7, 0):
                    for hops in (0, 3):
                        say(f"[gpu] nearfar-long {hg.name} n={hg.n} far={far} delta={delta} "
                            f"hops={hops}")
                        o = gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED, delta=delta,
                                         hops=hops, far_degree=far)
                        got = g.sssp(s, opts=o).cpu().numpy()
                        assert g.stats()["rc"] == 0
                        np.testing.assert_array_equal(got, want,
                                                      err_msg=f"{hg.name} far={far} d={delta}")
            with pytest.raises(gg.GGError):
                g.sssp(s, opts=gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED,
                                            far_degree=-1))
        finally:
            g.free()


def test_local_expansion(gg):
    """Worklist rounds whose wavefronts serve their own updates again in the
    same round (opts.hops) give the same distances, levels and labels; on a
    path they cover many levels per round."""
    rng = np.random.default_rng(1665)
    graphs = [read_golden(f)[:2] for f in golden_files()]
    for i in range(6):
        n = int(rng.integers(1, 400))
        graphs.append((random_graph(rng, n, int(rng.integers(0, 5 * n + 1)), 1, 9,
                                    name=f"loc{i}"), int(rng.integers(0, n))))
    hub = gen.workload("rmat14")  # heavy rows: the chunk kernel under local expansion
    graphs += [(gen.workload("er16k"), 0), (gen.workload("grid96"), 0),
               (hub, int(gen.pick_sources(hub, 1, stream=gen.STREAM["sources"])[0])),
               (path_graph(700, np.arange(1, 700) % 5 + 1), 0),
               (star(200, [[5, 3, 9]] * 200), 0)]
    for hg, s in graphs:
        want = expected(hg, s)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            for hops in (1, 3, 64):
                for algo, sched, delta, fl in (
                        ("sssp", gg.ASYNC, 0, 0), ("sssp", gg.NEARFAR, 0, 0),
                        ("sssp", gg.NEARFAR, 5, 0), ("sssp", gg.NEARFAR, 5, gg.OPT_LISTS_DIRECT),
                        ("sssp", gg.ASYNC, 0, gg.OPT_LISTS_DIRECT),
                        ("sssp", gg.NEARFAR, 0, gg.OPT_LISTS_CHECKED),
                        ("bfs", gg.ASYNC, 0, 0), ("cc", gg.ASYNC, 0, 0)):
                    say(f"[gpu] local {hg.name} n={hg.n} {algo} sched={sched} delta={delta} "
                        f"hops={hops} flags={fl}")
                    o = gg.make_opts(gg.VERTEX, sched, gg.MAP_BALANCED, delta=delta, hops=hops,
                                     flags=fl)
                    got = (g.cc(opts=o) if algo == "cc" else getattr(g, algo)(s, opts=o))
                    st = g.stats()
                    assert st["rc"] == 0, st
                    np.testing.assert_array_equal(got.cpu().numpy()[: hg.n], want[algo],
                                                  err_msg=f"{hg.name} {algo} hops={hops}")
                    if hg.name == "path" and algo == "bfs":
                        # one wavefront walks hops + 1 levels per round
                        assert st["iterations"] <= 700 // (hops + 1) + 2, st
            for bad in (-1, 65):
                with pytest.raises(gg.GGError):
                    g.bfs(s, opts=gg.make_opts(gg.VERTEX, gg.ASYNC, gg.MAP_BALANCED, hops=bad))
        finally:
            g.free()


def test_diropt_bfs(gg):
    """Direction-optimizing BFS (push small frontiers, pull large ones) gives
    the same levels; both directions run on these graphs."""
    rng = np.random.default_rng(77)
    graphs = [read_golden(f)[:2] for f in golden_files()]
    for i in range(8):
        n = int(rng.integers(1, 400))
        graphs.append((random_graph(rng, n, int(rng.integers(0, 8 * n + 1)), 1, 9,
                                    name=f"do{i}"), int(rng.integers(0, n))))
    hub = gen.workload("rmat14")
    graphs += [(gen.workload("er16k"), 0), (gen.workload("grid96"), 0),
               (hub, int(gen.pick_sources(hub, 1, stream=gen.STREAM["sources"])[0])),
               (gen.workload("rmat12"), 0), (path_graph(300, np.ones(299)), 0)]
    for hg, s in graphs:
        want = oracle.bfs(hg.n, hg.row_ptr, hg.col, s)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            say(f"[gpu] diropt {hg.name} n={hg.n}")
            for rep in range(2):
                got = g.bfs(s, gg.VERTEX, gg.DIROPT).cpu().numpy()
                assert g.stats()["rc"] == 0
                np.testing.assert_array_equal(got, want, err_msg=hg.name)
        finally:
            g.free()
    # without in-neighbours the schedule is refused
    hg = gen.workload("er300x900")
    g = gg.Graph(hg.n, hg.row_ptr, hg.col, hg.w)
    try:
        with pytest.raises(gg.GGError):
            g.bfs(0, gg.VERTEX, gg.DIROPT)
    finally:
        g.free()


def test_diropt_cc(gg):
    """CC with the per-round choice (edge sweeps while the frontier is large,
    then the worklist) gives the minimum-id labels, with and without the
    shortcut, at any grid size; on a skewed graph both forms run."""
    rng = np.random.default_rng(78)
    graphs = [read_golden(f)[0] for f in golden_files()]
    for i in range(8):
        n = int(rng.integers(1, 400))
        graphs.append(random_graph(rng, n, int(rng.integers(0, 3 * n + 1)), 1, 9, name=f"dc{i}"))
    graphs += [gen.workload("er16k"), gen.workload("grid96"), gen.workload("rmat14"),
               gen.workload("rmat12"), path_graph(300, np.ones(299)), gen.workload("rmat16")]
    for hg in graphs:
        want = oracle.cc(hg.n, hg.row_ptr, hg.col)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            caps = (0, 8, 7, 1) if hg.m >= 1 << 20 else (0, 3)
            for cap in caps:
                for flags in (0, gg.OPT_CC_NO_JUMP):
                    say(f"[gpu] cc diropt {hg.name} n={hg.n} m={hg.m} cap={cap} flags={flags}")
                    o = gg.make_opts(EDGE, gg.DIROPT, max_blocks=cap, flags=flags)
                    for rep in range(2):
                        got = g.cc(opts=o).cpu().numpy()[: hg.n]
                        assert g.stats()["rc"] == 0
                        np.testing.assert_array_equal(got, want, err_msg=hg.name)
            if hg.name in ("rmat14", "rmat16"):
                o = gg.make_opts(EDGE, gg.DIROPT, flags=gg.OPT_PROFILE)
                np.testing.assert_array_equal(g.cc(opts=o).cpu().numpy(), want)
                pr = g.profile()
                # round 0 reads every both-directions row; later rounds sweep
                # the stored edges or serve a worklist
                assert pr["round"]["edges_processed"] >= 2 * hg.m, pr
                assert pr["round"]["swept_edges"] > 0 or pr["round"]["vertices_processed"] > 0, pr
            # the vertex-based form pulls its dense rounds; AUTO takes the edge mode
            np.testing.assert_array_equal(g.cc(VERTEX, gg.DIROPT).cpu().numpy()[: hg.n], want)
            np.testing.assert_array_equal(g.cc(gg.MODE_AUTO, gg.DIROPT).cpu().numpy()[: hg.n],
                                          want)
        finally:
            g.free()
    # without the both-directions CSR the schedule is refused
    hg = gen.workload("er300x900")
    g = gg.Graph(hg.n, hg.row_ptr, hg.col, hg.w)
    try:
        with pytest.raises(gg.GGError):
            g.cc(EDGE, gg.DIROPT)
    finally:
        g.free()


def test_partitioned_edge_sweep(gg):
    """Graphs with >= 2^20 edges sweep a head-partitioned edge list, one part
    per die; any grid size gives the same result."""
    for name in ("rmat16", "grid724"):
        hg = gen.workload(name)
        assert hg.m >= 1 << 20
        s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
        want = expected(hg, s)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            for cap in (0, 8, 7, 24, 1):
                say(f"[gpu] partitioned edge sweep {name} cap={cap}")
                o = gg.make_opts(EDGE, SYNC, max_blocks=cap)
                np.testing.assert_array_equal(g.sssp(s, opts=o).cpu().numpy(), want["sssp"])
                np.testing.assert_array_equal(g.bfs(s, opts=o).cpu().numpy(), want["bfs"])
                np.testing.assert_array_equal(g.cc(opts=o).cpu().numpy(), want["cc"])
        finally:
            g.free()


def test_one_workspace_one_host_call_at_a_time(gg):
    """Host threads sharing a graph's default workspace: each call either
    runs alone on it and returns the exact result, or returns GG_EBUSY."""
    import threading

    import torch
    hg = gen.workload("rmat14")
    srcs = [int(x) for x in gen.pick_sources(hg, 8, stream=gen.STREAM["sources"])]
    want = {s: oracle.bfs(hg.n, hg.row_ptr, hg.col, s) for s in srcs}
    g = gg.Graph.from_host(hg, symmetrize=True)
    results, busy, errors = [], [], []
    lock = threading.Lock()

    def worker(k):
        st = torch.cuda.Stream()
        out = torch.empty(hg.n, dtype=torch.int32, device="cuda")
        for i in range(6):
            s = srcs[(k + i) % len(srcs)]
            try:
                g.bfs(s, out=out, stream=st)
                st.synchronize()
                with lock:
                    results.append((s, out.cpu().numpy().copy()))
            except gg.GGError as e:
                with lock:
                    (busy if e.code == -4 else errors).append(e)

    try:
        threads = [threading.Thread(target=worker, args=(k,)) for k in range(6)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        say(f"[gpu] shared workspace: {len(results)} calls ran, {len(busy)} busy")
        assert not errors, errors
        assert results
        for s, got in results:
            np.testing.assert_array_equal(got, want[s])
    finally:
        g.free()


def test_auto_never_picks_an_unavailable_variant(gg):
    """A tuning table may name the direction-optimizing BFS; on a graph without
    in-neighbours AUTO falls back instead of failing."""
    saved = gg.tune_get()
    try:
        gg.tune_set([dict(algo=1, size_class=8, skew_class=2, depth_class=-1, mode=0, sched=4,
                          mapping=3)])
        hg = gen.workload("rmat12")
        g = gg.Graph(hg.n, hg.row_ptr, hg.col, hg.w)  # no in-neighbours
        try:
            np.testing.assert_array_equal(g.bfs(0).cpu().numpy(),
                                          oracle.bfs(hg.n, hg.row_ptr, hg.col, 0))
            assert g.resolve(gg.ALGO_BFS).sched == gg.ASYNC
        finally:
            g.free()
    finally:
        gg.tune_set(saved)


def test_null_options_mean_auto(gg):
    """A NULL opts pointer resolves every field through the tuning table, as
    explicit AUTO fields do (a zeroed struct would name vertex-sync)."""
    import ctypes
    hg = gen.workload("rmat12")
    g = gg.Graph.from_host(hg, symmetrize=True)
    try:
        for algo in (gg.ALGO_SSSP, gg.ALGO_BFS, gg.ALGO_CC):
            a, b = gg.Opts(), gg.Opts()
            assert gg.lib().gg_resolve(g.handle, algo, None, ctypes.byref(a)) == 0
            assert gg.lib().gg_resolve(g.handle, algo, ctypes.byref(gg.make_opts()),
                                       ctypes.byref(b)) == 0
            assert (a.mode, a.sched, a.mapping, a.delta) == (b.mode, b.sched, b.mapping, b.delta)
        # the server runs its queries with the tuned variant
        import torch
        srv = gg.Server(2, 0)
        try:
            gid = srv.add_graph(gg.Graph.from_host(hg, symmetrize=True))
            out = torch.empty(hg.n, dtype=torch.int32, device="cuda")
            srv.submit(gid, gg.ALGO_SSSP, 0, out)
            while not srv.poll():
                pass
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(),
                                          oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, 0))
        finally:
            srv.free()
    finally:
        g.free()


def test_binding_loaded_before_torch(gg):
    """A process that loads the library before it imports torch gets one HIP
    runtime (torch's wheel carries its own): streams and device memory from
    torch work in libgg.so calls, here a traversal and a small batch."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1903_01665_amd import gg, gen\n"
        "gg.lib()\n"
        "import numpy as np, torch, oracle\n"
        "hg = gen.workload('er300x900')\n"
        "g = gg.Graph.from_host(hg)\n"
        "d = g.sssp(0).cpu().numpy()\n"
        "assert np.array_equal(d, oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, 0))\n"
        "g.free()\n"
        "b = gg.Batch([(0, hg, 0), (1, hg, 5)])\n"
        "out = torch.empty(b.info()['total_n'], dtype=torch.int32, device='cuda')\n"
        "b.run(out); torch.cuda.synchronize()\n"
        "got = out.cpu().numpy(); off = b.offsets()\n"
        "assert np.array_equal(got[off[0]:off[0] + hg.n], d)\n"
        "assert np.array_equal(got[off[1]:off[1] + hg.n], oracle.bfs(hg.n, hg.row_ptr, hg.col, 5))\n"
        "b.free()\n"
        "print('one runtime ok', flush=True)\n" % root)
    say("[gpu] library loaded before torch (subprocess)")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "one runtime ok" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]


def test_auto_carries_the_tuned_schedule_knobs(gg):
    """AUTO resolution takes the table entry's passes of local expansion,
    long-row threshold and bucket width with its schedule (and an explicit
    schedule keeps the caller's), and the traversal it resolves to is exact."""
    hg = gen.workload("rmat12")
    s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
    g = gg.Graph.from_host(hg, symmetrize=True)
    saved = gg.tune_get()
    try:
        sc, kc, dc = g.graph_class()
        gg.tune_set([dict(algo=0, size_class=sc, skew_class=kc, depth_class=-1, mode=gg.VERTEX,
                          sched=gg.NEARFAR, mapping=3, delta_eighths=3, hops=4, far_degree=40),
                     dict(algo=1, size_class=sc, skew_class=kc, depth_class=-1, mode=gg.VERTEX,
                          sched=gg.ASYNC, mapping=3, hops=6)])
        o = g.resolve(gg.ALGO_SSSP)
        avg_w = float(hg.w.mean())
        assert (o.mode, o.sched, o.mapping, o.hops, o.far_degree) == (gg.VERTEX, gg.NEARFAR, 3,
                                                                     4, 40)
        assert o.delta == max(1, int(3 * avg_w / 8))
        assert (g.resolve(gg.ALGO_BFS).sched, g.resolve(gg.ALGO_BFS).hops) == (gg.ASYNC, 6)
        # an explicit schedule keeps the caller's knobs
        e = g.resolve(gg.ALGO_SSSP, gg.make_opts(gg.VERTEX, gg.ASYNC, 3, hops=2))
        assert (e.sched, e.hops, e.far_degree) == (gg.ASYNC, 2, 0)
        say(f"[gpu] auto knobs {hg.name} class={(sc, kc, dc)}")
        np.testing.assert_array_equal(g.sssp(s).cpu().numpy(),
                                      oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s))
        np.testing.assert_array_equal(g.bfs(s).cpu().numpy(),
                                      oracle.bfs(hg.n, hg.row_ptr, hg.col, s))
    finally:
        gg.tune_set(saved)
        g.free()


def test_unionfind_cc(gg):
    """CC through the union-find Set (sampled links, the giant root, the rest
    linked): the smallest-id labels on graphs of every shape -- empty rows,
    isolated vertices, many small components, a path (high diameter), hubs,
    self-loops and parallel edges -- in the caller's and the renumbered
    order, and at grid caps that make every block loop."""
    rng = np.random.default_rng(5150)
    graphs = [read_golden(f)[0] for f in golden_files()]
    for i in range(10):
        n = int(rng.integers(1, 500))
        graphs.append(random_graph(rng, n, int(rng.integers(0, 2 * n + 1)), 1, 9, name=f"uf{i}"))
    graphs += [gen.workload("er16k"), gen.workload("grid96"), gen.workload("rmat14"),
               path_graph(3000, np.ones(2999)), star(200, [[1, 2]] * 200),
               random_graph(rng, 5000, 1200, 1, 9, name="sparse5000")]
    for hg in graphs:
        want = oracle.cc(hg.n, hg.row_ptr, hg.col)
        for renumber in (False, True):
            g = gg.Graph.from_host(hg, symmetrize=True, renumber=renumber)
            try:
                for cap in (0, 1, 7):
                    say(f"[gpu] unionfind cc {hg.name} n={hg.n} renumber={renumber} cap={cap}")
                    o = gg.make_opts(VERTEX, gg.UNIONFIND, BALANCED, max_blocks=cap)
                    got = g.cc(opts=o).cpu().numpy()
                    st = g.stats()
                    assert st["rc"] == 0 and st["iterations"] == 4, st
                    np.testing.assert_array_equal(got, want, err_msg=f"{hg.name} cap={cap}")
                with pytest.raises(gg.GGError):
                    g.bfs(0, opts=gg.make_opts(VERTEX, gg.UNIONFIND, BALANCED))
            finally:
                g.free()
    # without the both-directions CSR the schedule cannot run
    hg = gen.workload("er300x900")
    g = gg.Graph(hg.n, hg.row_ptr, hg.col, hg.w)
    try:
        with pytest.raises(gg.GGError):
            g.cc(opts=gg.make_opts(VERTEX, gg.UNIONFIND, BALANCED))
    finally:
        g.free()


def _rows_of(rng, n, degs, wlo=1, whi=9, name="rows"):
    """Vertex v with degs[v] out-edges to random heads."""
    degs = np.asarray(degs, np.int64)
    src = np.repeat(np.arange(n, dtype=np.int32), degs)
    dst = rng.integers(0, n, size=len(src), dtype=np.int64).astype(np.int32)
    w = rng.integers(wlo, whi + 1, size=len(src), dtype=np.int64).astype(np.int32)
    return gen.from_edges(n, src, dst, w, name=name)


def test_local_short_rows(gg):
    """Local-expansion passes over lists whose rows all have at most five
    edges take one lane per row; lists with a longer row take the balanced
    walk.  Graphs with every row short, and with row lengths around the
    limit (so that a traversal switches between the two), give the oracle's
    distances, levels and labels."""
    rng = np.random.default_rng(55)
    graphs = [_rows_of(rng, 3000, np.full(3000, d), name=f"deg{d}") for d in (1, 2, 4, 5)]
    graphs.append(_rows_of(rng, 4000, rng.integers(0, 9, size=4000), name="deg0to8"))
    graphs.append(_rows_of(rng, 4000, rng.choice([4, 5, 6], size=4000, p=[0.9, 0.08, 0.02]),
                           wlo=1, whi=1000, name="deg456"))
    graphs.append(gen.workload("grid96"))
    for hg in graphs:
        s = int(rng.integers(0, hg.n))
        want = expected(hg, s)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            for algo, sched, delta, hops, fl in (
                    ("sssp", gg.NEARFAR, 0, 64, gg.OPT_LISTS_DIRECT),
                    ("sssp", gg.NEARFAR, 0, 64, gg.OPT_LISTS_CHECKED),
                    ("sssp", gg.NEARFAR, 3, 8, 0), ("sssp", gg.ASYNC, 0, 8, 0),
                    ("bfs", gg.ASYNC, 0, 8, 0), ("cc", gg.ASYNC, 0, 4, 0)):
                say(f"[gpu] short rows {hg.name} n={hg.n} {algo} sched={sched} hops={hops} "
                    f"flags={fl}")
                o = gg.make_opts(gg.VERTEX, sched, gg.MAP_BALANCED, delta=delta, hops=hops,
                                 flags=fl)
                got = (g.cc(opts=o) if algo == "cc" else getattr(g, algo)(s, opts=o))
                assert g.stats()["rc"] == 0
                np.testing.assert_array_equal(got.cpu().numpy()[: hg.n], want[algo],
                                              err_msg=f"{hg.name} {algo} hops={hops}")
        finally:
            g.free()


def test_cc_plain_sweeps_under_contention(gg):
    """Plain CC edge sweeps lower labels with stores: concurrent stores into
    one label can lose the lower value, which a later sweep restores.  Hubs
    with the largest ids and tens of thousands of smaller neighbours make
    every lane of a sweep store into the same labels; the labels must still
    be the smallest id of each component, on every repetition, with the
    both-directions arrays (head stores only) and without them (both ends)."""
    rng = np.random.default_rng(77)
    n = 40000
    hubs = np.arange(n - 8, n, dtype=np.int32)  # eight hubs with the largest ids
    leaves = np.arange(0, n - 8, dtype=np.int32)
    src = np.concatenate([leaves, leaves[::-1]])
    dst = np.concatenate([hubs[leaves % 8], hubs[(leaves * 7 + 3) % 8]])
    stars = gen.from_edges(n, src, dst, np.ones(len(src), np.int32), name="hubs")
    # two components: even and odd vertices, each a random graph in one direction
    m = 200000
    a = rng.integers(0, n // 2, size=m).astype(np.int32)
    b = rng.integers(0, n // 2, size=m).astype(np.int32)
    par = rng.integers(0, 2, size=m).astype(np.int32)
    split = gen.from_edges(n, 2 * a + par, 2 * b + par, np.ones(m, np.int32), name="evenodd")
    def both_ways(hg):
        # the edges in both directions, uploaded as a symmetric graph: the
        # sweeps store into head labels only
        s0 = np.repeat(np.arange(hg.n, dtype=np.int32), np.diff(hg.row_ptr))
        c0 = np.asarray(hg.col, np.int32)
        return gen.from_edges(hg.n, np.concatenate([s0, c0]), np.concatenate([c0, s0]),
                              np.ones(2 * len(c0), np.int32), name=hg.name + "-sym",
                              symmetric=True)

    for hg in (stars, split, both_ways(stars), both_ways(split)):
        want = oracle.cc(hg.n, hg.row_ptr, hg.col)
        for sym in ((True,) if hg.symmetric else (True, False)):
            g = gg.Graph.from_host(hg, symmetrize=sym)
            try:
                for cap in (0, 7, 64):
                    for rep in range(5):
                        say(f"[gpu] cc plain sweeps {hg.name} symmetrize={sym} cap={cap} "
                            f"rep={rep}")
                        o = gg.make_opts(EDGE, SYNC, 0, max_blocks=cap)
                        got = g.cc(opts=o).cpu().numpy()
                        assert g.stats()["rc"] == 0
                        np.testing.assert_array_equal(got, want,
                                                      err_msg=f"{hg.name} sym={sym} cap={cap}")
            finally:
                g.free()
