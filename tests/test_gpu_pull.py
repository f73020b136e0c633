"""Pull rounds (the DSL's innbrs iterator, Sec. 2) of the per-round schedule:
SSSP (vertex-based, over the weighted in-edge CSR) and CC (vertex-based, over
the both-directions rows) pull their dense rounds and push the sparse ones;
every result is bit-exact against the oracle, and the pull rounds do run."""
import sys

import numpy as np
import pytest

import oracle
from helpers import INF, golden_files, path_graph, random_graph, read_golden, star
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu

VERTEX, EDGE = 0, 1


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


def graphs(seed):
    rng = np.random.default_rng(seed)
    out = [read_golden(f)[:2] for f in golden_files()]
    for i in range(8):
        n = int(rng.integers(1, 400))
        out.append((random_graph(rng, n, int(rng.integers(0, 8 * n + 1)), 0, 9, name=f"p{i}"),
                    int(rng.integers(0, n))))
    # hubs: heavy in-rows and out-rows (chunked in both directions)
    src, dst = [], []
    for hub, deg in [(0, 3000), (1, 700), (65, 1500)]:
        src += [hub] * deg
        dst += list(rng.integers(0, 4000, size=deg))
        src += list(rng.integers(0, 4000, size=deg))
        dst += [hub + 2] * deg
    src += list(rng.integers(0, 4000, size=6000))
    dst += list(rng.integers(0, 4000, size=6000))
    out.append((gen.from_edges(4000, src, dst, rng.integers(1, 50, size=len(src)), name="hubs"),
                0))
    hub = gen.workload("rmat14")
    out += [(hub, int(gen.pick_sources(hub, 1, stream=gen.STREAM["sources"])[0])),
            (gen.workload("er16k"), 0), (gen.workload("grid96"), 0),
            (gen.workload("rmat16"), 1), (path_graph(300, np.arange(1, 300) % 5 + 1), 0),
            (star(300, [[4, 9, 2]] * 300), 0)]
    # weights across the INF line
    w = rng.integers(2**29, INF, size=hub.m, dtype=np.int64).astype(np.int32)
    big = gen.from_edges(hub.n, np.repeat(np.arange(hub.n, dtype=np.int32),
                                          np.diff(hub.row_ptr)), hub.col, w, name="rmat14-big")
    out.append((big, out[-6][1]))
    return out


def test_sssp_pull_rounds(gg):
    pulled_somewhere = False
    for hg, s in graphs(1903):
        want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
        g = gg.Graph.from_host(hg, transpose=True)
        try:
            for cap in (0, 7):
                say(f"[gpu] sssp pull {hg.name} n={hg.n} m={hg.m} cap={cap}")
                o = gg.make_opts(VERTEX, gg.DIROPT, gg.MAP_BALANCED, max_blocks=cap,
                                 flags=gg.OPT_PROFILE)
                got = g.sssp(s, opts=o).cpu().numpy()
                assert g.stats()["rc"] == 0
                np.testing.assert_array_equal(got, want, err_msg=f"{hg.name} cap={cap}")
                pulled_somewhere |= g.profile()["round"]["swept_edges"] > 0
            # AUTO with an explicit per-round schedule takes the vertex mode
            np.testing.assert_array_equal(g.sssp(s, gg.MODE_AUTO, gg.DIROPT).cpu().numpy(), want)
        finally:
            g.free()
    assert pulled_somewhere
    # without the in-edge CSR the schedule is refused
    hg = gen.workload("er300x900")
    g = gg.Graph.from_host(hg, symmetrize=True)
    try:
        with pytest.raises(gg.GGError) as e:
            g.sssp(0, VERTEX, gg.DIROPT)
        assert e.value.code == -5
        with pytest.raises(gg.GGError):
            g.sssp(0, EDGE, gg.DIROPT)
    finally:
        g.free()


def test_cc_pull_rounds(gg):
    pulled_somewhere = False
    for hg, _ in graphs(1665):
        want = oracle.cc(hg.n, hg.row_ptr, hg.col)
        g = gg.Graph.from_host(hg, symmetrize=True)
        try:
            for cap in (0, 7):
                for flags in (0, gg.OPT_CC_NO_JUMP):
                    say(f"[gpu] cc pull {hg.name} n={hg.n} m={hg.m} cap={cap} flags={flags}")
                    o = gg.make_opts(VERTEX, gg.DIROPT, gg.MAP_BALANCED, max_blocks=cap,
                                     flags=flags | gg.OPT_PROFILE)
                    for rep in range(2):
                        got = g.cc(opts=o).cpu().numpy()[: hg.n]
                        assert g.stats()["rc"] == 0
                        np.testing.assert_array_equal(got, want, err_msg=hg.name)
                    pulled_somewhere |= g.profile()["round"]["swept_edges"] > 0
        finally:
            g.free()
    assert pulled_somewhere


def test_auto_falls_back_without_the_in_edge_csr(gg):
    """A tuning table may name SSSP's per-round schedule; on a graph uploaded
    without GG_TRANSPOSE, AUTO falls back to the worklist."""
    saved = gg.tune_get()
    try:
        hg = gen.workload("rmat12")
        g = gg.Graph.from_host(hg, symmetrize=True)
        sc, kc, dc = g.graph_class()
        gg.tune_set([dict(algo=0, size_class=sc, skew_class=kc, depth_class=-1, mode=0,
                          sched=gg.DIROPT, mapping=3)])
        try:
            assert g.resolve(gg.ALGO_SSSP).sched == gg.ASYNC
            np.testing.assert_array_equal(g.sssp(5).cpu().numpy(),
                                          oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, 5))
        finally:
            g.free()
        g = gg.Graph.from_host(hg, transpose=True)
        try:
            assert g.resolve(gg.ALGO_SSSP).sched == gg.DIROPT
            np.testing.assert_array_equal(g.sssp(5).cpu().numpy(),
                                          oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, 5))
        finally:
            g.free()
    finally:
        gg.tune_set(saved)
