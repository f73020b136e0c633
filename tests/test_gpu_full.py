"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses (AUTO variant) and in every mode/schedule combination.

The oracle finishes these sizes in seconds, so every element is compared;
the certificates are checked on the GPU output as well.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1903_01665_amd import gen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

COMBOS = [("auto", None), ("vertex-sync", (0, 0, 3)), ("vertex-async", (0, 1, 3)),
          ("edge-sync", (1, 0, 0)), ("edge-async", (1, 1, 0))]
# per-round schedules: (name, variant, algorithms it applies to)
PER_ROUND = [("vertex-diropt", (0, 4, 3), ("sssp", "bfs", "cc")),
             ("edge-diropt", (1, 4, 0), ("cc",)), ("unionfind", (0, 5, 3), ("cc",))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_full(name, combos, mapping_extra=()):
    from paper_1903_01665_amd import gg
    hg = gen.workload(name)
    s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0]) if name.startswith("rmat") \
        else 0
    want = {"sssp": oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s),
            "bfs": oracle.bfs(hg.n, hg.row_ptr, hg.col, s),
            "cc": oracle.cc(hg.n, hg.row_ptr, hg.col)}
    g = gg.Graph.from_host(hg, symmetrize=True, transpose=True)
    try:
        runs = [(c, v, ("sssp", "bfs", "cc")) for c, v in list(combos) + list(mapping_extra)]
        for cname, v, algos in runs + PER_ROUND:
            o = gg.make_opts(*v) if v else gg.make_opts()
            for algo in algos:
                say(f"[gpu-full] {name} {algo} {cname}")
                out = g.cc(opts=o) if algo == "cc" else getattr(g, algo)(s, opts=o)
                got = out.cpu().numpy()
                st = g.stats()
                assert st["rc"] == 0, st
                bad = np.flatnonzero(got != want[algo])
                assert bad.size == 0, (name, algo, cname, bad.size, int(bad[0]))
                if algo == "sssp":
                    assert oracle.check_sssp(hg.n, hg.row_ptr, hg.col, hg.w, s, got) == 0
                elif algo == "bfs":
                    assert oracle.check_bfs(hg.n, hg.row_ptr, hg.col, s, got) == 0
                else:
                    assert oracle.check_cc(hg.n, hg.row_ptr, hg.col, got) == 0
    finally:
        g.free()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()


def test_rmat22_all_variants():
    run_full("rmat22", COMBOS, [("vertex-sync-thread", (0, 0, 1)), ("vertex-async-wave", (0, 1, 2))])


def test_grid4096_all_variants():
    run_full("grid4096", COMBOS)


def test_er23_all_variants():
    run_full("er23", COMBOS)


@pytest.mark.parametrize("name", ["rmat22", "grid4096", "er23"])
def test_msf_full_size(name):
    """The forest on the full benchmark graphs, edge by edge."""
    import torch

    import oracle
    from paper_1903_01665_amd import gg
    hg = gen.workload(name)
    want, total = oracle.msf(hg.n, hg.row_ptr, hg.col, hg.w)
    g = gg.Graph.from_host(hg)
    try:
        sel, tw, ne = g.msf()
        torch.cuda.synchronize()
        got = sel.cpu().numpy()
        assert np.array_equal(got, want), (name, int((got != want).sum()))
        assert tw == total and ne == int(want.sum())
    finally:
        g.free()
