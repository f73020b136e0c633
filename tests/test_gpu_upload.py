"""Upload: device-resident input (GG_INPUT_ON_DEVICE) is checked on the
device (column range, weight sign) and gives the same graph as host input;
the head-partitioned edge list is split on the device in CSR order; the
in-edge CSR (GG_TRANSPOSE) and both-directions CSR come from one in-degree
count.  Every result is checked against the oracle."""
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


def upload_dev(gg, hg, flags, col=None, w=None):
    import torch
    row = torch.as_tensor(hg.row_ptr, device="cuda")
    col = torch.as_tensor(hg.col if col is None else col, device="cuda")
    w = torch.as_tensor(hg.w if w is None else w, device="cuda")
    torch.cuda.synchronize()
    h = ctypes.c_void_p()
    rc = gg.lib().gg_graph_upload(hg.n, hg.m, ctypes.c_void_p(row.data_ptr()),
                                  ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                  flags | gg.INPUT_ON_DEVICE,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.byref(h))
    return rc, h


def wrap(gg, h, n, m):
    g = gg.Graph.__new__(gg.Graph)
    g.handle, g.n, g.m = h, n, m
    return g


@pytest.mark.parametrize("name", ["rmat14", "rmat16", "grid96"])
def test_device_input_matches_the_oracle(gg, name):
    hg = gen.workload(name)
    s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
    rc, h = upload_dev(gg, hg, gg.SYMMETRIZE | gg.TRANSPOSE)
    assert rc == 0
    g = wrap(gg, h, hg.n, hg.m)
    try:
        say(f"[gpu] device-input upload {name} n={hg.n} m={hg.m}")
        want = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
        for o in (gg.make_opts(), gg.make_opts(gg.EDGE, gg.SYNC),
                  gg.make_opts(gg.VERTEX, gg.DIROPT, gg.MAP_BALANCED)):
            np.testing.assert_array_equal(g.sssp(s, opts=o).cpu().numpy(), want)
        np.testing.assert_array_equal(g.cc(gg.EDGE, gg.SYNC).cpu().numpy(),
                                      oracle.cc(hg.n, hg.row_ptr, hg.col))
        np.testing.assert_array_equal(g.bfs(s, gg.EDGE, gg.SYNC).cpu().numpy(),
                                      oracle.bfs(hg.n, hg.row_ptr, hg.col, s))
        # the near-far default width comes from the mean weight the device
        # computed: the same as from a host upload's
        nf = gg.make_opts(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED)
        gh = gg.Graph.from_host(hg)
        try:
            assert g.resolve(gg.ALGO_SSSP, nf).delta == gh.resolve(gg.ALGO_SSSP, nf).delta
        finally:
            gh.free()
    finally:
        g.free()


def test_device_input_is_checked(gg):
    hg = gen.workload("er300x900")
    bad_col = hg.col.copy()
    bad_col[123] = hg.n
    rc, _ = upload_dev(gg, hg, 0, col=bad_col)
    assert rc == -1
    bad_col[123] = -1
    rc, _ = upload_dev(gg, hg, 0, col=bad_col)
    assert rc == -1
    bad_w = hg.w.copy()
    bad_w[7] = -5
    rc, _ = upload_dev(gg, hg, 0, w=bad_w)
    assert rc == -1
    rc, h = upload_dev(gg, hg, 0)
    assert rc == 0
    g = wrap(gg, h, hg.n, hg.m)
    np.testing.assert_array_equal(g.sssp(3).cpu().numpy(),
                                  oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, 3))
    g.free()
