"""The C-ABI library loads and exports every symbol include/gg.h declares;
host-side argument checks reject bad input before any device work (no GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gg.h")
LIB = os.path.join(ROOT, "paper_1903_01665_amd", "libgg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\**\s*(gg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def libgg():
    if not os.path.exists(LIB):
        pytest.fail("libgg.so is not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ["gg_graph_upload", "gg_sssp", "gg_bfs", "gg_cc", "gg_graph_free"]:
        assert f in fns
    from paper_1903_01665_amd import gg
    assert sorted(gg.EXPORTS) == fns


def test_library_exports_every_declared_symbol(libgg):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        getattr(libgg, f)


def test_version_and_status_strings(libgg):
    from paper_1903_01665_amd import gg
    assert gg.lib().gg_version() == 1
    assert gg.status_str(0) == "GG_OK"
    assert gg.status_str(-1) == "GG_EINVAL"
    assert gg.status_str(-6) == "GG_ETIMEOUT"


def _upload(n, m, row, col, w=None, flags=0):
    from paper_1903_01665_amd import gg
    h = ctypes.c_void_p()
    row = np.ascontiguousarray(row, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    pw = None
    if w is not None:
        w = np.ascontiguousarray(w, np.int32)
        pw = w.ctypes.data_as(ctypes.c_void_p)
    return gg.lib().gg_graph_upload(n, m, row.ctypes.data_as(ctypes.c_void_p),
                                    col.ctypes.data_as(ctypes.c_void_p), pw, flags, None,
                                    ctypes.byref(h))


def test_upload_rejects_bad_input_on_the_host():
    EINVAL = -1
    assert _upload(0, 0, [0], [0]) == EINVAL                       # n < 1
    assert _upload(3, -1, [0, 0, 0, 0], [0]) == EINVAL             # m < 0
    assert _upload(3, 2, [0, 2, 1, 2], [0, 1]) == EINVAL           # row_ptr decreases
    assert _upload(3, 2, [1, 1, 2, 2], [0, 1]) == EINVAL           # row_ptr[0] != 0
    assert _upload(3, 2, [0, 1, 2, 3], [0, 1]) == EINVAL           # row_ptr[n] != m
    assert _upload(3, 2, [0, 1, 2, 2], [0, 3]) == EINVAL           # column out of range
    assert _upload(3, 2, [0, 1, 2, 2], [0, 1], [4, -2]) == EINVAL  # negative weight
    assert _upload(3, 1 << 31, [0, 0, 0, 0], [0]) == EINVAL        # m too large


def test_null_handles_are_rejected():
    from paper_1903_01665_amd import gg
    L = gg.lib()
    assert L.gg_graph_free(None) == -1
    assert L.gg_sssp(None, 0, 0, 0, None, None) == -1
    assert L.gg_cc(None, 0, 0, None, None) == -1
    assert L.gg_last_stats(None, None, None) == -1


def test_binding_loads_torch_first():
    """torch's HIP runtime must be the one in the process before libgg.so is
    loaded (see gg.lib)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1903_01665_amd import gg\n"
            "assert 'torch' not in sys.modules\n"
            "gg.lib()\n"
            "assert 'torch' in sys.modules\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
