"""Planted mistakes in a copy of the oracle must be caught by its pins.

Each mutant is a plausible slip (a dropped term, a wrong index, a transposed
operand, a wrong comparison) applied to the text of oracle.c, compiled on the
CPU into a temporary library, and run against scipy and the closed forms.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from helpers import random_graph
from test_oracle import scipy_cc, scipy_sssp
from test_oracle_msf import scipy_msf_weight

pytestmark = pytest.mark.timeout(120)

ORACLE_C = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                        "oracle.c")

MUTANTS = {
    # SSSP: weight dropped, relaxation along the reversed edge, the tail's
    # distance stored instead of the candidate, stale-entry test off by one.
    # Every mutant still terminates.  (A broken heap order is not a
    # mistake here: every improvement is pushed again, so pop order changes
    # only the running time of this lazy-deletion form, not its result.)
    "sssp_drop_weight": ("int64_t nd = it.d + (int64_t)w[e];", "int64_t nd = it.d + 1;"),
    "sssp_transposed": ("int32_t v = col[e];\n            int64_t nd", "int32_t v = u;\n            int64_t nd"),
    "sssp_stores_tail": ("D[v] = nd;\n                rc = heap_push(&h, nd, v);",
                         "D[v] = it.d;\n                rc = heap_push(&h, nd, v);"),
    "sssp_stale_test": ("if (it.d > D[u]) continue;", "if (it.d >= D[u]) continue;"),
    # BFS: level not incremented, source level wrong
    "bfs_no_increment": ("dist[v] = dist[u] + 1;", "dist[v] = dist[u];"),
    "bfs_source_level": ("    dist[source] = 0;\n    queue[tail++] = source;\n    while (head < tail) {\n        int32_t u = queue[head++];\n        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {\n            int32_t v = col[e];\n            if (dist[v] == ORACLE_INF) {",
                         "    dist[source] = 1;\n    queue[tail++] = source;\n    while (head < tail) {\n        int32_t u = queue[head++];\n        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {\n            int32_t v = col[e];\n            if (dist[v] == ORACLE_INF) {"),
    # CC: max instead of min id, union skipped for one side
    "cc_max_label": ("if (v < minid[r]) minid[r] = v;", "if (minid[r] == n || v > minid[r]) minid[r] = v;"),
    "cc_self_union": ("int32_t a = uf_find(parent, u), b = uf_find(parent, col[e]);",
                      "int32_t a = uf_find(parent, u), b = uf_find(parent, u);"),
    # MSF: edge index dropped from the key, order reversed, union skipped,
    # one end of the edge taken twice
    "msf_key_no_index": ("return ((uint64_t)w[e] << 32) | (uint64_t)e;",
                         "return ((uint64_t)w[e] << 32);"),
    "msf_descending": ("return x < y ? -1 : x > y;", "return x > y ? -1 : x < y;"),
    "msf_no_union": ("parent[b] = a;\n        size[a] += size[b];\n        in_msf[e] = 1;",
                     "size[a] += size[b];\n        in_msf[e] = 1;"),
    "msf_same_end": ("int32_t a = uf_find(parent, src[e]), b = uf_find(parent, col[e]);",
                     "int32_t a = uf_find(parent, src[e]), b = uf_find(parent, src[e]);"),
}


def _build_mutant(tmp_path, name, old, new):
    text = open(ORACLE_C).read()
    assert text.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / f"{name}.c"
    src.write_text(text.replace(old, new, 1))
    hdr_dir = os.path.dirname(ORACLE_C)
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", f"-I{hdr_dir}", str(src), "-o", str(so)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    for f in ("oracle_sssp", "oracle_bfs", "oracle_cc", "oracle_msf"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pins_fail(lib) -> bool:
    """True when some pin disagrees with the mutant on a seeded case set."""
    rng = np.random.default_rng(5)
    for i in range(60):
        n = int(rng.integers(2, 30))
        g = random_graph(rng, n, int(rng.integers(n, 4 * n)), 1, 9)
        s = int(rng.integers(0, n))
        row, col, w = g.row_ptr, g.col, g.w
        out = np.empty(n, np.int32)
        if lib.oracle_sssp(n, _p(row), _p(col), _p(w), s, _p(out)) != 0 or \
                not np.array_equal(out, scipy_sssp(g, s)):
            return True
        if lib.oracle_bfs(n, _p(row), _p(col), s, _p(out)) != 0 or \
                not np.array_equal(out, scipy_sssp(g, s, unit=True)):
            return True
        if lib.oracle_cc(n, _p(row), _p(col), _p(out)) != 0 or \
                not np.array_equal(out, scipy_cc(g)):
            return True
    # MSF against exhaustive search (tiny graphs) and scipy's weight
    for i in range(60):
        n = int(rng.integers(2, 9))
        g = random_graph(rng, n, int(rng.integers(1, 15)), 1, 4)
        sel = np.zeros(max(g.m, 1), np.uint8)
        total = ctypes.c_int64()
        if lib.oracle_msf(n, _p(g.row_ptr), _p(g.col), _p(g.w), _p(sel),
                          ctypes.byref(total)) != 0:
            return True
        if not np.array_equal(sel[: g.m], oracle.msf_brute(g.n, g.row_ptr, g.col, g.w)):
            return True
    for i in range(20):
        n = int(rng.integers(2, 200))
        g = random_graph(rng, n, int(rng.integers(n, 4 * n)), 1, 99)
        sel = np.zeros(max(g.m, 1), np.uint8)
        total = ctypes.c_int64()
        if lib.oracle_msf(n, _p(g.row_ptr), _p(g.col), _p(g.w), _p(sel),
                          ctypes.byref(total)) != 0 or total.value != scipy_msf_weight(g):
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    assert _pins_fail(lib), f"pins did not catch mutant {name}"


def test_unmutated_copy_passes(tmp_path):
    lib = _build_mutant(tmp_path, "identity", "#include", "#include")
    assert not _pins_fail(lib)
