"""CPU oracle for the traversal results -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never does, and it shares
no code with it.  The C routines (``oracle.c``) compute the plain definitions
that the paper's fixpoint methods reach:

* SSSP  shortest-path distance from the source, clamped to INF = 2^31-1
        (Algorithms 1-2 relax t.dist to p.dist + weight along every edge until
        nothing changes);
* BFS   hop distance (Algorithm 3's level-synchronous fixpoint);
* CC    smallest vertex id in the component of the graph with every edge taken
        both ways (Sec. 4.1 names the algorithm, Sec. 2 the union-find Set);
* MSF   the minimum spanning forest of the graph with every stored edge taken
        as undirected, edge keys (weight, edge index) so that it is unique
        (Sec. 4.1 names MST); Kruskal with the union-find Set.

Each returns a new int32 numpy array.  Brute-force variants and O(n+m)
certificates are exposed for pinning and for checking full-size outputs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
INF = 2**31 - 1
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(LIB_PATH)
        i32, vp = ctypes.c_int32, ctypes.c_void_p
        sigs = {
            "oracle_sssp": [i32, vp, vp, vp, i32, vp],
            "oracle_bfs": [i32, vp, vp, i32, vp],
            "oracle_cc": [i32, vp, vp, vp],
            "oracle_sssp_floyd_warshall": [i32, vp, vp, vp, i32, vp],
            "oracle_sssp_bellman_ford": [i32, vp, vp, vp, i32, vp],
            "oracle_cc_warshall": [i32, vp, vp, vp],
            "oracle_check_sssp": [i32, vp, vp, vp, i32, vp],
            "oracle_check_cc": [i32, vp, vp, vp],
            "oracle_msf": [i32, vp, vp, vp, vp, vp],
            "oracle_msf_brute": [i32, vp, vp, vp, vp],
            "oracle_check_msf": [i32, vp, vp, vp, vp],
        }
        for name, args in sigs.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col, w=None):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if len(col) == 0:
        col = np.zeros(1, np.int32)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.int32)
        if len(w) == 0:
            w = np.zeros(1, np.int32)
    return row_ptr, col, w


def _run(name, n, row_ptr, col, w, extra):
    row_ptr, col, w = _csr(row_ptr, col, w)
    out = np.empty(n, np.int32)
    args = [n, _p(row_ptr), _p(col)]
    if w is not None or name in ("oracle_sssp", "oracle_sssp_floyd_warshall",
                                 "oracle_sssp_bellman_ford"):
        args.append(_p(w))
    args += list(extra) + [_p(out)]
    rc = getattr(_load(), name)(*args)
    if rc != 0:
        raise ValueError(f"{name} returned {rc}")
    return out


def sssp(n, row_ptr, col, w, source):
    return _run("oracle_sssp", n, row_ptr, col, w, [source])


def bfs(n, row_ptr, col, source):
    return _run("oracle_bfs", n, row_ptr, col, None, [source])


def cc(n, row_ptr, col):
    return _run("oracle_cc", n, row_ptr, col, None, [])


def sssp_floyd_warshall(n, row_ptr, col, w, source):
    return _run("oracle_sssp_floyd_warshall", n, row_ptr, col, w, [source])


def sssp_bellman_ford(n, row_ptr, col, w, source):
    return _run("oracle_sssp_bellman_ford", n, row_ptr, col, w, [source])


def cc_warshall(n, row_ptr, col):
    return _run("oracle_cc_warshall", n, row_ptr, col, None, [])


def check_sssp(n, row_ptr, col, w, source, dist) -> int:
    """0 when ``dist`` is the exact SSSP result (w=None: BFS levels)."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    dist = np.ascontiguousarray(dist, dtype=np.int32)
    return _load().oracle_check_sssp(n, _p(row_ptr), _p(col), _p(w), source, _p(dist))


def check_bfs(n, row_ptr, col, source, dist) -> int:
    return check_sssp(n, row_ptr, col, None, source, dist)


def check_cc(n, row_ptr, col, label) -> int:
    row_ptr, col, _ = _csr(row_ptr, col)
    label = np.ascontiguousarray(label, dtype=np.int32)
    return _load().oracle_check_cc(n, _p(row_ptr), _p(col), _p(label))


def msf(n, row_ptr, col, w):
    """(in_msf uint8[m], total weight) of the minimum spanning forest."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    m = int(row_ptr[-1])
    out = np.zeros(max(m, 1), np.uint8)
    total = ctypes.c_int64()
    rc = _load().oracle_msf(n, _p(row_ptr), _p(col), _p(w), _p(out), ctypes.byref(total))
    if rc != 0:
        raise ValueError(f"oracle_msf returned {rc}")
    return out[:m], int(total.value)


def msf_brute(n, row_ptr, col, w):
    row_ptr, col, w = _csr(row_ptr, col, w)
    m = int(row_ptr[-1])
    out = np.zeros(max(m, 1), np.uint8)
    rc = _load().oracle_msf_brute(n, _p(row_ptr), _p(col), _p(w), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_msf_brute returned {rc}")
    return out[:m]


def check_msf(n, row_ptr, col, w, in_msf) -> int:
    """0 when ``in_msf`` marks exactly the minimum spanning forest."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    sel = np.zeros(max(len(in_msf), 1), np.uint8)
    sel[: len(in_msf)] = np.asarray(in_msf, dtype=np.uint8)
    return _load().oracle_check_msf(n, _p(row_ptr), _p(col), _p(w), _p(sel))
