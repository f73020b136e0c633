"""Seeded synthetic graph inputs (host side, numpy arrays).

This module only synthesises inputs: random numbers, edge lists and their
stable CSR sort.  It holds no traversal arithmetic, so both the GPU path and
the CPU oracle may consume what it makes.  The C core is ``ggen.c`` (built into
``libggen.so`` next to this file).

Workload recipes (sizes, distributions and the readings that fix the details
the paper leaves open) live in :func:`workload`.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libggen.so")
_lib = None

MASTER_SEED = 0x190301665
INF = 2**31 - 1

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.ggen_raw.argtypes = [u64, u64, u64, i64, vp]
    lib.ggen_uniform.argtypes = [i32, i64, i32, i32, u64, u64, vp, vp, vp]
    lib.ggen_rmat.argtypes = [i32, i64, dbl, dbl, dbl, i32, i32, u64, u64, vp, vp, vp]
    lib.ggen_grid_edges.argtypes = [i32, i32, i64]
    lib.ggen_grid_edges.restype = i64
    lib.ggen_grid.argtypes = [i32, i32, i64, i32, i32, i32, u64, u64, vp, vp, vp]
    lib.ggen_csr_from_edges.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    lib.ggen_pick_sources.argtypes = [i32, vp, i32, u64, u64, vp]
    lib.ggen_fnv1a.argtypes = [vp, i64]
    lib.ggen_fnv1a.restype = u64
    for f in ("ggen_raw", "ggen_uniform", "ggen_rmat", "ggen_grid", "ggen_csr_from_edges",
              "ggen_pick_sources"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class HostGraph:
    """CSR graph on the host: rows sorted by source, int32 everywhere."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [m]
    w: np.ndarray | None  # int32 [m] or None when unweighted
    name: str = ""
    symmetric: bool = False  # every edge u->v has a matching v->u

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def edge_list(self):
        """(src, dst, w) in CSR order."""
        src = np.repeat(np.arange(self.n, dtype=np.int32), self.degrees())
        return src, self.col, self.w


def _alloc(n, m, weighted=True):
    return (np.zeros(n + 1, np.int32), np.zeros(max(m, 1), np.int32),
            np.zeros(max(m, 1), np.int32) if weighted else None)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


def raw(seed: int, stream: int, chunk: int, count: int) -> np.ndarray:
    out = np.zeros(max(count, 1), np.uint64)
    _check(_load().ggen_raw(seed, stream, chunk, count, _p(out)), "ggen_raw")
    return out[:count]


def _finish(n, row, col, w, m, name, symmetric=False):
    return HostGraph(n, row, col[:m], None if w is None else w[:m], name, symmetric)


def uniform(n: int, m: int, wlo=1, whi=100, seed=MASTER_SEED, stream=0, weighted=True,
            name="uniform") -> HostGraph:
    row, col, w = _alloc(n, m, weighted)
    _check(_load().ggen_uniform(n, m, wlo, whi, seed, stream, _p(row), _p(col), _p(w)),
           "ggen_uniform")
    return _finish(n, row, col, w, m, name)


def rmat(scale: int, m: int, a=0.57, b=0.19, c=0.19, wlo=1, whi=100, seed=MASTER_SEED, stream=0,
         weighted=True, name="rmat") -> HostGraph:
    n = 1 << scale
    row, col, w = _alloc(n, m, weighted)
    _check(_load().ggen_rmat(scale, m, a, b, c, wlo, whi, seed, stream, _p(row), _p(col), _p(w)),
           "ggen_rmat")
    return _finish(n, row, col, w, m, name)


def grid(width: int, height: int, n_shortcuts: int = 0, span: int = 8, wlo=1, whi=1000,
         seed=MASTER_SEED, stream=0, name="grid") -> HostGraph:
    lib = _load()
    m = int(lib.ggen_grid_edges(width, height, n_shortcuts))
    if m < 0:
        raise ValueError("bad grid size")
    n = width * height
    row, col, w = _alloc(n, m, True)
    _check(lib.ggen_grid(width, height, n_shortcuts, span, wlo, whi, seed, stream, _p(row),
                         _p(col), _p(w)), "ggen_grid")
    return _finish(n, row, col, w, m, name, symmetric=True)


def from_edges(n: int, src, dst, w=None, name="edges", symmetric=False) -> HostGraph:
    """Stable CSR from an explicit edge list (generation order kept in a row)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = len(src)
    if len(dst) != m or (w is not None and len(w) != m):
        raise ValueError("edge arrays differ in length")
    wt = None if w is None else np.ascontiguousarray(w, dtype=np.int32)
    row, col, wout = _alloc(n, m, w is not None)
    _check(_load().ggen_csr_from_edges(n, m, _p(src) if m else None, _p(dst) if m else None,
                                       _p(wt) if m else None, _p(row), _p(col),
                                       _p(wout) if m else None), "ggen_csr_from_edges")
    return _finish(n, row, col, wout, m, name, symmetric)


def pick_sources(g: HostGraph, count: int, seed=MASTER_SEED, stream=0) -> np.ndarray:
    out = np.zeros(max(count, 1), np.int32)
    rc = _load().ggen_pick_sources(g.n, _p(g.row_ptr), count, seed, stream, _p(out))
    _check(rc, "ggen_pick_sources")
    return out[:count]


def fnv1a(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a, dtype=np.int32)
    return int(_load().ggen_fnv1a(_p(a), len(a)))


# ---------------------------------------------------------------- workloads --
# Stream ids keep each workload's random numbers apart under one master seed.
STREAM = {"er16k": 1, "rmat22": 2, "grid4096": 3, "er23": 4, "batch": 5, "serve": 6,
          "sources": 100}

GRID_SIDE = 4096
GRID_SHORTCUTS = (2 * GRID_SIDE * (GRID_SIDE - 1)) // 100  # 1% of undirected grid edges


def workload(name: str, seed: int = MASTER_SEED) -> HostGraph:
    """The named synthetic workloads.

    er16k     directed uniform graph, 16,384 vertices, exactly 131,072 edges
              (self-loops redrawn), weights uniform in [1, 100]
    rmat22    R-MAT scale 22, edge factor 16 (67,108,864 edges), a,b,c,d =
              .57,.19,.19,.05, duplicates and self-loops kept, weights [1, 100]
    grid4096  4096 x 4096 4-neighbour grid, both directions, plus 1% of the
              undirected grid edges again as shortcuts of Chebyshev span <= 8
              (both directions), weights [1, 1000] shared by both directions
    er23      directed uniform graph, 2^23 vertices, 2^26 edges, weights [1, 100]
    Small variants for tests: rmat<s> (scale s, edge factor 16), grid<w>
    (w x w grid, 1% shortcuts), er<n>x<m>.
    """
    if name == "er16k":
        return uniform(16384, 131072, 1, 100, seed, STREAM["er16k"], name=name)
    if name == "rmat22":
        return rmat(22, 16 << 22, 0.57, 0.19, 0.19, 1, 100, seed, STREAM["rmat22"], name=name)
    if name == "grid4096":
        return grid(GRID_SIDE, GRID_SIDE, GRID_SHORTCUTS, 8, 1, 1000, seed, STREAM["grid4096"],
                    name=name)
    if name == "er23":
        return uniform(1 << 23, 1 << 26, 1, 100, seed, STREAM["er23"], name=name)
    if name.startswith("rmat"):
        s = int(name[4:])
        return rmat(s, 16 << s, 0.57, 0.19, 0.19, 1, 100, seed, STREAM["rmat22"] + 1000 * s,
                    name=name)
    if name.startswith("grid"):
        side = int(name[4:])
        return grid(side, side, (2 * side * (side - 1)) // 100, 8, 1, 1000, seed,
                    STREAM["grid4096"] + 1000 * side, name=name)
    if name.startswith("er"):
        nn, mm = name[2:].split("x")
        return uniform(int(nn), int(mm), 1, 100, seed, STREAM["er23"] + 7 * int(nn) + int(mm),
                       name=name)
    raise KeyError(name)


def batch_instances(count: int = 512, seed: int = MASTER_SEED):
    """The batched workload: `count` independent instances [(algo, graph,
    source)], each an R-MAT graph with scale uniform in 10..18 and edge
    factor uniform in 8..32 (weights [1, 100]), algorithm SSSP (0) or BFS (1)
    with probability 1/2, from a seeded source with out-degree > 0.  Each
    instance draws from its own stream of the master seed."""
    rng = np.random.default_rng(STREAM["batch"])
    out = []
    for i in range(count):
        scale = int(rng.integers(10, 19))
        ef = int(rng.integers(8, 33))
        hg = rmat(scale, ef << scale, seed=seed, stream=STREAM["batch"] * 100000 + i,
                  name=f"i{i}-rmat{scale}x{ef}")
        algo = int(rng.integers(0, 2))
        src = int(pick_sources(hg, 1, seed=seed, stream=STREAM["batch"] * 100000 + 50000 + i)[0])
        out.append((algo, hg, src))
    return out
