"""Small seeded input builders and fixture readers shared by the tests.

Input synthesis only: no traversal arithmetic lives here.
"""
from __future__ import annotations

import os

import numpy as np

from paper_1903_01665_amd import gen

INF = 2**31 - 1
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def random_graph(rng: np.random.Generator, n: int, m: int, wlo=1, whi=9, self_loops=True,
                 name="rand"):
    src = rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32)
    if not self_loops and n > 1:
        bad = src == dst
        dst[bad] = (dst[bad] + 1) % n
    w = rng.integers(wlo, whi + 1, size=m, dtype=np.int64).astype(np.int32)
    return gen.from_edges(n, src, dst, w, name=name)


def path_graph(n, weights):
    src = np.arange(n - 1, dtype=np.int32)
    return gen.from_edges(n, src, src + 1, np.asarray(weights, np.int32), name="path")


def complete_digraph(n, w=1):
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != d
    s, d = s[keep].astype(np.int32), d[keep].astype(np.int32)
    return gen.from_edges(n, s, d, np.full(len(s), w, np.int32), name="complete")


def star(n_leaves, weights_per_leaf):
    """Hub 0 with parallel edges to each leaf: weights_per_leaf[i] lists them."""
    src, dst, w = [], [], []
    for leaf, ws in enumerate(weights_per_leaf, start=1):
        for x in ws:
            src.append(0)
            dst.append(leaf)
            w.append(x)
    return gen.from_edges(n_leaves + 1, src, dst, w, name="star")


def read_golden(fname):
    n = source = None
    src, dst, w, want = [], [], [], {}
    with open(os.path.join(GOLDEN, fname)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "source":
                source = int(tok[1])
            elif tok[0] == "edge":
                src.append(int(tok[1]))
                dst.append(int(tok[2]))
                w.append(int(tok[3]))
            else:
                want[tok[0]] = np.array([INF if t == "INF" else int(t) for t in tok[1:]],
                                        np.int32)
    g = gen.from_edges(n, src, dst, w, name=fname)
    return g, source, want


def golden_files():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))
