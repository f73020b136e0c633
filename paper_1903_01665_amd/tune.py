"""Autotuner: measured choice of mode x schedule x mapping per graph class.

The paper generates vertex- or edge-based, synchronous or asynchronous code
from one program and picks the variant per input by a compile-time switch
(Sec. 3, Sec. 4.3).  Here the choice is made by measurement: every variant
runs on a calibration set of synthetic graphs of each class (size, degree
skew, BFS depth: see gg_class_of in include/gg.h); for each (algorithm,
class) the variant with the lowest geometric mean of its time relative to
the best variant of each graph wins.  The table is written as JSON and the
binding installs it when the library loads.

    python -m paper_1903_01665_amd.tune --out paper_1903_01665_amd/tune_table.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import gen, gg

ALGOS = ("sssp", "bfs", "cc")
# (mode, schedule, mapping, near-far bucket width in mean weights)
VARIANTS = [(gg.VERTEX, gg.SYNC, gg.MAP_THREAD, 0), (gg.VERTEX, gg.SYNC, gg.MAP_WAVE, 0),
            (gg.VERTEX, gg.SYNC, gg.MAP_BALANCED, 0), (gg.VERTEX, gg.ASYNC, gg.MAP_THREAD, 0),
            (gg.VERTEX, gg.ASYNC, gg.MAP_WAVE, 0), (gg.VERTEX, gg.ASYNC, gg.MAP_BALANCED, 0),
            (gg.EDGE, gg.SYNC, gg.MAP_AUTO, 0), (gg.EDGE, gg.ASYNC, gg.MAP_AUTO, 0)]
NEARFAR = [(gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED, dm) for dm in (1, 2, 4, 8, 16, 64)]
DIROPT = [(gg.VERTEX, gg.DIROPT, gg.MAP_BALANCED, 0)]
CC_DIROPT = [(gg.EDGE, gg.DIROPT, gg.MAP_BALANCED, 0)]

# calibration graphs: the size classes of the workloads, from a seed stream of
# their own so that no benchmark graph is itself in the set
CALIB_STREAM = 0xCA11B
CALIBRATION = [("rmat", 12), ("rmat", 16), ("rmat", 20), ("rmat", 21), ("rmat", 22),
               ("er", 14), ("er", 18), ("er", 22), ("er", 23),
               ("grid", 128), ("grid", 512), ("grid", 2048), ("grid", 4100)]


def make(kind, p, seed):
    if kind == "rmat":
        return gen.rmat(p, 16 << p, stream=CALIB_STREAM + p, seed=seed, name=f"rmat{p}")
    if kind == "er":
        return gen.uniform(1 << p, 8 << p, 1, 100, stream=CALIB_STREAM + 100 + p, seed=seed,
                           name=f"er{p}")
    return gen.grid(p, p, (2 * p * (p - 1)) // 100, 8, 1, 1000, stream=CALIB_STREAM + 200 + p,
                    seed=seed, name=f"grid{p}")


def time_variant(g, algo, src, v, reps, out, avg_w):
    import torch
    mode, sched, mapping, dm = v
    o = gg.make_opts(mode, sched, mapping, time_limit_ms=4000,
                     delta=max(1, int(dm * avg_w)) if sched == gg.NEARFAR else 0)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        try:
            if algo == "cc":
                g.cc(opts=o, out=out)
            else:
                getattr(g, algo)(src, opts=o, out=out)
            torch.cuda.synchronize()
        except gg.GGError:
            return math.inf
        ts.append(time.perf_counter() - t)
    return sorted(ts)[len(ts) // 2]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=gg.TUNE_TABLE)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=gen.MASTER_SEED)
    args = ap.parse_args(argv)
    import torch
    gg.tune_set([])  # measure with the built-in rules in place
    results = []  # (algo, class, {variant: time})
    for kind, p in CALIBRATION:
        hg = make(kind, p, args.seed)
        g = gg.Graph.from_host(hg, symmetrize=True)
        cls = g.probe()
        src = int(gen.pick_sources(hg, 1, stream=CALIB_STREAM)[0])
        out = torch.empty(hg.n, dtype=torch.int32, device="cuda")
        avg_w = float(hg.w.mean()) if hg.w is not None and hg.m else 1.0
        for algo in ALGOS:
            times = {}
            extra = NEARFAR if algo == "sssp" else DIROPT if algo == "bfs" else CC_DIROPT
            for v in VARIANTS + extra:
                times[v] = time_variant(g, algo, src, v, args.reps, out, avg_w)
            best = min(times.values())
            print(f"[tune] {hg.name:8s} class={cls} {algo:4s} best "
                  f"{min(times, key=times.get)} {best * 1e3:.3f} ms", file=sys.stderr, flush=True)
            results.append((algo, cls, times))
        g.free()
        del out
    # per (algo, class): geometric mean of time / best-of-graph over the graphs
    groups = {}
    for algo, cls, times in results:
        best = min(times.values())
        for v, t in times.items():
            r = t / best if math.isfinite(t) else 1e6
            groups.setdefault((algo, cls), {}).setdefault(v, []).append(math.log(r))
    entries, detail = [], []
    for (algo, cls), per_v in sorted(groups.items()):
        score = {v: sum(x) / len(x) for v, x in per_v.items()}
        v = min(score, key=score.get)
        entries.append({"algo": ALGOS.index(algo), "size_class": cls[0], "skew_class": cls[1],
                        "depth_class": cls[2], "mode": v[0], "sched": v[1], "mapping": v[2],
                        "delta_mult": v[3]})
        detail.append({"algo": algo, "class": list(cls),
                       "relative_to_best": {f"{m}/{s}/{mp}/{dm}": round(math.exp(x), 3)
                                            for (m, s, mp, dm), x in score.items()}})
    raw = [{"algo": a, "class": list(c), "ms": {f"{m}/{s}/{mp}/{dm}": (round(t * 1e3, 4)
                                                                    if math.isfinite(t) else None)
                                                 for (m, s, mp, dm), t in ts.items()}}
           for a, c, ts in results]
    with open(args.out, "w") as f:
        json.dump({"entries": entries, "scores": detail, "measurements": raw,
                   "calibration": [f"{k}{p}" for k, p in CALIBRATION]}, f, indent=1)
    print(f"[tune] wrote {len(entries)} entries to {args.out}", file=sys.stderr)
    gg.tune_set(entries)


if __name__ == "__main__":
    main()
