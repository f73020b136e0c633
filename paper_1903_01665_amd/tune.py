"""Autotuner: measured choice of mode x schedule x mapping per graph class.

The paper generates vertex- or edge-based, synchronous or asynchronous code
from one program and picks the variant per input by a compile-time switch
(Sec. 3, Sec. 4.3).  Here the choice is made by measurement: every variant
runs on a calibration set of synthetic graphs of each class (size, degree
skew, BFS depth: see gg_class_of in include/gg.h); for each (algorithm,
class) the variant with the lowest geometric mean of its time relative to
the best variant of each graph wins.  A graph's time for a variant is the sum
over a few sources of the median of repeated runs (traversal times vary with
the source).  Variants include the near-far bucket width and the passes of
local expansion.  The table is written as JSON and the binding installs it
when the library loads.

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
# (mode, schedule, mapping, near-far bucket width in eighths of the mean
# weight, passes of local expansion, near-far far_degree)
V, NF, BAL = gg.VERTEX, gg.NEARFAR, gg.MAP_BALANCED
VARIANTS = [(V, gg.SYNC, gg.MAP_THREAD, 0, 0, 0), (V, gg.SYNC, gg.MAP_WAVE, 0, 0, 0),
            (V, gg.SYNC, BAL, 0, 0, 0), (V, gg.ASYNC, gg.MAP_THREAD, 0, 0, 0),
            (V, gg.ASYNC, gg.MAP_WAVE, 0, 0, 0), (V, gg.ASYNC, BAL, 0, 0, 0),
            (gg.EDGE, gg.SYNC, gg.MAP_AUTO, 0, 0, 0), (gg.EDGE, gg.ASYNC, gg.MAP_AUTO, 0, 0, 0)]
LOCAL = [(V, gg.ASYNC, BAL, 0, h, 0) for h in (2, 8)]
NEARFAR = ([(V, NF, BAL, de, 0, 0) for de in (8, 16, 32, 64, 128, 512)] +
           [(V, NF, BAL, de, h, 0) for de in (8, 16, 32, 64, 128) for h in (2, 8, 32)] +
           # long chains of passes (deep graphs) and finer widths around them
           [(V, NF, BAL, de, 64, 0) for de in (24, 32, 48)] +
           [(V, NF, BAL, de, 32, 0) for de in (24, 48)] +
           # narrow buckets that hold back only long rows (skewed graphs)
           [(V, NF, BAL, de, 4, far) for de in (2, 3, 4, 6) for far in (32, 96)])
DIROPT = [(V, gg.DIROPT, BAL, 0, 0, 0)]
# CC's per-round schedule with edge sweeps or vertex pulls as dense rounds
CC_DIROPT = [(gg.EDGE, gg.DIROPT, BAL, 0, 0, 0), (V, gg.DIROPT, BAL, 0, 0, 0),
             # the union-find Set (sampled links, then the rest off the giant)
             (V, gg.UNIONFIND, BAL, 0, 0, 0)]
# SSSP's per-round schedule (pull rounds over the weighted in-edge CSR)
SSSP_DIROPT = [(V, gg.DIROPT, BAL, 0, 0, 0)]

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


def time_variant(g, algo, srcs, v, reps, out, avg_w):
    """Sum over the sources of the median time of `reps` runs (CC: one
    source-free run set)."""
    import torch
    mode, sched, mapping, de, hops, far = v
    o = gg.make_opts(mode, sched, mapping, time_limit_ms=4000,
                     delta=max(1, int(de * avg_w / 8)) if sched == gg.NEARFAR else 0, hops=hops,
                     far_degree=far)
    total = 0.0
    for src in srcs[:1] if algo == "cc" else srcs:
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
        total += sorted(ts)[len(ts) // 2]
    return total


# Two variants whose scores differ by less than this factor are a tie
# (repeated calibration runs differ by a few per cent); a tie goes to the
# variant with fewer schedule knobs.
TIE = 1.03


def knobs(v):
    """Schedule knobs a variant sets: near-far buckets, local expansion,
    deferral of long rows only."""
    return int(v[1] == gg.NEARFAR) + int(v[4] > 0) + int(v[5] > 0)


def variant_key(k):
    """Variant tuple from a measurement key "mode/sched/mapping/delta_eighths/
    hops/far_degree"."""
    return tuple(int(x) for x in k.split("/"))


def choose(results):
    """Table entries from (algo, class, {variant: seconds}) measurements: per
    (algo, class) the lowest geometric mean of time / best-of-graph over the
    graphs of the class; ties (within TIE) go to fewer knobs."""
    groups = {}
    for algo, cls, times in results:
        best = min(times.values())
        for v, t in times.items():
            r = t / best if math.isfinite(t) else 1e6
            groups.setdefault((algo, tuple(cls)), {}).setdefault(v, []).append(math.log(r))
    entries, detail = [], []
    for (algo, cls), per_v in sorted(groups.items()):
        score = {v: sum(x) / len(x) for v, x in per_v.items()}
        top = min(score.values())
        near = [v for v in score if score[v] <= top + math.log(TIE)]
        v = min(near, key=lambda u: (knobs(u), score[u]))
        entries.append({"algo": ALGOS.index(algo), "size_class": cls[0], "skew_class": cls[1],
                        "depth_class": cls[2], "mode": v[0], "sched": v[1], "mapping": v[2],
                        "delta_eighths": v[3], "hops": v[4], "far_degree": v[5]})
        detail.append({"algo": algo, "class": list(cls),
                       "relative_to_best": {"/".join(map(str, k)): round(math.exp(x), 3)
                                            for k, x in score.items()}})
    return entries, detail


def measure(args, known=None):
    """Time every variant on every calibration graph; with `known` (the
    measurements of an earlier table, in calibration order: (algo, class,
    {variant: seconds})) only the variants missing there are timed and the
    rest are taken over."""
    import torch
    gg.tune_set([])  # measure with the built-in rules in place
    results = []  # (algo, class, {variant: time})
    redo = set(getattr(args, "remeasure", "").split(",")) - {""}
    for kind, p in CALIBRATION:
        hg = make(kind, p, args.seed)
        g = gg.Graph.from_host(hg, symmetrize=True, transpose=True)
        cls = g.probe()
        # traversal times vary with the source: every variant runs from the
        # same few
        srcs = [int(x) for x in gen.pick_sources(hg, args.sources, stream=CALIB_STREAM)]
        out = torch.empty(hg.n, dtype=torch.int32, device="cuda")
        avg_w = float(hg.w.mean()) if hg.w is not None and hg.m else 1.0
        for algo in ALGOS:
            times = {}
            if known:
                ka, kc, kt = known[len(results)]
                if (ka, tuple(kc)) != (algo, tuple(cls)):
                    raise RuntimeError(f"measurements do not match: {ka} {kc} vs {algo} {cls}")
                algos = set(getattr(args, "remeasure_algos", "").split(",")) - {""}
                if hg.name not in redo or (algos and algo not in algos):
                    times = dict(kt)
                elif args.remeasure_local:
                    # only the variants with local expansion are timed again
                    times = {v: t for v, t in kt.items() if v[4] == 0}
            extra = (NEARFAR + SSSP_DIROPT if algo == "sssp" else DIROPT if algo == "bfs"
                     else CC_DIROPT)
            for v in VARIANTS + LOCAL + extra:
                if v not in times:
                    times[v] = time_variant(g, algo, srcs, v, args.reps, out, avg_w)
            best = min(times.values())
            print(f"[tune] {hg.name:8s} class={cls} {algo:4s} best "
                  f"{min(times, key=times.get)} {best * 1e3:.3f} ms", file=sys.stderr, flush=True)
            results.append((algo, cls, times))
        g.free()
        del out
    return results


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=gg.TUNE_TABLE)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sources", type=int, default=3)
    ap.add_argument("--seed", type=int, default=gen.MASTER_SEED)
    ap.add_argument("--from-measurements", metavar="TABLE_JSON",
                    help="re-derive the entries from the measurements of an earlier table "
                         "(no GPU needed)")
    ap.add_argument("--extend", metavar="TABLE_JSON",
                    help="time only the variants that the measurements of this table lack "
                         "and keep the others")
    ap.add_argument("--remeasure", default="", metavar="NAMES",
                    help="with --extend: time every variant again on these calibration "
                         "graphs (comma-separated, e.g. rmat20,rmat22)")
    ap.add_argument("--remeasure-local", action="store_true",
                    help="with --remeasure: only the variants with local expansion")
    ap.add_argument("--remeasure-algos", default="", metavar="ALGOS",
                    help="with --remeasure: only these algorithms (comma-separated, e.g. cc)")
    args = ap.parse_args(argv)

    def load(path):
        with open(path) as f:
            raw = json.load(f)["measurements"]
        return [(r["algo"], tuple(r["class"]),
                 {variant_key(k): (t * 1e-3 if t is not None else math.inf)
                  for k, t in r["ms"].items()}) for r in raw]

    if args.from_measurements:
        results = load(args.from_measurements)
    elif args.extend:
        results = measure(args, load(args.extend))
    else:
        results = measure(args)
    entries, detail = choose(results)
    raw = [{"algo": a, "class": list(c),
            "ms": {"/".join(map(str, k)): (round(t * 1e3, 4) if math.isfinite(t) else None)
                   for k, t in ts.items()}}
           for a, c, ts in results]
    with open(args.out, "w") as f:
        json.dump({"entries": entries, "scores": detail, "measurements": raw,
                   "calibration": [f"{k}{p}" for k, p in CALIBRATION]}, f, indent=1)
    print(f"[tune] wrote {len(entries)} entries to {args.out}", file=sys.stderr)
    gg.tune_set(entries)


if __name__ == "__main__":
    main()
