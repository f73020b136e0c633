"""Benchmark: GTEPS of SSSP + BFS + CC on one MI355X.

One step is one pass of the hot path over the resident graph: SSSP and BFS
from one source and CC over the whole graph, each in the variant the library
picks (AUTO).  The source rotates over 8 seeded sources with out-degree > 0.

value      traversed edges of all steps / wall time of the timed steps (GTEPS);
           traversed edges: out-edges of every reached vertex for SSSP/BFS,
           every edge of the both-directions graph for CC.
roofline   for the kernel with the most device time in a profiled repeat of
           the steps: algorithmic bytes (per-unit figures x the work counters
           of those launches) / summed launch time (HIP events on the stream
           the kernels run on), against 8 TB/s HBM.
cpu_baseline  the oracle (Dijkstra, FIFO BFS, union-find CC) on the same
           graph and first source, single-threaded, timed on this host.

Other configurations (``--config``):
batched    512 independent SSSP/BFS instances over R-MAT graphs (scale 10..18,
           edge factor 8..32, weights 1..100), run as one batch (grouped by
           class, tuned variant, HIP-graph replay) and as 512 plain calls;
           value = GTEPS of the batch.
serve      Poisson arrivals (2000 queries/s) of SSSP/BFS queries over 32
           resident R-MAT graphs (scale 12..22, edge factor 16), a new graph
           uploaded every 5 s; served (continuous batching) and plain (one
           query at a time) on the same trace; value = GTEPS served, with
           p50/p99 latency of both.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INF = 2**31 - 1
ALGOS = ("sssp", "bfs", "cc")
# (mode, schedule, mapping, passes of local expansion, near-far far_degree,
# near-far bucket width in eighths of the mean weight; 0 = the tuned width)
VARIANTS = {"vertex-sync": (0, 0, 3, 0, 0, 0), "vertex-async": (0, 1, 3, 0, 0, 0),
            "edge-sync": (1, 0, 0, 0, 0, 0), "edge-async": (1, 1, 0, 0, 0, 0),
            "nearfar": (0, 3, 3, 0, 0, 0), "diropt": (0, 4, 3, 0, 0, 0),
            "vertex-async-h8": (0, 1, 3, 8, 0, 0), "nearfar-h32": (0, 3, 3, 32, 0, 0),
            "nearfar-long64-h4": (0, 3, 3, 4, 64, 3), "unionfind": (0, 5, 3, 0, 0, 0)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------- algorithmic bytes --
# Bytes the method itself must move per unit of executed work (int32 = 4 B).
# round kernels:
#   vertex sync   8 B per vertex scanned (row offset + value; every vertex,
#                 every sweep); per edge 12 B SSSP (col, w, head value) or
#                 8 B BFS/CC (col, head value); 4 B per update
#   edge sync     per edge 20 B SSSP (src, col, w, two values), 16 B BFS/CC
#                 (src, col, two values); 4 B per update
#   vertex async  1 B per tile flag scanned; 16 B per frontier vertex (flag,
#                 row pair, value); per edge 12 B SSSP / 8 B BFS, CC;
#                 2 B per push (vertex and tile flag bytes)
#                 (local expansion: a vertex served again from the
#                 wavefront's own list reads only its row pair, 8 B; it is
#                 counted at 16 B here, an upper bound)
#   edge async    as vertex async, plus the 4 B edge-list source per edge
#   CC diropt     swept edges as edge sync (16 B), the other edges, vertices
#                 and tiles as vertex async; 4 B per update; per push 2 B of
#                 flags and 8 B for the pushed vertex's row length
#   CC union-find 8 B per vertex per phase (row offsets), 16 B per linked edge
#                 (column, two roots, the swap); the compressions as aux
# heavy kernels: per edge 12 / 8 B, per push 2 B (10 B under CC diropt)
# aux kernels:   init 4 B per vertex (+2 B of flags when async); CC shortcut
#                8 B per vertex per launch
def algorithmic_bytes(algo, mode, sched, kind, n, prof_kind, launches):
    E = prof_kind["edges_processed"]
    V = prof_kind["vertices_processed"]
    U = prof_kind["updates"]
    P = prof_kind["pushes"]
    if sched == 5 and kind == "round":
        # union-find: the row offsets of every vertex per linking phase, per
        # linked edge its column, the two roots found and the swap
        return 8 * n * launches + 16 * E
    per_edge = 12 if algo == "sssp" else 8
    if sched == 4 and (algo == "sssp" or (algo == "cc" and mode == 0)):
        # per-round push/pull (SSSP; CC in vertex mode): an edge is 12 B
        # (SSSP) or 8 B (CC) either way -- pushed: column, weight, head
        # value; pulled: column and tail flag, plus weight and tail value
        # for a frontier tail -- 16 B per vertex, 10 B per push (flags and
        # the pushed vertex's row length)
        if kind == "round":
            return per_edge * E + 16 * V + ((n + 63) // 64) * launches + 4 * U + 10 * P
        if kind == "heavy":
            return per_edge * E + 10 * P
    if algo == "cc" and sched == 4:
        D = prof_kind.get("swept_edges", 0)
        if kind == "round":
            return (16 * D + 8 * (E - D) + 16 * V + ((n + 63) // 64) * launches
                    + 4 * U + 10 * P)
        if kind == "heavy":
            return 8 * E + 10 * P
    if kind == "round":
        if sched == 0 and mode == 0:
            return 8 * n * launches + per_edge * E + 4 * U
        # asynchronous and near-far rounds (near-far: U counts deferred vertices,
        # each a flag read and a flag store)
        if sched == 0 and mode == 1:
            return (20 if algo == "sssp" else 16) * E + 4 * U
        ntiles = (n + 63) // 64
        extra = 4 * E if mode == 1 else 0
        return ntiles * launches + 16 * V + per_edge * E + extra + 2 * P
    if kind == "heavy":
        return per_edge * E + 2 * P
    return (4 + (2 if sched == 1 else 0)) * n + 8 * n * max(0, launches - 1)


def kernel_symbol(algo, kind, mode, sched, mapping, hops=0):
    """HIP symbol of the kernel that runs (algo, kind) in a variant (None when
    the variant launches no kernel of that kind)."""
    a = {"sssp": 0, "bfs": 1, "cc": 2}[algo]
    if sched == 5:  # union-find CC: linking rounds and compressions, no chunk kernel
        return {"round": "gg::k_uf(gg::Round)", "aux": "gg::k_uf_compress(gg::Round)"}.get(kind)
    if kind == "heavy":
        return f"void gg::k_heavy<{a}>(gg::Round)"
    if kind == "aux":
        return "gg::k_init(gg::Round, int, int)"
    if sched == 4:
        return f"gg::k_{algo}_diropt(gg::Round)"
    if mode == 1:
        return f"void gg::k_{'esync' if sched == 0 else 'easync'}<{a}>(gg::Round)"
    if sched == 0:
        return f"void gg::k_vsync<{a}, {mapping}>(gg::Round)"
    nf = "true" if sched == 3 else "false"  # the near-far schedule has its own instantiation
    if hops > 0 and mapping == 3:  # worklist rounds with local expansion
        return f"void gg::k_vlocal<{a}, {nf}>(gg::Round)"
    return f"void gg::k_vasync<{a}, {mapping}, {nf}>(gg::Round)"


def kernel_code_hash(src=None):
    """SHA-256 of the kernel source (default: gg_internal.h, which fixes the
    kernels' structures and constants, then gg_kernels.hip) with comments and
    blank lines removed: it changes when the code does, not when a comment
    does."""
    import hashlib
    import re
    if src is None:
        csrc = os.path.join(ROOT, "paper_1903_01665_amd", "csrc")
        src = "".join(open(os.path.join(csrc, f)).read() + "\n"
                      for f in ("gg_internal.h", "gg_kernels.hip"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*", "", ln).rstrip() for ln in src.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln.strip()).encode()).hexdigest()


def measured_traffic(symbol, workload):
    """HBM bytes per dispatch from the committed counter summary, or None when
    the summary is for another workload or the kernel code changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel_code_sha256") != kernel_code_hash():
        return None
    return t["bytes_per_dispatch"].get(symbol)


def traversed_edges(deg, dist):
    return int(deg[dist < INF].sum())


SCHED_NAMES = ["sync", "async", "auto", "nearfar", "diropt", "unionfind"]


def host_info():
    """Host facts recorded with every CPU baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"nproc": os.cpu_count(), "cpus_allowed": allowed, "cpu_model": model}


def copy_ceiling(torch, mib=1024, reps=20):
    """Achievable HBM bandwidth on this device: a plain device-to-device
    copy of 1 GiB (read + write), timed with HIP events on its stream."""
    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbps = 2 * n * 4 / (ms * 1e-3) / 1e9
    del a, b
    return {"GBps": round(gbps, 1), "frac_of_peak": round(gbps / HBM_PEAK_GBS, 4),
            "bytes_per_copy": 2 * n * 4,
            "kind": "device-to-device copy of 1 GiB (torch copy_, read + write), "
                    f"{reps} copies timed with HIP events"}


def variant_name(c):
    name = ["vertex", "edge"][c.mode] + "-" + SCHED_NAMES[c.sched]
    if c.hops:
        name += f"-h{c.hops}"
    if c.sched == 3 and c.far_degree:
        name += f"-long{c.far_degree}"
    return name


def run_workload(name, args, *, sources_kind="random8", variants=False, cpu=True, named=None):
    """One workload: upload, AUTO step timed (SSSP, BFS and CC in flight
    together from this host thread), roofline of the dominant kernel from a
    profiled repeat, optional per-variant table and named-variant latency,
    the oracle on the host and a bit-exact check.  Returns a dict."""
    import torch

    from paper_1903_01665_amd import gen, gg

    t = time.time()
    hg = gen.workload(name)
    deg = hg.degrees()
    log(f"[bench] {name}: n={hg.n} m={hg.m} generated in {time.time() - t:.1f}s")
    if sources_kind == "zero":
        sources = [0]
    elif sources_kind == "zero+4":
        sources = [0] + [int(x) for x in gen.pick_sources(hg, 4, stream=gen.STREAM["sources"])]
    else:
        sources = [int(x) for x in gen.pick_sources(hg, 8, stream=gen.STREAM["sources"])]
    t = time.time()
    g = gg.Graph.from_host(hg, symmetrize=True)
    torch.cuda.synchronize()
    upload_s = time.time() - t
    # depth class for the AUTO choice (one BFS, outside the timed region)
    gclass = g.probe()
    m_sym = hg.m if hg.symmetric else 2 * hg.m
    log(f"[bench] {name}: uploaded in {upload_s:.2f}s; class {gclass}; sources {sources}")

    outs = {a: torch.empty(hg.n, dtype=torch.int32, device="cuda") for a in ALGOS}
    auto = gg.make_opts()
    chosen = {a: g.resolve(i, auto) for i, a in enumerate(ALGOS)}
    wss = {a: gg.Workspace(g) for a in ALGOS}
    cur = torch.cuda.current_stream()

    def step_sequential(i, opts=None):
        s = sources[i % len(sources)]
        g.sssp(s, out=outs["sssp"], opts=opts)
        g.bfs(s, out=outs["bfs"], opts=opts)
        g.cc(out=outs["cc"], opts=opts)

    # the three traversals of a step are independent: they are issued from
    # this thread with the host-asynchronous calls, each on a workspace (and
    # so a stream) of its own, with no barrier between them (the paper's
    # barrier-free independent kernels, Sec. 3.2); the current stream then
    # waits for all three on the device
    def step_async(i, opts=None):
        s = sources[i % len(sources)]
        ts = [g.sssp_async(s, out=outs["sssp"], ws=wss["sssp"], opts=opts),
              g.bfs_async(s, out=outs["bfs"], ws=wss["bfs"], opts=opts),
              g.cc_async(out=outs["cc"], ws=wss["cc"], opts=opts)]
        for tk in ts:
            tk.stream_wait(cur)
            tk.free()

    step = step_sequential if args.sequential else step_async

    # traversed edges per source (from the GPU results of a first pass)
    m_trav, n_reach = {}, {}
    for i, s in enumerate(sources):
        step_sequential(i)
        torch.cuda.synchronize()
        d = outs["sssp"].cpu().numpy()
        m_trav[s] = (traversed_edges(deg, d), traversed_edges(deg, outs["bfs"].cpu().numpy()))
        n_reach[s] = int((d < INF).sum())
    steps = args.steps
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # ------------------------------------------------------------ timed --
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    srcs = [sources[i % len(sources)] for i in range(steps)]
    edges = sum(m_trav[s][0] + m_trav[s][1] + m_sym for s in srcs)
    gteps = edges / elapsed / 1e9
    log(f"[bench] {name}: {steps} steps in {elapsed * 1e3:.1f} ms -> {gteps:.2f} GTEPS")
    # work-efficient bytes: what one pass over the reached part needs --
    # SSSP 12 B per traversed edge + 8 B per reached vertex, BFS and CC 8 B
    # per edge + 8 B per vertex (n for CC) -- over the step time; redundant
    # relaxations and extra sweeps lower it
    we_bytes = sum(12 * m_trav[s][0] + 8 * n_reach[s] + 8 * m_trav[s][1] + 8 * n_reach[s]
                   + 8 * m_sym + 8 * hg.n for s in srcs)
    work_efficient = round(we_bytes / elapsed / 1e9 / HBM_PEAK_GBS, 4)

    # ----------------------------------------- profiled repeat: roofline --
    per_kernel = []
    for i in range(steps):
        s = sources[i % len(sources)]
        for a in ALGOS:
            o = gg.make_opts(flags=gg.OPT_PROFILE)
            if a == "cc":
                g.cc(out=outs[a], opts=o)
            else:
                getattr(g, a)(s, out=outs[a], opts=o)
            p = g.profile()
            c = chosen[a]
            for kind in gg.KINDS:
                pk = p[kind]
                if pk["launches"] == 0:
                    continue
                b = algorithmic_bytes(a, c.mode, c.sched, kind, hg.n, pk, pk["launches"])
                per_kernel.append((a, kind, pk["launches"], pk["total_ms"], b))
    agg = {}
    for a, kind, L, ms, b in per_kernel:
        x = agg.setdefault((a, kind), [0, 0.0, 0])
        x[0] += L
        x[1] += ms
        x[2] += b
    (da, dk), (dl, dms, db) = max(agg.items(), key=lambda kv: kv[1][1])
    c = chosen[da]
    mname = variant_name(c)
    achieved = db / (dms * 1e-3) / 1e9
    sym = kernel_symbol(da, dk, c.mode, c.sched, c.mapping, c.hops)
    traffic = measured_traffic(sym, name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "traffic_unit": "bytes/launch (L2-miss: FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                "kernel": f"{da} {mname} {dk} kernel", "symbol": sym, "launches": dl,
                "avg_launch_us": round(dms * 1e3 / dl, 2),
                "algorithmic_bytes_per_launch": int(db / dl),
                "algorithmic_bytes_total": int(db)}
    kernel_table = {f"{a}/{k}": {"launches": L, "ms": round(ms, 3),
                                 "GBps": round(b / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                                 "algorithmic_bytes": int(b)}
                    for (a, k), (L, ms, b) in agg.items()}
    log(f"[bench] {name}: dominant {roofline['kernel']} {achieved:.0f} GB/s over {dl} launches")

    # ------------------------------------------------ per-variant table --
    table = {}
    avg_w = float(hg.w.mean()) if hg.w is not None and hg.m else 1.0
    if variants:
        s = sources[0]
        for a in ALGOS:
            for vname, (mode, sched, mp, hops, far, de) in VARIANTS.items():
                if (sched == 3 and a != "sssp") or (sched == 4 and a == "sssp"):
                    continue  # near-far is an SSSP schedule, the per-round choice BFS/CC
                if sched == 5 and a != "cc":
                    continue  # union-find: CC only
                if hops and a == "cc":
                    continue  # label propagation gains nothing from local expansion
                if sched == 4 and a == "cc":
                    mode = 1  # CC's per-round choice starts from edge sweeps
                o = gg.make_opts(mode, sched, mp, hops=hops, far_degree=far,
                                 delta=max(1, int(de * avg_w / 8)) if de else 0)
                times = []
                for _ in range(max(args.reps, 5 if hg.m >= 1 << 20 else 100)):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    if a == "cc":
                        g.cc(out=outs[a], opts=o)
                    else:
                        getattr(g, a)(s, out=outs[a], opts=o)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t1)
                st = g.stats()
                tm = float(np.median(times))
                me = m_sym if a == "cc" else m_trav[s][0 if a == "sssp" else 1]
                table[f"{a}/{vname}"] = {"ms": round(tm * 1e3, 3),
                                         "p99_ms": round(float(np.percentile(times, 99)) * 1e3, 3),
                                         "reps": len(times),
                                         "GTEPS": round(me / tm / 1e9, 3),
                                         "iterations": st["iterations"],
                                         "edges_processed": st["edges_processed"]}
                log(f"[bench] {a:4s} {vname:13s} {tm * 1e3:9.3f} ms "
                    f"{me / tm / 1e9:7.2f} GTEPS it={st['iterations']}")

    # ------------------------------- named variant: per-query latency --
    named_res = None
    if named is not None:
        a, mode, sched, warm, reps = named
        o = gg.make_opts(mode, sched)
        s = sources[0]
        for _ in range(warm):
            getattr(g, a)(s, out=outs[a], opts=o)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t1 = time.perf_counter()
            getattr(g, a)(s, out=outs[a], opts=o)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        st = g.stats()
        me = m_trav[s][0 if a == "sssp" else 1]
        tm = float(np.median(times))
        named_res = {"algo": a, "variant": variant_name(g.resolve(ALGOS.index(a), o)),
                     "warmup": warm, "reps": reps, "median_ms": round(tm * 1e3, 4),
                     "p99_ms": round(float(np.percentile(times, 99)) * 1e3, 4),
                     "GTEPS": round(me / tm / 1e9, 4), "iterations": st["iterations"],
                     "timing": "host clock around the call and a device synchronize"}
        log(f"[bench] {name}: {a} {named_res['variant']} median {tm * 1e3:.4f} ms, "
            f"p99 {named_res['p99_ms']} ms over {reps} reps")

    # ------------------------------------------------- CPU oracle leg --
    cpu_res = None
    verified = None
    if cpu:
        import oracle

        s = sources[0]
        t1 = time.perf_counter()
        d = oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
        t2 = time.perf_counter()
        b = oracle.bfs(hg.n, hg.row_ptr, hg.col, s)
        t3 = time.perf_counter()
        lab = oracle.cc(hg.n, hg.row_ptr, hg.col)
        t4 = time.perf_counter()
        ce = m_trav[s][0] + m_trav[s][1] + m_sym
        cpu_res = {"value": round(ce / (t4 - t1) / 1e9, 4), "unit": "GTEPS", "cores": 1,
                   "threads": 1, "kind": "oracle",
                   "sample": f"full {name} graph, source {s}: Dijkstra + FIFO BFS + "
                             f"union-find CC, one thread",
                   "seconds": {"sssp": round(t2 - t1, 3), "bfs": round(t3 - t2, 3),
                               "cc": round(t4 - t3, 3)},
                   "host": host_info()}
        step(0)
        torch.cuda.synchronize()
        verified = bool(np.array_equal(outs["sssp"].cpu().numpy(), d) and
                        np.array_equal(outs["bfs"].cpu().numpy(), b) and
                        np.array_equal(outs["cc"].cpu().numpy(), lab))
        log(f"[bench] {name}: oracle {t4 - t1:.2f}s ({cpu_res['value']} GTEPS); "
            f"GPU results match: {verified}")

    for w in wss.values():
        w.free()
    g.free()
    res = {"workload": name, "n": hg.n, "m": hg.m, "m_sym": m_sym,
           "GTEPS": round(gteps, 3), "steps": steps, "ms_per_step": round(elapsed * 1e3 / steps, 3),
           "step": "sssp+bfs+cc, AUTO variants, " + (
               "one after the other on one stream" if args.sequential
               else "in flight together (host-asynchronous calls from one thread)"),
           "variant": {a: {"mode": ["vertex", "edge"][chosen[a].mode],
                           "sched": SCHED_NAMES[chosen[a].sched],
                           "mapping": chosen[a].mapping, "hops": chosen[a].hops,
                           "delta": chosen[a].delta if chosen[a].sched == 3 else 0,
                           "far_degree": chosen[a].far_degree} for a in ALGOS},
           "sources": sources, "upload_s": round(upload_s, 2), "graph_class": list(gclass),
           "verified_vs_oracle": verified, "roofline": roofline,
           "work_efficient_frac": work_efficient, "cpu_baseline": cpu_res,
           "kernels": kernel_table}
    if table:
        res["variants"] = table
    if named_res:
        res["named_variant"] = named_res
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--no-variants", action="store_true", help="skip the per-variant table")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the other configurations (er16k, grid4096, er23, batched) "
                         "and the copy ceiling")
    ap.add_argument("--reps", type=int, default=3, help="repeats per variant in the table")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--config", default="single",
                    choices=["single", "batched", "serve", "concurrent", "msf"])
    ap.add_argument("--workloads", default="er16k,rmat16,rmat22",
                    help="concurrent: workloads to run")
    ap.add_argument("--instances", type=int, default=512, help="batched: instance count")
    ap.add_argument("--no-batched", action="store_true",
                    help="single: leave the batched configuration out of the default run")
    ap.add_argument("--duration", type=float, default=12.0, help="serve: trace seconds")
    ap.add_argument("--serve-warmup", type=float, default=0.0,
                    help="serve: seconds of trace before the measured part")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: queries per second")
    ap.add_argument("--slots", type=int, default=8, help="serve: queries in flight at most")
    ap.add_argument("--no-plain", action="store_true", help="serve: skip the plain run")
    ap.add_argument("--sequential", action="store_true",
                    help="single: run a step's SSSP, BFS and CC one after the other on one "
                         "stream (default: in flight together)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.config == "batched":
        return bench_batched(args)
    if args.config == "serve":
        return bench_serve(args)
    if args.config == "concurrent":
        return bench_concurrent(args)
    if args.config == "msf":
        return bench_msf(args)

    import torch

    from paper_1903_01665_amd import gg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    gg.lib()

    if args.calib_copy_mib:
        # a plain copy of known size: reading its FETCH_SIZE / WRITE_SIZE
        # counters scales the counters of the traversal kernels
        nbytes = args.calib_copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB done (3 dispatches)")
        del a, b

    ceiling = None if args.headline_only else copy_ceiling(torch)
    if ceiling:
        log(f"[bench] device copy ceiling {ceiling['GBps']} GB/s")
    head = run_workload(args.workload, args, variants=not args.no_variants,
                        cpu=not args.no_cpu,
                        sources_kind={"er16k": "zero", "grid4096": "zero+4",
                                      "er23": "zero+4"}.get(args.workload, "random8"),
                        named=("sssp", 0, 0, 5, 100) if args.workload == "er16k" else None)
    others = {}
    if not args.headline_only:
        # the other configurations: C1 (its named variant, vertex-synchronous
        # SSSP from vertex 0, 5 warm-up + 100 timed calls, beside the AUTO
        # step), the road-like grid and the large uniform graph (source 0 and
        # four random sources)
        plan = [("er16k", "zero", ("sssp", 0, 0, 5, 100)), ("grid4096", "zero+4", None),
                ("er23", "zero+4", None)]
        for w, sk, named in plan:
            if w == args.workload:
                continue
            others[w] = run_workload(w, args, sources_kind=sk, variants=False,
                                     cpu=not args.no_cpu, named=named)
            torch.cuda.empty_cache()
        # C4: the batched launch of 512 small instances
        if not args.no_batched:
            others["batched"] = bench_batched(args, emit=False)
            torch.cuda.empty_cache()

    line = {
        "metric": "GTEPS (SSSP+BFS+CC)", "value": head["GTEPS"], "unit": "GTEPS",
        "n_gpus": 1, "steps": head["steps"], "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {k: head[k] for k in ("workload", "n", "m", "m_sym", "step", "variant",
                                        "sources", "upload_s", "graph_class",
                                        "verified_vs_oracle")},
        "roofline": head["roofline"],
        "work_efficient_frac": head["work_efficient_frac"],
        "cpu_baseline": head["cpu_baseline"],
        "copy_ceiling": ceiling,
        "kernels": head["kernels"],
    }
    if "variants" in head:
        line["variants"] = head["variants"]
    if "named_variant" in head:
        line["named_variant"] = head["named_variant"]
    if others:
        line["configs"] = others
    print(json.dumps(line), flush=True)


def make_line(args, metric, value, unit, ms_per_step, config, **extra):
    line = {"metric": metric, "value": round(value, 4), "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic", "config": config}
    line.update(extra)
    return line


def common_line(args, metric, value, unit, ms_per_step, config, **extra):
    print(json.dumps(make_line(args, metric, value, unit, ms_per_step, config, **extra)),
          flush=True)


def bench_batched(args, emit=True):
    """512 instances: one batch (tuned groups, HIP-graph replay) vs plain calls.
    emit=False returns the line instead of printing it."""
    import torch

    from paper_1903_01665_amd import gen, gg

    t = time.time()
    inst = gen.batch_instances(args.instances)
    total_m = sum(hg.m for _, hg, _ in inst)
    log(f"[bench] {len(inst)} instances, {total_m} edges, generated in {time.time() - t:.1f}s")

    t = time.time()
    b = gg.Batch(inst)
    info = b.info()
    out = torch.empty(info["total_n"], dtype=torch.int32, device="cuda")
    b.run(out)  # eager run + capture of every group
    torch.cuda.synchronize()
    log(f"[bench] batch built and captured in {time.time() - t:.1f}s: {info}")
    res = out.cpu().numpy()
    off = b.offsets()
    m_trav = v_reach = min_bytes = 0
    for i, (algo, hg, s) in enumerate(inst):
        reached = res[off[i]: off[i] + hg.n] != INF
        e = int(hg.degrees()[reached].sum())
        v = int(reached.sum())
        m_trav += e
        v_reach += v
        # work-efficient minimum: every reached vertex's row offsets and value
        # (read and written) once, every edge of it once (column, weight for
        # SSSP, head value)
        min_bytes += (12 if algo == 0 else 8) * e + 16 * v
    for _ in range(args.warmup):
        b.run(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run(out)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    groups = [b.group(i) for i in range(info["groups"])]
    log(f"[bench] batched: {tb * 1e3:.2f} ms per run -> {m_trav / tb / 1e9:.2f} GTEPS")

    # plain: one graph per instance, one blocking call per instance, AUTO variant
    graphs = [gg.Graph.from_host(hg) for _, hg, _ in inst]
    outs = [torch.empty(hg.n, dtype=torch.int32, device="cuda") for _, hg, _ in inst]
    torch.cuda.synchronize()

    def plain():
        for (algo, hg, s), g, o in zip(inst, graphs, outs):
            (g.sssp if algo == 0 else g.bfs)(s, out=o)
        torch.cuda.synchronize()

    plain()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        plain()
    tp = (time.perf_counter() - t0) / max(1, args.steps // 2)
    same = all(np.array_equal(outs[i].cpu().numpy(), res[off[i]: off[i] + hg.n])
               for i, (_, hg, _) in enumerate(inst))
    log(f"[bench] plain: {tp * 1e3:.2f} ms per pass -> {m_trav / tp / 1e9:.2f} GTEPS; "
        f"batched == plain: {same}")
    for g in graphs:
        g.free()
    b.free()

    # the whole run is the unit here: the groups' kernels run inside HIP-graph
    # replays on streams of their own, overlapped, so no single kernel's
    # launch time stands for the run
    roof = {"bound": "hbm", "achieved": round(min_bytes / tb / 1e9, 1), "peak": 8000.0,
            "unit": "GB/s", "frac": round(min_bytes / tb / 1e9 / 8000.0, 4), "traffic": None,
            "kernel": "whole batched run (every group's round kernels, HIP-graph replays)",
            "launches": len(groups), "avg_launch_us": round(tb * 1e6, 2),
            "algorithmic_bytes_per_launch": int(min_bytes / max(1, len(groups))),
            "algorithmic_bytes_total": int(min_bytes),
            "algorithmic_bytes_rule": "12 B (SSSP) / 8 B (BFS) per traversed edge + 16 B per "
                                      "reached vertex, once each"}

    cpu = verified = None
    if not args.no_cpu:
        import concurrent.futures

        import oracle
        threads = min(16, host_info()["cpus_allowed"] or os.cpu_count() or 1)

        def one(i):
            algo, hg, s = inst[i]
            if algo == 0:
                return oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s)
            return oracle.bfs(hg.n, hg.row_ptr, hg.col, s)

        # ctypes releases the GIL inside the C oracle: the instances run in
        # parallel, one per thread at a time
        t0 = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(threads) as ex:
            want = list(ex.map(one, range(len(inst))))
        tc = time.perf_counter() - t0
        verified = all(np.array_equal(want[i], res[off[i]: off[i] + hg.n])
                       for i, (_, hg, _) in enumerate(inst))
        cpu = {"value": round(m_trav / tc / 1e9, 4), "unit": "GTEPS", "cores": threads,
               "threads": threads, "kind": "oracle", "seconds": round(tc, 3),
               "sample": f"all {len(inst)} instances: Dijkstra / FIFO BFS per instance, "
                         f"instances spread over {threads} threads",
               "host": host_info()}
        log(f"[bench] oracle on {threads} threads: {tc:.2f}s ({cpu['value']} GTEPS); "
            f"GPU results match: {verified}")
    out = (common_line if emit else make_line)(
                args, "GTEPS batched (512 SSSP/BFS instances)", m_trav / tb / 1e9, "GTEPS",
                tb * 1e3,
                {"workload": "batched-rmat-10..18", "instances": len(inst), "edges": total_m,
                 "traversed_edges": m_trav, "reached_vertices": v_reach, "groups": groups,
                 "verified_vs_oracle": verified},
                roofline=roof, cpu_baseline=cpu,
                plain={"GTEPS": round(m_trav / tp / 1e9, 4), "ms_per_pass": round(tp * 1e3, 3)},
                speedup_vs_plain=round(tp / tb, 3), results_identical_to_plain=same)
    return out


def bench_msf(args):
    """Minimum spanning forest of one workload graph (every stored edge taken
    as undirected): device Boruvka rounds vs the oracle's Kruskal."""
    import torch

    from paper_1903_01665_amd import gen, gg

    hg = gen.workload(args.workload)
    g = gg.Graph.from_host(hg)
    out = torch.empty(max(hg.m, 1), dtype=torch.uint8, device="cuda")
    for _ in range(max(1, args.warmup)):
        g.msf(out=out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        sel, tw, ne = g.msf(out=out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    st = g.stats()
    tm = float(np.median(ts))
    log(f"[bench] msf {args.workload}: {tm * 1e3:.3f} ms, {st['iterations']} rounds, "
        f"{ne} edges, weight {tw}")
    cpu = verified = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        want, total = oracle.msf(hg.n, hg.row_ptr, hg.col, hg.w)
        tc = time.perf_counter() - t0
        verified = bool(np.array_equal(sel.cpu().numpy(), want) and total == tw)
        cpu = {"value": round(hg.m / tc / 1e9, 4), "unit": "G edges/s", "cores": 1,
               "kind": "oracle", "seconds": round(tc, 3),
               "sample": f"full {args.workload} graph: Kruskal (sort by key, union-find), "
                         f"one thread"}
        log(f"[bench] oracle {tc:.2f}s; GPU forest matches: {verified}")
    g.free()
    common_line(args, "G edges/s (minimum spanning forest)", hg.m / tm / 1e9, "G edges/s",
                tm * 1e3, {"workload": args.workload, "n": hg.n, "m": hg.m,
                           "rounds": st["iterations"], "forest_edges": ne,
                           "forest_weight": tw, "verified_vs_oracle": verified},
                cpu_baseline=cpu)


def bench_concurrent(args):
    """SSSP and BFS from the same source on one resident graph: one after the
    other on one stream, or at the same time on two streams with a workspace
    each and no barrier between them (the paper's barrier-free independent
    kernels, Sec. 3.2)."""
    import threading

    import torch

    from paper_1903_01665_amd import gen, gg

    per = {}
    tot_e = tot_t = 0.0
    for w in args.workloads.split(","):
        hg = gen.workload(w)
        g = gg.Graph.from_host(hg, symmetrize=True)
        s = int(gen.pick_sources(hg, 1, stream=gen.STREAM["sources"])[0])
        deg = hg.degrees()
        ws = [gg.Workspace(g), gg.Workspace(g)]
        st = [torch.cuda.Stream(), torch.cuda.Stream()]
        outs = [torch.empty(hg.n, dtype=torch.int32, device="cuda") for _ in range(4)]
        calls = [lambda: g.sssp(s, out=outs[0], ws=ws[0], stream=st[0]),
                 lambda: g.bfs(s, out=outs[1], ws=ws[1], stream=st[1])]

        def seq():
            g.sssp(s, out=outs[2], ws=ws[0], stream=st[0])
            g.bfs(s, out=outs[3], ws=ws[0], stream=st[0])
            torch.cuda.synchronize()

        def both():
            th = threading.Thread(target=calls[1])
            th.start()
            calls[0]()
            th.join()
            torch.cuda.synchronize()

        reps = max(args.steps, 200 if hg.m < 1 << 20 else 10)
        res = {}
        for name, fn in (("sequential", seq), ("concurrent", both)):
            for _ in range(max(1, args.warmup)):
                fn()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t0)
            res[name] = float(np.median(ts))
        same = bool(torch.equal(outs[0], outs[2]) and torch.equal(outs[1], outs[3]))
        d = outs[0].cpu().numpy()
        edges = 2 * traversed_edges(deg, d)  # SSSP and BFS reach the same vertices
        per[w] = {"sequential_ms": round(res["sequential"] * 1e3, 4),
                  "concurrent_ms": round(res["concurrent"] * 1e3, 4),
                  "speedup": round(res["sequential"] / res["concurrent"], 3),
                  "GTEPS_concurrent": round(edges / res["concurrent"] / 1e9, 3),
                  "results_identical": same, "reps": reps}
        log(f"[bench] concurrent {w}: seq {res['sequential'] * 1e3:.3f} ms, "
            f"two streams {res['concurrent'] * 1e3:.3f} ms, same={same}")
        tot_e += edges
        tot_t += res["concurrent"]
        for x in ws:
            x.free()
        g.free()
    common_line(args, "GTEPS SSSP+BFS on two streams", tot_e / tot_t / 1e9, "GTEPS",
                tot_t * 1e3, {"workload": "concurrent-" + args.workloads.replace(",", "+")},
                per_workload=per)


def bench_serve(args):
    """Poisson trace served with continuous batching vs one query at a time."""
    import torch

    from paper_1903_01665_amd import gen, gg, serve

    n_pool, upload_every = 32, 5.0
    n_up = int((args.serve_warmup + args.duration) // upload_every)
    scales = serve.pool_scales(n_pool + n_up, 12, 22, gen.STREAM["serve"])
    t = time.time()
    hosts = [serve.make_graph(i, sc) for i, sc in enumerate(scales)]
    log(f"[bench] serve: {len(hosts)} graphs ({sum(h.m for h in hosts)} edges) in "
        f"{time.time() - t:.1f}s")
    sources = {i: gen.pick_sources(h, 16, stream=gen.STREAM["serve"] * 1000 + i)
               for i, h in enumerate(hosts)}

    def graphs_at(ti):
        k = int(ti // upload_every)  # uploads done by time ti
        return list(range(min(k, n_up), n_pool + min(k, n_up)))

    # the trace covers the warm-up and the measured part; latencies count
    # the queries that arrive after the warm-up
    total_s = args.serve_warmup + args.duration
    trace = serve.make_trace(args.rate, total_s, graphs_at, sources, gen.STREAM["serve"])
    measured = trace.t >= args.serve_warmup
    # traversed edges per (graph, source)
    trav = {}
    for i, h in enumerate(hosts):
        g = gg.Graph.from_host(h, symmetrize=True)
        trav[i] = serve.traversed_edges(g, h, sources[i])
        g.free()
    edges = sum(trav[int(gi)][int(s)] for gi, s in zip(trace.graph, trace.source))
    log(f"[bench] trace: {len(trace.t)} queries over {total_s}s ({int(measured.sum())} after "
        f"the {args.serve_warmup}s warm-up), {edges} traversed edges")
    svc_s = np.full(len(trace.t), np.nan)
    lat_s, st, wall_s = serve.run_served(hosts, trace, slots=args.slots,
                                         upload_every=upload_every, n_pool=n_pool, service=svc_s,
                                         log=log)
    ok = int((st == 0).sum())
    log(f"[bench] served: wall {wall_s:.2f}s p50 {serve.percentile(lat_s[measured], 50) * 1e3:.2f} ms "
        f"p99 {serve.percentile(lat_s[measured], 99) * 1e3:.2f} ms ({ok}/{len(st)} ok), "
        f"service mean {np.nanmean(svc_s) * 1e3:.3f} ms")
    svc_p = np.full(len(trace.t), np.nan)
    if args.no_plain:
        lat_p, wall_p = np.array([np.nan]), float("nan")
    else:
        lat_p, wall_p = serve.run_plain(hosts, trace, n_pool=n_pool, upload_every=upload_every,
                                        service=svc_p, log=log)
        log(f"[bench] plain: wall {wall_p:.2f}s p50 {serve.percentile(lat_p[measured], 50) * 1e3:.2f} ms "
            f"p99 {serve.percentile(lat_p[measured], 99) * 1e3:.2f} ms, "
            f"service mean {np.nanmean(svc_p) * 1e3:.3f} ms")
    q = lambda x, p: round(serve.percentile(x[measured] if len(x) == len(measured) else x, p)
                           * 1e3, 3)
    sv = lambda x: {"mean": round(float(np.nanmean(x)) * 1e3, 4),
                    "p50": round(float(np.nanpercentile(x, 50)) * 1e3, 4)} \
        if np.isfinite(x).any() else None
    common_line(args, "GTEPS served (Poisson SSSP/BFS queries)", edges / wall_s / 1e9, "GTEPS",
                wall_s * 1e3 / max(1, len(trace.t)),
                {"workload": "serve-rmat-12..22", "graphs": n_pool, "uploads": n_up,
                 "rate_qps": args.rate, "duration_s": args.duration,
                 "warmup_s": args.serve_warmup, "queries": len(trace.t),
                 "measured_queries": int(measured.sum()),
                 "traversed_edges": edges, "slots": args.slots},
                latency_ms={"served": {"p50": q(lat_s, 50), "p99": q(lat_s, 99)},
                            "plain": {"p50": q(lat_p, 50), "p99": q(lat_p, 99)}},
                plain={"GTEPS": round(edges / wall_p / 1e9, 4), "wall_s": round(wall_p, 3)},
                service_ms={"served": sv(svc_s), "plain": sv(svc_p)},
                served_ok=ok, served_wall_s=round(wall_s, 3))


if __name__ == "__main__":
    main()
