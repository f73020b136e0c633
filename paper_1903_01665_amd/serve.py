"""Serving driver: Poisson arrivals of SSSP/BFS queries over resident graphs.

Two ways to serve the same arrival trace:

served  the continuous-batching server of libgg (gg_server_*): queries are
        submitted at their arrival time; the server's native driver thread
        admits them while a slot and the memory budget allow and advances
        them together on a pool of streams; a new graph
        is uploaded on a background thread every `upload_every` seconds and the
        oldest graph is retired (its queued queries still finish).
plain   one query at a time in arrival order, each a blocking single-query
        call on one stream (the plain kernels without batching).

Latency of a query = completion time - arrival time (queueing included).
Traversed edges of a query = out-edges of the vertices it reaches; they are
measured once per (graph, source) pair with a BFS before the runs, so the
served run reads no results back.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass

import numpy as np

from . import gen, gg

SERVE_STREAM = 0x5E7E


@dataclass
class Trace:
    t: np.ndarray        # arrival seconds
    graph: np.ndarray    # index into the graph list (pool, then uploads)
    algo: np.ndarray     # 0 SSSP, 1 BFS
    source: np.ndarray   # vertex id


def make_graph(i, scale, seed=gen.MASTER_SEED, ef=16):
    return gen.rmat(scale, ef << scale, stream=SERVE_STREAM + 17 * i + scale, seed=seed,
                    name=f"pool{i}-rmat{scale}")


def pool_scales(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(lo, hi + 1, size=count)]


def make_trace(rate, duration, graphs_at, sources, seed):
    """Poisson arrivals; each query picks a graph among those resident at its
    arrival time (graphs_at(t) -> list of graph indices), an algorithm
    (50/50) and one of that graph's sources."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.2) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration]
    g = np.empty(len(t), np.int64)
    for i, ti in enumerate(t):
        cand = graphs_at(ti)
        g[i] = cand[rng.integers(0, len(cand))]
    algo = rng.integers(0, 2, size=len(t))
    src = np.array([sources[int(gi)][rng.integers(0, len(sources[int(gi)]))] for gi in g],
                   np.int64)
    return Trace(t, g, algo, src)


def traversed_edges(graph: gg.Graph, hg, srcs):
    """Out-edges of the vertices each source reaches (one BFS per source)."""
    import torch
    deg = torch.as_tensor(hg.degrees(), device="cuda")
    out = {}
    buf = torch.empty(hg.n, dtype=torch.int32, device="cuda")
    for s in srcs:
        graph.bfs(int(s), out=buf)
        out[int(s)] = int(deg[buf != gg.INF].sum().item())
    return out


def percentile(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def run_served(hosts, trace, slots=32, mem_budget=8 << 30, upload_every=5.0, n_pool=None,
               log=None, service=None):
    """Serve the trace; returns per-query latencies (s) in trace order, the
    per-query status and the wall time of the run.  With `service` (an array
    of the trace's length) the time from admission to completion of each
    query is stored there."""
    import torch
    n_pool = n_pool or len(hosts)
    srv = gg.Server(slots, mem_budget)
    gid = {}
    for i in range(n_pool):
        gid[i] = srv.add_graph(gg.Graph.from_host(hosts[i], symmetrize=True))
    lock = threading.Lock()
    stop = threading.Event()

    retire = []  # (due time, graph index) of uploads done, oldest first

    def uploader(t0):
        # a new graph every upload_every seconds; the main loop retires the
        # oldest one once every query that arrived before the upload is in
        k = n_pool
        while k < len(hosts) and not stop.is_set():
            due = (k - n_pool + 1) * upload_every
            while time.perf_counter() - t0 < due and not stop.is_set():
                time.sleep(0.01)
            if stop.is_set():
                break
            s = torch.cuda.Stream()
            g = gg.Graph.from_host(hosts[k], symmetrize=True, stream=s)
            with lock:
                gid[k] = srv.add_graph(g)
                retire.append((due, k - n_pool))
            k += 1

    # output buffers: a small free list per graph (a buffer is reused after
    # its query finished; nothing is read back)
    free_bufs = {i: [] for i in range(len(hosts))}

    def buf_for(i):
        lst = free_bufs[i]
        return lst.pop() if lst else torch.empty(hosts[i].n, dtype=torch.int32, device="cuda")

    lat = np.full(len(trace.t), np.nan)
    status = np.zeros(len(trace.t), np.int32)
    inflight = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = threading.Thread(target=uploader, args=(t0,), daemon=True)
    th.start()
    nxt = 0
    done = 0
    nq = len(trace.t)
    next_log = 10.0
    while done < nq:
        now = time.perf_counter() - t0
        while nxt < nq and trace.t[nxt] <= now:
            gi = int(trace.graph[nxt])
            with lock:
                while gi not in gid:  # its upload is still in progress
                    lock.release()
                    time.sleep(0.0005)
                    lock.acquire()
                b = buf_for(gi)
                qid = srv.submit(gid[gi], int(trace.algo[nxt]), int(trace.source[nxt]), b)
            inflight[qid] = (nxt, gi, b)
            nxt += 1
        with lock:
            while retire and (nxt >= nq or trace.t[nxt] >= retire[0][0]):
                srv.remove_graph(gid[retire.pop(0)[1]])
            res = srv.poll()
        tnow = time.perf_counter() - t0
        for qid, st, rounds, ts, ta, td in res:
            k, gi, b = inflight.pop(qid)
            lat[k] = tnow - trace.t[k]
            status[k] = st
            if service is not None:
                service[k] = td - ta
            free_bufs[gi].append(b)
            done += 1
        if log is not None and tnow >= next_log:
            log(f"[serve] served: {tnow:.0f}s, {done}/{nq} queries done")
            next_log += 10.0
        if not res and nxt < nq and trace.t[nxt] > now + 0.0005:
            time.sleep(0.0001)
    wall = time.perf_counter() - t0
    stop.set()
    th.join()
    torch.cuda.synchronize()
    srv.free()
    return lat, status, wall


def run_plain(hosts, trace, n_pool=None, upload_every=5.0, service=None, log=None):
    """One blocking query at a time in arrival order, graphs uploaded when
    they first appear in the trace (upload time not charged to queries).
    With `service` the time of each call is stored there."""
    import torch
    graphs = {}
    lat = np.full(len(trace.t), np.nan)
    out = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    upload_s = 0.0
    next_log = 10.0
    for k in range(len(trace.t)):
        gi = int(trace.graph[k])
        if gi not in graphs:
            tu = time.perf_counter()
            graphs[gi] = gg.Graph.from_host(hosts[gi], symmetrize=True)
            out[gi] = torch.empty(hosts[gi].n, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            upload_s += time.perf_counter() - tu
        now = time.perf_counter() - t0 - upload_s
        if now < trace.t[k]:
            time.sleep(trace.t[k] - now)
        g = graphs[gi]
        tq = time.perf_counter()
        if trace.algo[k] == 0:
            g.sssp(int(trace.source[k]), out=out[gi])
        else:
            g.bfs(int(trace.source[k]), out=out[gi])
        torch.cuda.synchronize()
        tn = time.perf_counter()
        if service is not None:
            service[k] = tn - tq
        lat[k] = tn - t0 - upload_s - trace.t[k]
        if log is not None and tn - t0 >= next_log:
            log(f"[serve] plain: {tn - t0:.0f}s, {k + 1}/{len(trace.t)} queries done")
            next_log += 10.0
    wall = time.perf_counter() - t0 - upload_s
    for g in graphs.values():
        g.free()
    return lat, wall
