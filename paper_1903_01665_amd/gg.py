"""Thin ctypes binding of libgg (the C ABI declared in include/gg.h).

Argument marshalling only: every step of a traversal runs in the HIP kernels
of ``libgg.so``.  PyTorch provides device memory (int32 tensors on cuda:0) and
the current HIP stream.  There is no fallback: if ``libgg.so`` is missing or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgg.so")
INF = 2**31 - 1

# enums of gg.h
VERTEX, EDGE, MODE_AUTO = 0, 1, 2
SYNC, ASYNC, SCHED_AUTO, NEARFAR, DIROPT, UNIONFIND = 0, 1, 2, 3, 4, 5
MAP_AUTO, MAP_THREAD, MAP_WAVE, MAP_BALANCED = 0, 1, 2, 3
ALGO_SSSP, ALGO_BFS, ALGO_CC, ALGO_MSF = 0, 1, 2, 3
SYMMETRIZE, INPUT_ON_DEVICE, SYMMETRIC, TRANSPOSE = 1, 2, 4, 8
RENUMBER, KEEP_ORDER = 16, 32
OPT_CC_NO_JUMP = 1
OPT_PROFILE = 2
OPT_LISTS_CHECKED, OPT_LISTS_DIRECT = 4, 8
KINDS = ("round", "heavy", "aux")

STATUS = {0: "GG_OK", -1: "GG_EINVAL", -2: "GG_ENOMEM", -3: "GG_EHIP", -4: "GG_EBUSY",
          -5: "GG_ENOTSUP", -6: "GG_ETIMEOUT", -7: "GG_EITER"}

# every symbol include/gg.h declares
EXPORTS = ["gg_graph_upload", "gg_graph_free", "gg_graph_info", "gg_graph_error", "gg_sssp",
           "gg_bfs", "gg_cc", "gg_ws_create", "gg_ws_free", "gg_sssp_ex", "gg_bfs_ex",
           "gg_cc_ex", "gg_msf", "gg_last_stats", "gg_last_profile", "gg_resolve", "gg_status_str",
           "gg_version", "gg_tune_set", "gg_tune_get", "gg_class_of", "gg_tune_lookup",
           "gg_graph_probe", "gg_graph_class", "gg_batch_create", "gg_batch_run",
           "gg_batch_offsets", "gg_batch_info", "gg_batch_group", "gg_batch_free",
           "gg_server_create", "gg_server_add_graph", "gg_server_remove_graph",
           "gg_server_submit", "gg_server_poll", "gg_server_state", "gg_server_now",
           "gg_server_free", "gg_sssp_async", "gg_bfs_async", "gg_cc_async", "gg_ticket_query",
           "gg_ticket_wait", "gg_ticket_stream_wait", "gg_ticket_times", "gg_ticket_free",
           "gg_bfs_noalloc", "gg_graph_order"]
BATCH_NO_GRAPH, BATCH_ONE_GROUP = 1, 2

TUNE_TABLE = os.path.join(_HERE, "tune_table.json")


class GGError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("sched", ctypes.c_int32), ("mapping", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
                ("heavy_threshold", ctypes.c_int32), ("time_limit_ms", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("delta", ctypes.c_int32),
                ("hops", ctypes.c_int32), ("far_degree", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]


class Stats(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("mode", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("mapping", ctypes.c_int32), ("status", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("edges_processed", ctypes.c_int64),
                ("vertices_processed", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("pushes", ctypes.c_int64), ("reserved", ctypes.c_int64 * 4)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class TuneEntry(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("size_class", ctypes.c_int32),
                ("skew_class", ctypes.c_int32), ("depth_class", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("sched", ctypes.c_int32), ("mapping", ctypes.c_int32),
                ("delta_eighths", ctypes.c_int32), ("hops", ctypes.c_int32),
                ("far_degree", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("source", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class QueryResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class KindProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int32), ("total_ms", ctypes.c_float),
                ("edges_processed", ctypes.c_int64), ("vertices_processed", ctypes.c_int64),
                ("updates", ctypes.c_int64), ("pushes", ctypes.c_int64),
                ("swept_edges", ctypes.c_int64)]


class Profile(ctypes.Structure):
    _fields_ = [("profiled", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("kind", KindProfile * 3), ("begin_ms", ctypes.c_double),
                ("end_ms", ctypes.c_double)]

    def as_dict(self):
        return {"profiled": bool(self.profiled), "rounds": self.rounds,
                "begin_ms": self.begin_ms, "end_ms": self.end_ms,
                **{KINDS[i]: {k: getattr(self.kind[i], k) for k, _ in KindProfile._fields_}
                   for i in range(3)}}


_lib = None


def lib():
    """The loaded libgg.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch first: its wheel carries its own HIP runtime, which its libraries
    # ask for by a name that does not match the soname libgg.so asks for.
    # Loaded in this order there is one runtime in the process (libgg.so's
    # request matches the loaded soname); the other order loads two, and
    # torch's streams and device memory are then foreign to libgg.so.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
    P = ctypes.POINTER
    L.gg_graph_upload.argtypes = [i32, i64, vp, vp, vp, u32, vp, P(vp)]
    L.gg_graph_free.argtypes = [vp]
    L.gg_graph_info.argtypes = [vp, P(i32), P(i64), P(i32), P(i32), P(i32)]
    L.gg_graph_error.argtypes = [vp]
    L.gg_graph_order.argtypes = [vp, P(i32)]
    L.gg_sssp.argtypes = [vp, i32, i32, i32, vp, vp]
    L.gg_bfs.argtypes = [vp, i32, i32, i32, vp, vp]
    L.gg_cc.argtypes = [vp, i32, i32, vp, vp]
    L.gg_ws_create.argtypes = [vp, P(vp)]
    L.gg_ws_free.argtypes = [vp]
    L.gg_sssp_ex.argtypes = [vp, vp, i32, P(Opts), vp, vp]
    L.gg_bfs_ex.argtypes = [vp, vp, i32, P(Opts), vp, vp]
    L.gg_cc_ex.argtypes = [vp, vp, P(Opts), vp, vp]
    L.gg_msf.argtypes = [vp, vp, vp, P(i64), P(i64), vp]
    L.gg_last_stats.argtypes = [vp, vp, P(Stats)]
    L.gg_last_profile.argtypes = [vp, vp, P(Profile)]
    L.gg_resolve.argtypes = [vp, i32, P(Opts), P(Opts)]
    L.gg_tune_set.argtypes = [P(TuneEntry), i32]
    L.gg_tune_get.argtypes = [P(TuneEntry), i32]
    L.gg_class_of.argtypes = [i64, i32, i32, i32, P(i32), P(i32), P(i32)]
    L.gg_tune_lookup.argtypes = [i32, i32, i32, i32, P(TuneEntry)]
    L.gg_graph_probe.argtypes = [vp, vp]
    L.gg_graph_class.argtypes = [vp, P(i32), P(i32), P(i32)]
    L.gg_batch_create.argtypes = [P(Instance), i32, u32, vp, P(vp)]
    L.gg_batch_run.argtypes = [vp, vp, vp]
    L.gg_batch_offsets.argtypes = [vp, P(i64)]
    L.gg_batch_info.argtypes = [vp, P(i32), P(i64), P(i64)]
    L.gg_batch_group.argtypes = [vp, i32, P(i32), P(i32), P(i64), P(i64), P(i32), P(i32),
                                 P(i32), P(i32), P(i32)]
    L.gg_batch_free.argtypes = [vp]
    L.gg_server_create.argtypes = [i32, i64, P(vp)]
    L.gg_server_add_graph.argtypes = [vp, vp, P(i32)]
    L.gg_server_remove_graph.argtypes = [vp, i32]
    L.gg_server_submit.argtypes = [vp, i32, i32, i32, vp, vp, P(i64)]
    L.gg_server_poll.argtypes = [vp, P(QueryResult), i32, P(i32)]
    L.gg_server_state.argtypes = [vp, P(i32), P(i32), P(i64)]
    L.gg_server_now.argtypes = [vp]
    L.gg_server_now.restype = ctypes.c_double
    L.gg_server_free.argtypes = [vp]
    L.gg_sssp_async.argtypes = [vp, vp, i32, P(Opts), vp, vp, P(vp)]
    L.gg_bfs_async.argtypes = [vp, vp, i32, P(Opts), vp, vp, P(vp)]
    L.gg_cc_async.argtypes = [vp, vp, P(Opts), vp, vp, P(vp)]
    L.gg_ticket_query.argtypes = [vp]
    L.gg_ticket_wait.argtypes = [vp]
    L.gg_ticket_stream_wait.argtypes = [vp, vp]
    L.gg_ticket_times.argtypes = [vp, vp, P(ctypes.c_float), P(ctypes.c_float), P(i32)]
    L.gg_ticket_free.argtypes = [vp]
    L.gg_bfs_noalloc.argtypes = [vp, i32, P(Opts), vp, vp]
    L.gg_status_str.argtypes = [i32]
    L.gg_status_str.restype = ctypes.c_char_p
    L.gg_version.argtypes = []
    for f in EXPORTS:
        if f not in ("gg_status_str", "gg_server_now"):
            getattr(L, f).restype = ctypes.c_int32
    if L.gg_version() != 1:
        raise RuntimeError("libgg.so version mismatch")
    _lib = L
    if os.path.exists(TUNE_TABLE):
        load_tune_table(TUNE_TABLE)
    return L


# ------------------------------------------------------------- tuning ------
def tune_set(entries):
    """Install a tuning table: a list of dicts with algo, size_class,
    skew_class, depth_class, mode, sched, mapping (and optionally delta_eighths,
    hops, far_degree)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        for k in ("algo", "size_class", "skew_class", "depth_class", "mode", "sched", "mapping"):
            setattr(arr[i], k, int(e[k]))
        arr[i].delta_eighths = int(e.get("delta_eighths", 0))
        arr[i].hops = int(e.get("hops", 0))
        arr[i].far_degree = int(e.get("far_degree", 0))
    _check(lib().gg_tune_set(arr, len(entries)), "gg_tune_set")


def tune_get():
    n = lib().gg_tune_get(None, 0)
    arr = (TuneEntry * max(1, n))()
    lib().gg_tune_get(arr, n)
    return [{k: getattr(arr[i], k) for k, _ in TuneEntry._fields_} for i in range(n)]


def load_tune_table(path):
    import json
    with open(path) as f:
        tune_set(json.load(f)["entries"])


def class_of(m, n, max_out_degree, levels=-1):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().gg_class_of(m, n, max_out_degree, levels, ctypes.byref(a), ctypes.byref(b),
                             ctypes.byref(c)), "gg_class_of")
    return a.value, b.value, c.value


def tune_lookup(algo, size_class, skew_class, depth_class, full=False):
    """(mode, sched, mapping), or with full=True the whole chosen entry as a
    dict (mode, sched, mapping, delta_eighths, hops, far_degree)."""
    t = TuneEntry()
    _check(lib().gg_tune_lookup(algo, size_class, skew_class, depth_class, ctypes.byref(t)),
           "gg_tune_lookup")
    if full:
        return {k: getattr(t, k) for k in ("mode", "sched", "mapping", "delta_eighths", "hops",
                                           "far_degree")}
    return (t.mode, t.sched, t.mapping)


def _check(rc, what):
    if rc != 0:
        raise GGError(rc, what)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def make_opts(mode=MODE_AUTO, sched=SCHED_AUTO, mapping=MAP_AUTO, max_blocks=0, flags=0,
              time_limit_ms=0, delta=0, hops=0, far_degree=0) -> Opts:
    o = Opts()
    o.mode, o.sched, o.mapping = mode, sched, mapping
    o.max_blocks, o.flags, o.time_limit_ms, o.delta = max_blocks, flags, time_limit_ms, delta
    o.hops, o.far_degree = hops, far_degree
    return o


class Workspace:
    """Per-query scratch so that several traversals of one graph overlap."""

    def __init__(self, graph: "Graph"):
        self.graph = graph
        h = ctypes.c_void_p()
        _check(lib().gg_ws_create(graph.handle, ctypes.byref(h)), "gg_ws_create")
        self.handle = h

    def free(self):
        if self.handle:
            _check(lib().gg_ws_free(self.handle), "gg_ws_free")
            self.handle = None


class Graph:
    """A graph resident in HBM (CSR, edge list, optional both-directions CSR)."""

    def __init__(self, n, row_ptr, col, w=None, symmetrize=False, symmetric=False, stream=None,
                 transpose=False, renumber=None):
        """renumber: None lets the library decide (skewed graphs of >= 2^20
        edges are stored hottest vertex first), True forces it, False keeps
        the caller's order.  Ids at the interface are the caller's either way."""
        L = lib()
        self.n = int(n)
        self._row, prow = _arr(row_ptr)
        self._col, pcol = _arr(col if len(col) else np.zeros(1, np.int32))
        m = int(self._row[-1])
        pw = None
        if w is not None:
            self._w, pw = _arr(w if len(w) else np.zeros(1, np.int32))
        flags = (SYMMETRIZE if symmetrize else 0) | (SYMMETRIC if symmetric else 0) | \
            (TRANSPOSE if transpose else 0) | \
            (0 if renumber is None else RENUMBER if renumber else KEEP_ORDER)
        h = ctypes.c_void_p()
        _check(L.gg_graph_upload(self.n, m, prow, pcol, pw, flags, _stream_ptr(stream),
                                 ctypes.byref(h)), "gg_graph_upload")
        self.handle = h
        self.m = m
        del self._row, self._col
        if w is not None:
            del self._w

    @classmethod
    def from_host(cls, hg, symmetrize=False, stream=None, transpose=False, renumber=None):
        """Upload a :class:`paper_1903_01665_amd.gen.HostGraph`."""
        return cls(hg.n, hg.row_ptr, hg.col, hg.w, symmetrize=symmetrize and not hg.symmetric,
                   symmetric=hg.symmetric, stream=stream, transpose=transpose, renumber=renumber)

    def renumbered(self):
        """True when the library stores the graph in its own vertex order."""
        r = ctypes.c_int32()
        _check(lib().gg_graph_order(self.handle, ctypes.byref(r)), "gg_graph_order")
        return bool(r.value)

    def info(self):
        n, m, d, hw, hs = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(),
                           ctypes.c_int32())
        _check(lib().gg_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                   ctypes.byref(d), ctypes.byref(hw), ctypes.byref(hs)),
               "gg_graph_info")
        return {"n": n.value, "m": m.value, "max_out_degree": d.value,
                "weighted": bool(hw.value), "has_sym": bool(hs.value)}

    def free(self):
        if getattr(self, "handle", None):
            _check(lib().gg_graph_free(self.handle), "gg_graph_free")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.gg_graph_free(self.handle)
                self.handle = None
        except Exception:
            pass

    # -- traversals ---------------------------------------------------------
    def _out(self, out):
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        if out.dtype != torch.int32 or not out.is_cuda or out.numel() < self.n or \
                not out.is_contiguous():
            raise ValueError("output must be a contiguous int32 cuda tensor of >= n elements")
        return out

    def _run(self, fn, what, args, opts, out, ws, stream):
        out = self._out(out)
        o = opts if opts is not None else make_opts()
        wsh = ws.handle if ws is not None else None
        rc = fn(self.handle, wsh, *args, ctypes.byref(o), ctypes.c_void_p(out.data_ptr()),
                _stream_ptr(stream))
        _check(rc, what)
        return out

    def sssp(self, source, mode=MODE_AUTO, sched=SCHED_AUTO, mapping=MAP_AUTO, out=None,
             ws=None, stream=None, opts=None):
        o = opts or make_opts(mode, sched, mapping)
        return self._run(lib().gg_sssp_ex, "gg_sssp", [int(source)], o, out, ws, stream)

    def bfs(self, source, mode=MODE_AUTO, sched=SCHED_AUTO, mapping=MAP_AUTO, out=None,
            ws=None, stream=None, opts=None):
        o = opts or make_opts(mode, sched, mapping)
        return self._run(lib().gg_bfs_ex, "gg_bfs", [int(source)], o, out, ws, stream)

    def cc(self, mode=MODE_AUTO, sched=SCHED_AUTO, mapping=MAP_AUTO, out=None, ws=None,
           stream=None, opts=None):
        o = opts or make_opts(mode, sched, mapping)
        return self._run(lib().gg_cc_ex, "gg_cc", [], o, out, ws, stream)

    # -- host-asynchronous forms (return at once with a Ticket) -------------
    def _run_async(self, fn, what, args, opts, out, ws, stream):
        out = self._out(out)
        o = opts if opts is not None else make_opts()
        wsh = ws.handle if ws is not None else None
        t = ctypes.c_void_p()
        _check(fn(self.handle, wsh, *args, ctypes.byref(o), ctypes.c_void_p(out.data_ptr()),
                  _stream_ptr(stream), ctypes.byref(t)), what)
        return Ticket(t, out)

    def sssp_async(self, source, out=None, ws=None, stream=None, opts=None) -> "Ticket":
        return self._run_async(lib().gg_sssp_async, "gg_sssp_async", [int(source)], opts, out,
                               ws, stream)

    def bfs_async(self, source, out=None, ws=None, stream=None, opts=None) -> "Ticket":
        return self._run_async(lib().gg_bfs_async, "gg_bfs_async", [int(source)], opts, out,
                               ws, stream)

    def cc_async(self, out=None, ws=None, stream=None, opts=None) -> "Ticket":
        return self._run_async(lib().gg_cc_async, "gg_cc_async", [], opts, out, ws, stream)

    def msf(self, out=None, ws=None, stream=None):
        """Minimum spanning forest: (uint8 cuda tensor marking the forest's
        edges in CSR order, total weight, edge count)."""
        import torch
        m = self.m
        if out is None:
            out = torch.empty(max(m, 1), dtype=torch.uint8, device="cuda")
        if out.dtype != torch.uint8 or not out.is_cuda or out.numel() < m or \
                not out.is_contiguous():
            raise ValueError("output must be a contiguous uint8 cuda tensor of >= m elements")
        tw, ne = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gg_msf(self.handle, ws.handle if ws is not None else None,
                            ctypes.c_void_p(out.data_ptr()), ctypes.byref(tw), ctypes.byref(ne),
                            _stream_ptr(stream)), "gg_msf")
        return out[:m], tw.value, ne.value

    def stats(self, ws=None) -> dict:
        s = Stats()
        rc = lib().gg_last_stats(self.handle, ws.handle if ws is not None else None,
                                 ctypes.byref(s))
        d = s.as_dict()
        d["rc"] = rc
        return d

    def profile(self, ws=None) -> dict:
        p = Profile()
        _check(lib().gg_last_profile(self.handle, ws.handle if ws is not None else None,
                                     ctypes.byref(p)), "gg_last_profile")
        return p.as_dict()

    def probe(self, stream=None):
        """Measure the depth class (one BFS) so AUTO can use it."""
        _check(lib().gg_graph_probe(self.handle, _stream_ptr(stream)), "gg_graph_probe")
        return self.graph_class()

    def graph_class(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gg_graph_class(self.handle, ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)), "gg_graph_class")
        return a.value, b.value, c.value

    def resolve(self, algo, opts=None) -> Opts:
        out = Opts()
        _check(lib().gg_resolve(self.handle, algo, ctypes.byref(opts or make_opts()),
                                ctypes.byref(out)), "gg_resolve")
        return out


class Ticket:
    """A host-asynchronous traversal in flight (gg_*_async in gg.h).  Holds
    the output tensor so that it stays allocated until the traversal ends."""

    def __init__(self, handle, out):
        self.handle = handle
        self.out = out

    def query(self) -> bool:
        """True once every kernel of the traversal has completed."""
        rc = lib().gg_ticket_query(self.handle)
        if rc == -4:
            return False
        _check(rc, "gg_ticket_query")
        return True

    def wait(self):
        """Block until the traversal has completed; returns its output."""
        _check(lib().gg_ticket_wait(self.handle), "gg_ticket_wait")
        return self.out

    def stream_wait(self, stream=None):
        """Make `stream` (default: the current one) wait for the traversal."""
        _check(lib().gg_ticket_stream_wait(self.handle, _stream_ptr(stream)),
               "gg_ticket_stream_wait")
        return self.out

    def times(self, ref: "Ticket" = None):
        """(begin_ms, end_ms, rounds) on the device, from ref's begin."""
        b, e, r = ctypes.c_float(), ctypes.c_float(), ctypes.c_int32()
        _check(lib().gg_ticket_times(self.handle, ref.handle if ref is not None else None,
                                     ctypes.byref(b), ctypes.byref(e), ctypes.byref(r)),
               "gg_ticket_times")
        return b.value, e.value, r.value

    def free(self):
        if getattr(self, "handle", None):
            _check(lib().gg_ticket_free(self.handle), "gg_ticket_free")
            self.handle = None
            self.out = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.gg_ticket_free(self.handle)
                self.handle = None
        except Exception:
            pass


class Batch:
    """Many independent SSSP/BFS instances run together (gg_batch_* in gg.h).

    ``instances``: list of (algo, HostGraph, source) with algo ALGO_SSSP or
    ALGO_BFS.  ``run()`` returns one int32 cuda tensor holding every result;
    instance i's is ``out[off[i]: off[i] + n_i]`` with ``off = offsets()``.
    """

    def __init__(self, instances, flags=0, stream=None):
        L = lib()
        arr = (Instance * len(instances))()
        keep = []
        for i, (algo, hg, src) in enumerate(instances):
            row, prow = _arr(hg.row_ptr)
            col, pcol = _arr(hg.col if len(hg.col) else np.zeros(1, np.int32))
            pw = None
            if hg.w is not None:
                w, pw = _arr(hg.w if len(hg.w) else np.zeros(1, np.int32))
                keep.append(w)
            keep += [row, col]
            arr[i].algo, arr[i].n, arr[i].m = int(algo), int(hg.n), int(hg.m)
            arr[i].row_ptr, arr[i].col, arr[i].w = prow, pcol, pw
            arr[i].source = int(src)
        h = ctypes.c_void_p()
        _check(L.gg_batch_create(arr, len(instances), flags, _stream_ptr(stream),
                                 ctypes.byref(h)), "gg_batch_create")
        self.handle = h
        self.count = len(instances)
        self.sizes = [int(hg.n) for _, hg, _ in instances]
        info = self.info()
        self.total_n = info["total_n"]

    def info(self):
        g, n, m = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gg_batch_info(self.handle, ctypes.byref(g), ctypes.byref(n),
                                   ctypes.byref(m)), "gg_batch_info")
        return {"groups": g.value, "total_n": n.value, "total_m": m.value}

    def group(self, i):
        v = [ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(),
             ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
             ctypes.c_int32()]
        _check(lib().gg_batch_group(self.handle, i, *[ctypes.byref(x) for x in v]),
               "gg_batch_group")
        keys = ("algo", "instances", "n", "m", "mode", "sched", "mapping", "captured_rounds",
                "last_rounds")
        return {k: x.value for k, x in zip(keys, v)}

    def offsets(self):
        off = np.zeros(self.count, np.int64)
        _check(lib().gg_batch_offsets(self.handle, off.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int64))), "gg_batch_offsets")
        return off

    def run(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.total_n, dtype=torch.int32, device="cuda")
        if out.dtype != torch.int32 or not out.is_cuda or out.numel() < self.total_n:
            raise ValueError("output must be an int32 cuda tensor of >= total_n elements")
        _check(lib().gg_batch_run(self.handle, ctypes.c_void_p(out.data_ptr()),
                                  _stream_ptr(stream)), "gg_batch_run")
        return out

    def free(self):
        if getattr(self, "handle", None):
            _check(lib().gg_batch_free(self.handle), "gg_batch_free")
            self.handle = None


class Server:
    """Continuous-batching query server (gg_server_* in gg.h).

    ``add_graph`` hands an uploaded :class:`Graph` to the server (which owns
    it from then on); ``submit`` queues a query whose result goes to a
    caller-owned int32 cuda tensor; the server's own native thread admits and
    advances queries; ``poll`` returns the queries that finished since the
    last poll as (id, status, rounds, t_submit, t_admit, t_done).
    """

    def __init__(self, slots=16, mem_budget_bytes=0):
        h = ctypes.c_void_p()
        _check(lib().gg_server_create(slots, mem_budget_bytes, ctypes.byref(h)),
               "gg_server_create")
        self.handle = h
        self._res = (QueryResult * 4096)()
        self._graphs = {}
        self._outs = {}  # query id -> output tensor, held until the query is polled

    def add_graph(self, graph: Graph) -> int:
        gid = ctypes.c_int32()
        _check(lib().gg_server_add_graph(self.handle, graph.handle, ctypes.byref(gid)),
               "gg_server_add_graph")
        graph.handle = None  # owned by the server now
        self._graphs[gid.value] = graph.n
        return gid.value

    def remove_graph(self, gid: int):
        _check(lib().gg_server_remove_graph(self.handle, gid), "gg_server_remove_graph")
        self._graphs.pop(gid, None)

    def submit(self, gid, algo, source, out, stream=None) -> int:
        """Queue a query writing `out` (an int32 cuda tensor of >= n elements
        of that graph); it runs after the work enqueued on `stream` (default:
        the current stream) so far."""
        import torch
        n = self._graphs.get(gid)
        if n is None:
            raise GGError(-1, "gg_server_submit: unknown graph")
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous() or \
                out.numel() < n:
            raise ValueError("output must be a contiguous int32 cuda tensor of >= n elements")
        qid = ctypes.c_int64()
        _check(lib().gg_server_submit(self.handle, gid, algo, int(source),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream),
                                      ctypes.byref(qid)), "gg_server_submit")
        self._outs[qid.value] = out
        return qid.value

    def poll(self):
        n = ctypes.c_int32()
        _check(lib().gg_server_poll(self.handle, self._res, len(self._res), ctypes.byref(n)),
               "gg_server_poll")
        done = [(r.id, r.status, r.rounds, r.t_submit, r.t_admit, r.t_done)
                for r in self._res[: n.value]]
        for d in done:
            self._outs.pop(d[0], None)
        return done

    def state(self):
        q, f, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().gg_server_state(self.handle, ctypes.byref(q), ctypes.byref(f),
                                     ctypes.byref(b)), "gg_server_state")
        return {"queued": q.value, "in_flight": f.value, "state_bytes": b.value}

    def now(self) -> float:
        return lib().gg_server_now(self.handle)

    def free(self):
        if getattr(self, "handle", None):
            _check(lib().gg_server_free(self.handle), "gg_server_free")
            self.handle = None


def status_str(code: int) -> str:
    return lib().gg_status_str(code).decode()
