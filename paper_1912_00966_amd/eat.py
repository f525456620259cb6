"""Python binding of libeat (C ABI in include/eat.h).

Argument marshalling only: every step of a query runs in the library's HIP
kernels.  PyTorch provides device memory (result slabs, probe arrays) and the
stream a call is enqueued on.  The names follow the C ABI (``eat_graph_build``,
``eat_query``, ``eat_query_batch`` ...); ``Graph`` and ``Batch`` wrap the
opaque handles.  If ``libeat.so`` is missing, every call raises: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeat.so")
EAT_INF = np.iinfo(np.int32).max

EAT_OK = 0
EAT_ERR_INVALID_ARGUMENT = 1
EAT_ERR_OUT_OF_MEMORY = 2
EAT_ERR_DEVICE = 3
EAT_ERR_NOT_CONVERGED = 4
EAT_ERR_BUSY = 5
EAT_ERR_UNSUPPORTED = 6

EAT_LAYOUT_HYBRID = 0
EAT_LAYOUT_FLAT = 1
EAT_MODE_AUTO = 0
EAT_MODE_FRONTIER = 1
EAT_MODE_TOPOLOGY = 2
EAT_HEADERS_AUTO = 0
EAT_HEADERS_GRID = 1
EAT_HEADERS_COMPACT = 2
EAT_ORDER_AUTO = 0
EAT_ORDER_LOCALITY = 1
EAT_ORDER_LONGEST_FIRST = 2
EAT_ORDER_BANDED = 3

# every function include/eat.h declares
EXPORTS = (
    "eat_layout_build", "eat_layout_build_trips", "eat_layout_free", "eat_layout_info", "eat_layout_view_get",
    "eat_graph_build", "eat_graph_build_trips", "eat_graph_upload", "eat_graph_free", "eat_graph_info", "eat_graph_failures",
    "eat_query", "eat_query_goal", "eat_batch_create", "eat_batch_create_goal", "eat_batch_run", "eat_batch_wait",
    "eat_batch_free", "eat_parents", "eat_profile",
    "eat_batch_options", "eat_batch_tune", "eat_query_batch_static",
    "eat_query_batch", "eat_next_departure", "eat_status_string", "eat_last_error",
    "eat_version", "eat_session_create", "eat_session_admit", "eat_session_step",
    "eat_session_poll", "eat_session_sync", "eat_session_result", "eat_session_copy",
    "eat_session_query_stats",
    "eat_session_release", "eat_session_free", "eat_session_serve",
    "eat_ap_cover", "eat_esdg_levels", "eat_variant_graph_build", "eat_variant_graph_info", "eat_variant_query",
    "eat_variant_graph_free",
)

# the paper's algorithm ladder (eat_variant)
EAT_VARIANT_CONNECTION = 0
EAT_VARIANT_CONNECTION_TYPE = 1
EAT_VARIANT_CONNECTION_TYPE_AP = 2
EAT_VARIANT_CLUSTER_AP = 3
EAT_VARIANT_EDGE = 4
EAT_VARIANT_WARPS = 5
EAT_VARIANT_ESDG = 6
VARIANT_NAMES = {0: "connection", 1: "connection-type", 2: "connection-type-AP", 3: "cluster-AP", 4: "edge",
                 5: "warps", 6: "ESDG"}

_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p


class BuildOptions(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("cluster_seconds", ctypes.c_int32),
                ("n_threads", ctypes.c_int32), ("header_grid", ctypes.c_int32),
                ("subtrip_len", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("cluster_seconds", ctypes.c_int32), ("n_clusters", ctypes.c_int32),
                ("max_departure", ctypes.c_int32), ("max_types_per_vertex", ctypes.c_int32),
                ("n_conn_input", ctypes.c_int64), ("n_self_loops", ctypes.c_int64),
                ("n_duplicates", ctypes.c_int64), ("n_conn", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("n_types", ctypes.c_int64),
                ("n_headers", ctypes.c_int64), ("n_ap_clusters", ctypes.c_int64),
                ("n_array_clusters", ctypes.c_int64), ("n_pool", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("n_grid_entries", ctypes.c_int64),
                ("n_trips", ctypes.c_int64), ("n_shortcuts", ctypes.c_int64),
                ("subtrip_len", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LayoutView(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("n_vertices", ctypes.c_int32),
                ("cluster_seconds", ctypes.c_int32), ("n_clusters", ctypes.c_int32),
                ("n_types", ctypes.c_int64), ("n_headers", ctypes.c_int64),
                ("n_pool", ctypes.c_int64), ("vt", _i32p), ("order", _i32p), ("ty", _i32p),
                ("ty_mask_hi", _u32p), ("hdr", _i32p), ("pool", _i32p)]


class RunOptions(ctypes.Structure):
    _fields_ = [("threads_per_vertex", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("frontier_cap", ctypes.c_int32),
                ("table_cap", ctypes.c_int32), ("types_per_lane", ctypes.c_int32),
                ("headers", ctypes.c_int32), ("time_window", ctypes.c_int32),
                ("threads_per_query", ctypes.c_int32), ("query_order", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class QueryStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("sweep_rounds", ctypes.c_int32), ("max_frontier", ctypes.c_int32),
                ("reached", ctypes.c_int32), ("spilled", ctypes.c_int32),
                ("activations", ctypes.c_int64), ("type_evals", ctypes.c_int64),
                ("header_loads", ctypes.c_int64), ("pool_loads", ctypes.c_int64),
                ("improvements", ctypes.c_int64), ("elapsed_ns", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServeReport(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("launched", ctypes.c_int64), ("busy_waits", ctypes.c_int64),
                ("wall_s", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneOptions(ctypes.Structure):
    _fields_ = [("reps", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


class TuneResult(ctypes.Structure):
    _fields_ = [("options", RunOptions), ("ms", ctypes.c_float), ("reserved", ctypes.c_int32)]


class SessionOptions(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("n_streams", ctypes.c_int32),
                ("max_step_queries", ctypes.c_int32), ("run", RunOptions),
                ("reserved", ctypes.c_int32 * 4)]


class VariantBuildOptions(ctypes.Structure):
    _fields_ = [("cluster_seconds", ctypes.c_int32), ("esdg", ctypes.c_int32), ("n_threads", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class VariantInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_clusters", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_conn", ctypes.c_int64), ("n_types", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("n_type_aps", ctypes.c_int64), ("n_cluster_aps", ctypes.c_int64),
                ("n_esdg_edges", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class VariantOptions(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("warp_size", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("count", ctypes.c_int32), ("max_iterations", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class VariantStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("host_checks", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("examined", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class EatError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def lib():
    """The loaded libeat.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_00966_amd.build`"
                           " (there is no non-GPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    conn = [_i32p, _i32p, _i32p, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(BuildOptions)]
    L.eat_layout_build.argtypes = conn + [ctypes.POINTER(_vp)]
    conn_trips = [_i32p, _i32p, _i32p, _i32p, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(BuildOptions)]
    L.eat_layout_build_trips.argtypes = conn_trips + [ctypes.POINTER(_vp)]
    L.eat_graph_build_trips.argtypes = conn_trips + [_vp, ctypes.POINTER(_vp)]
    L.eat_layout_free.argtypes = [_vp]
    L.eat_layout_free.restype = None
    L.eat_layout_info.argtypes = [_vp, ctypes.POINTER(GraphInfo)]
    L.eat_layout_view_get.argtypes = [_vp, ctypes.POINTER(LayoutView)]
    L.eat_graph_build.argtypes = conn + [_vp, ctypes.POINTER(_vp)]
    L.eat_graph_upload.argtypes = [_vp, ctypes.POINTER(BuildOptions), _vp, ctypes.POINTER(_vp)]
    L.eat_graph_free.argtypes = [_vp]
    L.eat_graph_free.restype = None
    L.eat_graph_info.argtypes = [_vp, ctypes.POINTER(GraphInfo)]
    L.eat_graph_failures.argtypes = [_vp, _i32p]
    L.eat_query.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                            ctypes.POINTER(RunOptions), ctypes.POINTER(QueryStats)]
    L.eat_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, _i32p, _i32p, _i32p,
                                   ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(RunOptions),
                                   ctypes.POINTER(_vp)]
    L.eat_query_goal.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                 ctypes.POINTER(RunOptions), ctypes.POINTER(QueryStats)]
    L.eat_batch_create_goal.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, _i32p, _i32p, _i32p, _i32p,
                                        ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(RunOptions),
                                        ctypes.POINTER(_vp)]
    L.eat_parents.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp]
    L.eat_profile.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p,
                              _vp, _vp, ctypes.POINTER(RunOptions)]
    L.eat_ap_cover.argtypes = [_i32p, ctypes.c_int64, _i32p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.eat_esdg_levels.argtypes = [_i32p, _i32p, _i32p, _i32p, ctypes.c_int64, ctypes.c_int32, _i32p, _i32p,
                                  ctypes.POINTER(ctypes.c_int64)]
    L.eat_variant_graph_build.argtypes = conn[:6] + [ctypes.POINTER(VariantBuildOptions), ctypes.POINTER(_vp)]
    L.eat_variant_graph_info.argtypes = [_vp, ctypes.POINTER(VariantInfo)]
    L.eat_variant_query.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.POINTER(VariantOptions),
                                    ctypes.POINTER(VariantStats)]
    L.eat_variant_graph_free.argtypes = [_vp]
    L.eat_batch_run.argtypes = [_vp, _vp]
    L.eat_batch_wait.argtypes = [_vp, ctypes.POINTER(QueryStats)]
    L.eat_batch_free.argtypes = [_vp]
    L.eat_batch_free.restype = None
    L.eat_batch_options.argtypes = [_vp, ctypes.POINTER(RunOptions)]
    L.eat_batch_tune.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, _i32p, _i32p, _i32p, ctypes.c_int32,
                                 ctypes.POINTER(_vp), _vp, ctypes.POINTER(TuneOptions), ctypes.POINTER(RunOptions),
                                 ctypes.POINTER(TuneResult), ctypes.c_int32, _i32p]
    L.eat_query_batch.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, _i32p, _i32p, _i32p,
                                  ctypes.c_int32, ctypes.POINTER(_vp), _vp,
                                  ctypes.POINTER(RunOptions), ctypes.POINTER(QueryStats)]
    L.eat_query_batch_static.argtypes = L.eat_query_batch.argtypes
    L.eat_next_departure.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, _vp]
    L.eat_status_string.argtypes = [ctypes.c_int]
    L.eat_status_string.restype = ctypes.c_char_p
    L.eat_last_error.argtypes = []
    L.eat_last_error.restype = ctypes.c_char_p
    L.eat_version.argtypes = []
    L.eat_version.restype = ctypes.c_int32
    L.eat_session_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(SessionOptions),
                                     ctypes.POINTER(_vp)]
    L.eat_session_admit.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p]
    L.eat_session_step.argtypes = [_vp, _i32p]
    L.eat_session_poll.argtypes = [_vp, _i32p, ctypes.c_int32, _i32p]
    L.eat_session_sync.argtypes = [_vp]
    L.eat_session_result.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(_i32p), _i32p]
    L.eat_session_copy.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
    L.eat_session_query_stats.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(QueryStats)]
    L.eat_session_release.argtypes = [_vp, ctypes.c_int32]
    _f64p = ctypes.POINTER(ctypes.c_double)
    L.eat_session_serve.argtypes = [_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _f64p, ctypes.c_int32,
                                    ctypes.c_double, ctypes.POINTER(_vp), _vp, _f64p, ctypes.POINTER(ServeReport)]
    L.eat_session_free.argtypes = [_vp]
    L.eat_session_free.restype = None
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("eat_layout_free", "eat_graph_free", "eat_batch_free", "eat_status_string",
                        "eat_last_error", "eat_version", "eat_session_free", "eat_variant_graph_free"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != EAT_OK:
        msg = lib().eat_last_error().decode(errors="replace")
        raise EatError(status, msg or lib().eat_status_string(status).decode())


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr32(a):
    return a.ctypes.data_as(_i32p)


def _build_opts(layout, cluster_seconds, n_threads, header_grid=0, subtrip_len=0):
    o = BuildOptions()
    o.layout = int(layout)
    o.cluster_seconds = int(cluster_seconds)
    o.n_threads = int(n_threads)
    o.header_grid = int(header_grid)
    o.subtrip_len = int(subtrip_len)
    return o


def options_dict(o: RunOptions) -> dict:
    """The fields of a RunOptions structure (reserved words left out)."""
    return {name: int(getattr(o, name)) for name, _ in RunOptions._fields_ if name != "reserved"}


def _run_opts(options):
    if options is None:
        return None
    if isinstance(options, RunOptions):
        return options
    o = RunOptions()
    for k, v in dict(options).items():
        setattr(o, k, int(v))
    return o


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, n_min: int, what: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32:
        raise TypeError(f"{what} must be a CUDA int32 tensor")
    if not t.is_contiguous() or t.numel() < n_min:
        raise ValueError(f"{what} must be contiguous with at least {n_min} elements")
    return t.data_ptr()


# ---------------------------------------------------------------------------
# host layout
# ---------------------------------------------------------------------------
class Layout:
    """Host-side layout (eat_layout_build); needs no GPU."""

    def __init__(self, handle):
        self._h = handle

    def info(self) -> GraphInfo:
        gi = GraphInfo()
        _check(lib().eat_layout_info(self._h, ctypes.byref(gi)))
        return gi

    def view(self) -> dict:
        """Copies of the layout arrays as numpy arrays (see eat_layout_view)."""
        lv = LayoutView()
        _check(lib().eat_layout_view_get(self._h, ctypes.byref(lv)))

        def take(p, n, dt=np.int32):
            if n == 0 or not p:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(p, shape=(int(n),)).astype(dt, copy=True)

        out = dict(layout=lv.layout, n_vertices=lv.n_vertices, cluster_seconds=lv.cluster_seconds,
                   n_clusters=lv.n_clusters, n_types=lv.n_types, n_headers=lv.n_headers,
                   n_pool=lv.n_pool)
        out["vt"] = take(lv.vt, 2 * lv.n_vertices).reshape(-1, 2)
        out["order"] = take(lv.order, lv.n_vertices)
        out["ty"] = take(lv.ty, 4 * lv.n_types).reshape(-1, 4)
        out["ty_mask_hi"] = take(lv.ty_mask_hi, lv.n_types if lv.ty_mask_hi else 0, np.uint32)
        out["hdr"] = take(lv.hdr, 2 * lv.n_headers if lv.hdr else 0).reshape(-1, 2)
        out["pool"] = take(lv.pool, lv.n_pool)
        return out

    def free(self):
        if getattr(self, "_h", None):
            lib().eat_layout_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def eat_layout_build_trips(u, v, t, lam, trip, n_vertices, subtrip_len=0, layout=EAT_LAYOUT_HYBRID,
                           cluster_seconds=0, n_threads=0) -> Layout:
    """Host layout with sub-trip shortcuts (Section II-G); trip[i] = vehicle
    trip of connection i (-1: none); subtrip_len 0 = sqrt(mean trip length),
    -1 = sqrt(k) per trip, r >= 1 fixed."""
    u, v, t, lam, trip = (_i32(x) for x in (u, v, t, lam, trip))
    h = _vp()
    o = _build_opts(layout, cluster_seconds, n_threads, 0, subtrip_len)
    _check(lib().eat_layout_build_trips(_ptr32(u), _ptr32(v), _ptr32(t), _ptr32(lam), _ptr32(trip), len(u),
                                        int(n_vertices), ctypes.byref(o), ctypes.byref(h)))
    return Layout(h)


def eat_layout_build(u, v, t, lam, n_vertices, layout=EAT_LAYOUT_HYBRID, cluster_seconds=0,
                     n_threads=0) -> Layout:
    u, v, t, lam = (_i32(x) for x in (u, v, t, lam))
    h = _vp()
    o = _build_opts(layout, cluster_seconds, n_threads)
    _check(lib().eat_layout_build(_ptr32(u), _ptr32(v), _ptr32(t), _ptr32(lam), len(u),
                                  int(n_vertices), ctypes.byref(o), ctypes.byref(h)))
    return Layout(h)


# ---------------------------------------------------------------------------
# device graphs and queries
# ---------------------------------------------------------------------------
class Graph:
    """A device-resident timetable (eat_graph_build)."""

    def __init__(self, handle):
        self._h = handle
        gi = GraphInfo()
        _check(lib().eat_graph_info(self._h, ctypes.byref(gi)))
        self.info = gi
        self.n_vertices = gi.n_vertices

    @property
    def handle(self):
        return self._h

    def query(self, s: int, ts: int, out=None, stream=None, options=None, stats: bool = False):
        """Earliest arrival times from (s, ts) into `out` (a new CUDA int32 tensor
        if None).  Returns out, or (out, stats dict) with stats=True."""
        import torch
        if out is None:
            out = torch.empty(self.n_vertices, dtype=torch.int32, device="cuda")
        st = eat_query(self, s, ts, out, stream=stream, options=options, stats=stats)
        return (out, st) if stats else out

    def query_goal(self, s: int, ts: int, d: int, out=None, stream=None, options=None, stats: bool = False):
        """Goal-directed query (eat_query_goal): out[d] is the earliest arrival at
        d; other entries are upper bounds.  Returns out (or (out, stats))."""
        import torch
        if out is None:
            out = torch.empty(self.n_vertices, dtype=torch.int32, device="cuda")
        st = eat_query_goal(self, s, ts, d, out, stream=stream, options=options, stats=stats)
        return (out, st) if stats else out

    def parents(self, s: int, arr, out=None, stream=None):
        """Parent connection of every stop for the answer arr of a query from s
        (eat_parents): a (V, 3) CUDA int32 tensor of (u, t, lam), -1 where none."""
        import torch
        if out is None:
            out = torch.empty((self.n_vertices, 3), dtype=torch.int32, device="cuda")
        _check(lib().eat_parents(self.handle, int(s), _dev_ptr(arr, self.n_vertices, "arr"),
                                 _dev_ptr(out, 3 * self.n_vertices, "out"), _stream_handle(stream)))
        return out

    def profile(self, s: int, t_lo: int, t_hi: int, stream=None, options=None):
        """Profile of s over departures in [t_lo, t_hi] (eat_profile): (dep, arr)
        with dep a numpy int32 array of k departure times and arr a (k, V) CUDA
        int32 tensor, row i holding per stop the arrival of the Pareto-optimal
        journey leaving at dep[i] (EAT_INF where none)."""
        import torch
        n = np.zeros(1, dtype=np.int32)
        ro = _run_opts(options)
        rop = ctypes.byref(ro) if ro is not None else None
        _check(lib().eat_profile(self.handle, int(s), int(t_lo), int(t_hi), 0, None, _ptr32(n), None,
                                 _stream_handle(stream), rop))
        k = int(n[0])
        dep = np.zeros(max(k, 1), dtype=np.int32)
        arr = torch.empty((max(k, 1), self.n_vertices), dtype=torch.int32, device="cuda")
        if k:
            _check(lib().eat_profile(self.handle, int(s), int(t_lo), int(t_hi), k, _ptr32(dep), _ptr32(n),
                                     ctypes.c_void_p(arr.data_ptr()), _stream_handle(stream), rop))
        return dep[:k], arr[:k]

    def failures(self) -> int:
        """Plain queries (run without stats) on this graph that hit their round
        limit since it was built (eat_graph_failures)."""
        n = ctypes.c_int32()
        _check(lib().eat_graph_failures(self._h, ctypes.byref(n)))
        return int(n.value)

    def free(self):
        if getattr(self, "_h", None):
            lib().eat_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def eat_graph_build(u, v, t, lam, n_vertices, layout=EAT_LAYOUT_HYBRID, cluster_seconds=0,
                    n_threads=0, header_grid=0, stream=None) -> Graph:
    """header_grid: 0 = also build the device header grid (hybrid), -1 = compact headers only.
    The upload runs on `stream` (default: torch's current stream)."""
    u, v, t, lam = (_i32(x) for x in (u, v, t, lam))
    h = _vp()
    o = _build_opts(layout, cluster_seconds, n_threads, header_grid)
    _check(lib().eat_graph_build(_ptr32(u), _ptr32(v), _ptr32(t), _ptr32(lam), len(u),
                                 int(n_vertices), ctypes.byref(o), _stream_handle(stream), ctypes.byref(h)))
    return Graph(h)


def eat_graph_build_trips(u, v, t, lam, trip, n_vertices, subtrip_len=0, layout=EAT_LAYOUT_HYBRID,
                          cluster_seconds=0, n_threads=0, header_grid=0, stream=None) -> Graph:
    """Device graph with sub-trip shortcuts (see eat_layout_build_trips)."""
    u, v, t, lam, trip = (_i32(x) for x in (u, v, t, lam, trip))
    h = _vp()
    o = _build_opts(layout, cluster_seconds, n_threads, header_grid, subtrip_len)
    _check(lib().eat_graph_build_trips(_ptr32(u), _ptr32(v), _ptr32(t), _ptr32(lam), _ptr32(trip), len(u),
                                       int(n_vertices), ctypes.byref(o), _stream_handle(stream), ctypes.byref(h)))
    return Graph(h)


def eat_graph_upload(layout: Layout, header_grid: int = 0, stream=None) -> Graph:
    h = _vp()
    o = BuildOptions()
    o.header_grid = int(header_grid)
    _check(lib().eat_graph_upload(layout._h, ctypes.byref(o), _stream_handle(stream), ctypes.byref(h)))
    return Graph(h)


def graph_from_timetable(tt, layout=EAT_LAYOUT_HYBRID, cluster_seconds=0, header_grid=0,
                         subtrip_len=None) -> Graph:
    """subtrip_len None: the connections as given; else sub-trip shortcuts from
    the timetable's trips (see eat_layout_build_trips)."""
    if subtrip_len is not None:
        if tt.trip is None:
            raise ValueError("the timetable has no vehicle trips")
        return eat_graph_build_trips(tt.u, tt.v, tt.t, tt.lam, tt.trip, tt.n_vertices, subtrip_len=subtrip_len,
                                     layout=layout, cluster_seconds=cluster_seconds, header_grid=header_grid)
    return eat_graph_build(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, layout=layout,
                           cluster_seconds=cluster_seconds, header_grid=header_grid)


def eat_query(g: Graph, s: int, ts: int, arr, stream=None, options=None, stats: bool = False):
    ptr = _dev_ptr(arr, g.n_vertices, "arr")
    ro = _run_opts(options)
    st = QueryStats() if stats else None
    _check(lib().eat_query(g.handle, int(s), int(ts), ptr, _stream_handle(stream),
                           ctypes.byref(ro) if ro is not None else None,
                           ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def eat_query_goal(g: Graph, s: int, ts: int, d: int, arr, stream=None, options=None, stats: bool = False):
    ptr = _dev_ptr(arr, g.n_vertices, "arr")
    ro = _run_opts(options)
    st = QueryStats() if stats else None
    _check(lib().eat_query_goal(g.handle, int(s), int(ts), int(d), ptr, _stream_handle(stream),
                                ctypes.byref(ro) if ro is not None else None,
                                ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def journey(par, s: int, d: int):
    """The journey from s to d read from parents par ((V, 3) array of (u, t,
    lam), as returned by Graph.parents): a list of connections (u, v, t, lam)
    in travel order; [] for d == s; None if d has no parent chain to s."""
    par = np.asarray(par.cpu() if hasattr(par, "cpu") else par).reshape(-1, 3)
    legs, v = [], int(d)
    while v != s:
        u, t, lam = (int(x) for x in par[v])
        if u < 0 or len(legs) > len(par):
            return None
        legs.append((u, v, t, lam))
        v = u
    return legs[::-1]


class Batch:
    """A prepared batch (eat_batch_create, or eat_batch_create_goal when q_dst
    gives destinations, -1 = every stop); run() enqueues all its queries in
    one launch."""

    def __init__(self, graphs: Sequence[Graph], q_graph, q_src, q_ts, outs, options=None, q_dst=None):
        self.graphs = list(graphs)
        q_graph, q_src, q_ts = _i32(q_graph), _i32(q_src), _i32(q_ts)
        n = len(q_src)
        if not (len(q_graph) == len(q_ts) == len(outs) == n):
            raise ValueError("q_graph, q_src, q_ts and outs must have equal length")
        gh = (_vp * len(self.graphs))(*[g.handle for g in self.graphs])
        ptrs = []
        for i in range(n):
            gi = int(q_graph[i])
            nv = self.graphs[gi].n_vertices if 0 <= gi < len(self.graphs) else 0
            ptrs.append(_dev_ptr(outs[i], nv, f"outs[{i}]"))
        ah = (_vp * max(n, 1))(*ptrs)
        ro = _run_opts(options)
        h = _vp()
        rop = ctypes.byref(ro) if ro is not None else None
        if q_dst is not None:
            q_dst = _i32(q_dst)
            if len(q_dst) != n:
                raise ValueError("q_dst must have one entry per query")
            _check(lib().eat_batch_create_goal(gh, len(self.graphs), _ptr32(q_graph), _ptr32(q_src), _ptr32(q_ts),
                                               _ptr32(q_dst), n, ah, rop, ctypes.byref(h)))
        else:
            _check(lib().eat_batch_create(gh, len(self.graphs), _ptr32(q_graph), _ptr32(q_src),
                                          _ptr32(q_ts), n, ah, rop, ctypes.byref(h)))
        self._h = h
        self.n = n
        self._outs = outs  # keep the slabs alive as long as the batch

    def run(self, stream=None):
        _check(lib().eat_batch_run(self._h, _stream_handle(stream)))

    def options(self) -> dict:
        """The run options the batch was created with (eat_batch_options): the
        caller's, else the tuned record, else the defaults."""
        o = RunOptions()
        _check(lib().eat_batch_options(self._h, ctypes.byref(o)))
        return options_dict(o)

    def wait(self, stats: bool = False):
        if stats:
            arr = (QueryStats * max(self.n, 1))()
            _check(lib().eat_batch_wait(self._h, arr))
            return [arr[i].as_dict() for i in range(self.n)]
        _check(lib().eat_batch_wait(self._h, None))
        return None

    def free(self):
        if getattr(self, "_h", None):
            lib().eat_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def eat_query_batch(graphs: Sequence[Graph], q_graph, q_src, q_ts, outs, stream=None,
                    options=None, stats: bool = False):
    q_graph, q_src, q_ts = _i32(q_graph), _i32(q_src), _i32(q_ts)
    n = len(q_src)
    gh = (_vp * len(graphs))(*[g.handle for g in graphs])
    ptrs = [_dev_ptr(outs[i], graphs[int(q_graph[i])].n_vertices, f"outs[{i}]") for i in range(n)]
    ah = (_vp * max(n, 1))(*ptrs)
    ro = _run_opts(options)
    st = (QueryStats * max(n, 1))() if stats else None
    _check(lib().eat_query_batch(gh, len(graphs), _ptr32(q_graph), _ptr32(q_src), _ptr32(q_ts), n, ah,
                                 _stream_handle(stream), ctypes.byref(ro) if ro is not None else None,
                                 st))
    return [st[i].as_dict() for i in range(n)] if stats else None


def eat_query_batch_static(graphs: Sequence[Graph], q_graph, q_src, q_ts, outs, stream=None,
                           options=None, stats: bool = False):
    """eat_query_batch through the entry point that allocates nothing
    (eat_query_batch_static): at most 8192 queries over 64 graphs."""
    q_graph, q_src, q_ts = _i32(q_graph), _i32(q_src), _i32(q_ts)
    n = len(q_src)
    gh = (_vp * len(graphs))(*[g.handle for g in graphs])
    ptrs = []
    for i in range(n):
        gi = int(q_graph[i])
        nv = graphs[gi].n_vertices if 0 <= gi < len(graphs) else 0
        ptrs.append(_dev_ptr(outs[i], nv, f"outs[{i}]"))
    ah = (_vp * max(n, 1))(*ptrs)
    ro = _run_opts(options)
    st = (QueryStats * max(n, 1))() if stats else None
    _check(lib().eat_query_batch_static(gh, len(graphs), _ptr32(q_graph), _ptr32(q_src), _ptr32(q_ts), n, ah,
                                        _stream_handle(stream), ctypes.byref(ro) if ro is not None else None, st))
    return [st[i].as_dict() for i in range(n)] if stats else None


def eat_batch_tune(graphs: Sequence[Graph], q_graph, q_src, q_ts, outs, stream=None, reps: int = 0,
                   n_streams: int = 0):
    """Runs the library's autotuner (eat_batch_tune) on this batch; returns
    (best options dict, [(options dict, ms per run), ...]).  Batches created
    afterwards with options=None for the same graphs and batch size use the
    tuned options."""
    q_graph, q_src, q_ts = _i32(q_graph), _i32(q_src), _i32(q_ts)
    n = len(q_src)
    gh = (_vp * len(graphs))(*[g.handle for g in graphs])
    ptrs = [_dev_ptr(outs[i], graphs[int(q_graph[i])].n_vertices, f"outs[{i}]") for i in range(n)]
    ah = (_vp * max(n, 1))(*ptrs)
    to = TuneOptions()
    to.reps = int(reps)
    to.n_streams = int(n_streams)
    best = RunOptions()
    res = (TuneResult * 64)()
    nres = ctypes.c_int32()
    _check(lib().eat_batch_tune(gh, len(graphs), _ptr32(q_graph), _ptr32(q_src), _ptr32(q_ts), n, ah,
                                _stream_handle(stream), ctypes.byref(to), ctypes.byref(best), res, 64,
                                ctypes.byref(nres)))
    return options_dict(best), [(options_dict(res[i].options), float(res[i].ms)) for i in range(nres.value)]


def eat_next_departure(g: Graph, type_ids, x, out, headers=EAT_HEADERS_AUTO, stream=None):
    n = int(type_ids.numel())
    _check(lib().eat_next_departure(g.handle, int(headers), _dev_ptr(type_ids, n, "type_ids"),
                                    _dev_ptr(x, n, "x"), _dev_ptr(out, n, "out"), n,
                                    _stream_handle(stream)))


class Session:
    """A serving session (eat_session_*): continuous batching over resident graphs."""

    def __init__(self, graphs: Sequence[Graph], pool_bytes: int = 0, n_streams: int = 0,
                 max_step_queries: int = 0, options=None):
        self.graphs = list(graphs)
        o = SessionOptions()
        o.pool_bytes = int(pool_bytes)
        o.n_streams = int(n_streams)
        o.max_step_queries = int(max_step_queries)
        ro = _run_opts(options)
        if ro is not None:
            o.run = ro
        gh = (_vp * len(self.graphs))(*[g.handle for g in self.graphs])
        h = _vp()
        _check(lib().eat_session_create(gh, len(self.graphs), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._done = (ctypes.c_int32 * 65536)()

    def admit(self, graph: int, s: int, ts: int):
        """Slot id, or None when the pool has no room (EAT_ERR_BUSY)."""
        slot = ctypes.c_int32()
        st = lib().eat_session_admit(self._h, int(graph), int(s), int(ts), ctypes.byref(slot))
        if st == EAT_ERR_BUSY:
            return None
        _check(st)
        return int(slot.value)

    def step(self):
        """Launches the admitted queries; their count, or None when every step
        of the session is still in flight (EAT_ERR_BUSY: nothing launched)."""
        n = ctypes.c_int32()
        st = lib().eat_session_step(self._h, ctypes.byref(n))
        if st == EAT_ERR_BUSY:
            return None
        _check(st)
        return int(n.value)

    def poll(self):
        n = ctypes.c_int32()
        _check(lib().eat_session_poll(self._h, self._done, len(self._done), ctypes.byref(n)))
        return [int(self._done[i]) for i in range(n.value)]

    def sync(self):
        _check(lib().eat_session_sync(self._h))

    def result_ptr(self, slot: int):
        p = _i32p()
        n = ctypes.c_int32()
        _check(lib().eat_session_result(self._h, int(slot), ctypes.byref(p), ctypes.byref(n)))
        return ctypes.cast(p, ctypes.c_void_p).value, int(n.value)

    def result(self, slot: int, out=None, stream=None):
        """A finished slot's arrival array, copied into `out` (a new CUDA int32
        tensor if None) on `stream`."""
        import torch
        _, n = self.result_ptr(slot)
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().eat_session_copy(self._h, int(slot), _dev_ptr(out, n, "out"), _stream_handle(stream)))
        return out

    def stats(self, slot: int) -> dict:
        st = QueryStats()
        _check(lib().eat_session_query_stats(self._h, int(slot), ctypes.byref(st)))
        return st.as_dict()

    def release(self, slot: int):
        _check(lib().eat_session_release(self._h, int(slot)))

    def serve(self, graph, src, ts, arrival_s, min_batch: int = 64, max_delay_s: float = 50e-6,
              copy_dst=None, copy_stream=None):
        """eat_session_serve: the whole open-loop request stream in native code.
        copy_dst: None, or a list with a CUDA int32 tensor (or None) per
        request.  Returns (latency in seconds per request, report dict)."""
        graph, src, ts = (_i32(x) for x in (graph, src, ts))
        arrival = np.ascontiguousarray(arrival_s, dtype=np.float64)
        n = len(graph)
        if not (len(src) == len(ts) == len(arrival) == n):
            raise ValueError("request arrays differ in length")
        lat = np.zeros(n, np.float64)
        f64 = ctypes.POINTER(ctypes.c_double)
        dst = None
        if copy_dst is not None:
            if len(copy_dst) != n:
                raise ValueError("copy_dst needs one entry per request")
            dst = (_vp * n)(*[None if d is None else
                              _dev_ptr(d, self.graphs[int(graph[i])].n_vertices, "copy_dst")
                              for i, d in enumerate(copy_dst)])
        rep = ServeReport()
        _check(lib().eat_session_serve(self._h, n, _ptr32(graph), _ptr32(src), _ptr32(ts),
                                       arrival.ctypes.data_as(f64), int(min_batch), float(max_delay_s),
                                       dst, _stream_handle(copy_stream) if dst is not None else None,
                                       lat.ctypes.data_as(f64), ctypes.byref(rep)))
        return lat, rep.as_dict()

    def free(self):
        if getattr(self, "_h", None):
            lib().eat_session_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def eat_version() -> int:
    return int(lib().eat_version())


# ---------------------------------------------------------------------------
# The paper's algorithm ladder and its host utilities
# ---------------------------------------------------------------------------
def ap_cover(d) -> np.ndarray:
    """Greedy arithmetic-progression cover (eat_ap_cover) of strictly increasing
    values: a (k, 3) int32 array of {first, last, difference}."""
    d = _i32(d)
    n = ctypes.c_int64()
    _check(lib().eat_ap_cover(_ptr32(d), len(d), None, 0, ctypes.byref(n)))
    out = np.zeros((max(int(n.value), 1), 3), dtype=np.int32)
    _check(lib().eat_ap_cover(_ptr32(d), len(d), _ptr32(out), int(n.value), ctypes.byref(n)))
    return out[:int(n.value)]


def esdg_levels(u, v, t, lam, n_vertices):
    """ESDG level of every connection as given (eat_esdg_levels): (level array,
    number of levels, number of dependency edges)."""
    u, v, t, lam = (_i32(x) for x in (u, v, t, lam))
    level = np.zeros(max(len(u), 1), dtype=np.int32)
    nl = ctypes.c_int32()
    ne = ctypes.c_int64()
    _check(lib().eat_esdg_levels(_ptr32(u), _ptr32(v), _ptr32(t), _ptr32(lam), len(u), int(n_vertices),
                                 _ptr32(level), ctypes.byref(nl), ctypes.byref(ne)))
    return level[:len(u)], int(nl.value), int(ne.value)


class VariantGraph:
    """The arrays of every variant of the paper's ladder on the device
    (eat_variant_graph_build)."""

    def __init__(self, u, v, t, lam, n_vertices, cluster_seconds=0, esdg=False, n_threads=0):
        u, v, t, lam = (_i32(x) for x in (u, v, t, lam))
        o = VariantBuildOptions()
        o.cluster_seconds = int(cluster_seconds)
        o.esdg = 1 if esdg else 0
        o.n_threads = int(n_threads)
        h = _vp()
        _check(lib().eat_variant_graph_build(_ptr32(u), _ptr32(v), _ptr32(t), _ptr32(lam), len(u), int(n_vertices),
                                             ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        gi = VariantInfo()
        _check(lib().eat_variant_graph_info(self._h, ctypes.byref(gi)))
        self.info = gi.as_dict()
        self.n_vertices = gi.n_vertices

    def query(self, s: int, ts: int, variant: int, out=None, warp_size=0, check_every=0, count=False,
              stream=None, max_iterations=0):
        """(out, stats): the EAT answer by one variant, with its iteration count."""
        import torch
        if out is None:
            out = torch.empty(self.n_vertices, dtype=torch.int32, device="cuda")
        o = VariantOptions()
        o.variant, o.warp_size, o.check_every = int(variant), int(warp_size), int(check_every)
        o.count, o.max_iterations = 1 if count else 0, int(max_iterations)
        st = VariantStats()
        _check(lib().eat_variant_query(self._h, int(s), int(ts), _dev_ptr(out, self.n_vertices, "out"),
                                       _stream_handle(stream), ctypes.byref(o), ctypes.byref(st)))
        return out, st.as_dict()

    def free(self):
        if getattr(self, "_h", None):
            lib().eat_variant_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
