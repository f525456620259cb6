"""CPU oracle for the earliest-arrival-time (EAT) problem (arXiv 1912.00966).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library: it reads the raw connection list (u, v, t, lam), never the
library's layout, and the library never imports it.

Functions (plain C in this directory, loaded through ctypes):
  Csa              -- Connection-Scan Algorithm (Algorithm 1, Section I-A); the
                      reference answer for every query.
  brute_paths      -- enumeration of every time-respecting path (Section I).
  brute_states     -- closure over reachable (stop, time) states (Section I).
  te_dijkstra      -- Dijkstra on the time-expanded model (Section I).
  td_dijkstra      -- Dijkstra on the time-dependent model (Section I).
  certify          -- source / closure / witness check of an arrival array.
  parents          -- the parent connection of every reached stop (journeys).
  Csa.profile      -- Pareto-optimal (departure, arrival) pairs of a source over
                      an interval of departure times, one scan per departure.
  brute_profile    -- the same profile by enumerating every journey.
  next_departure   -- min{t in a connection type : t >= x} (Section II-B).
"""
import ctypes
import os

import numpy as np

INF = np.iinfo(np.int32).max
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    conn = [ctypes.c_int64, _i32p, _i32p, _i32p, _i32p, ctypes.c_int32]
    lib.oracle_validate.argtypes = conn
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_csa_new.argtypes = conn
    lib.oracle_csa_new.restype = ctypes.c_void_p
    lib.oracle_csa_free.argtypes = [ctypes.c_void_p]
    lib.oracle_csa_free.restype = None
    lib.oracle_csa_query.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _i32p]
    lib.oracle_csa_query.restype = ctypes.c_int
    lib.oracle_csa_query_many.argtypes = [ctypes.c_void_p, ctypes.c_int32, _i32p, _i32p, _i32p]
    lib.oracle_csa_query_many.restype = ctypes.c_int
    lib.oracle_brute_paths.argtypes = conn + [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _i32p]
    lib.oracle_brute_paths.restype = ctypes.c_int
    for name in ("oracle_brute_states", "oracle_te_dijkstra", "oracle_td_dijkstra"):
        f = getattr(lib, name)
        f.argtypes = conn + [ctypes.c_int32, ctypes.c_int32, _i32p]
        f.restype = ctypes.c_int
    lib.oracle_certify.argtypes = conn + [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p]
    lib.oracle_certify.restype = ctypes.c_int
    lib.oracle_parents.argtypes = conn + [ctypes.c_int32, _i32p, _i32p, _i32p, _i32p]
    lib.oracle_parents.restype = ctypes.c_int
    lib.oracle_profile.argtypes = [ctypes.c_int64, _i32p, _i32p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p]
    lib.oracle_profile.restype = ctypes.c_int
    lib.oracle_brute_profile.argtypes = conn + [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                                ctypes.c_int32, _i32p, _i32p, _i32p]
    lib.oracle_brute_profile.restype = ctypes.c_int
    lib.oracle_next_departure.argtypes = [ctypes.c_int64, _i32p, ctypes.c_int32]
    lib.oracle_next_departure.restype = ctypes.c_int32
    _lib = lib
    return lib


def _arr(a, dtype=np.int32):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _p32(a):
    return a.ctypes.data_as(_i32p)


def _conn(u, v, t, lam):
    u, v, t, lam = (_arr(x) for x in (u, v, t, lam))
    n = len(u)
    if not (len(v) == len(t) == len(lam) == n):
        raise ValueError("u, v, t, lam must have equal length")
    return u, v, t, lam


def validate(u, v, t, lam, nv) -> bool:
    u, v, t, lam = _conn(u, v, t, lam)
    return _load().oracle_validate(len(u), _p32(u), _p32(v), _p32(t), _p32(lam), nv) == 0


class Csa:
    """Connection-scan oracle over one connection list (Algorithm 1)."""

    def __init__(self, u, v, t, lam, nv):
        lib = _load()
        self._keep = _conn(u, v, t, lam)
        u, v, t, lam = self._keep
        self.nv = int(nv)
        self._h = lib.oracle_csa_new(len(u), _p32(u), _p32(v), _p32(t), _p32(lam), self.nv)
        if not self._h:
            raise OracleError("invalid connection list (need t>=0, lam>=1, t+lam<INF, 0<=u,v<nv)")
        self._u, self._t = u, t  # the departures of a source (profiles)
        self._keep = None

    def query(self, s, ts):
        out = np.empty(self.nv, dtype=np.int32)
        rc = _load().oracle_csa_query(self._h, int(s), int(ts), _p32(out))
        if rc != 0:
            raise OracleError(f"csa query failed ({rc})")
        return out

    def query_many(self, s, ts):
        s = _arr(s)
        ts = _arr(ts)
        out = np.empty((len(s), self.nv), dtype=np.int32)
        rc = _load().oracle_csa_query_many(self._h, len(s), _p32(s), _p32(ts), _p32(out))
        if rc != 0:
            raise OracleError(f"csa query failed ({rc})")
        return out

    def profile(self, s, t_lo, t_hi):
        """(dep, arr): dep = the k distinct departure times of connections
        leaving s inside [t_lo, t_hi], increasing; arr (k x nv): row i holds,
        per stop, the arrival of the Pareto-optimal journey leaving s at dep[i]
        (among all journeys leaving s at or after t_lo), INF where there is none
        (always at s)."""
        lib = _load()
        n_dep = np.zeros(1, dtype=np.int32)
        rc = lib.oracle_profile(len(self._u), _p32(self._u), _p32(self._t), self._h, self.nv, int(s), int(t_lo),
                                int(t_hi), 0, None, _p32(n_dep), None)
        if rc not in (0, 3):
            raise OracleError(f"profile failed ({rc})")
        k = int(n_dep[0])
        dep = np.empty(max(k, 1), dtype=np.int32)
        out = np.empty((max(k, 1), self.nv), dtype=np.int32)
        rc = lib.oracle_profile(len(self._u), _p32(self._u), _p32(self._t), self._h, self.nv, int(s), int(t_lo),
                                int(t_hi), k, _p32(dep), _p32(n_dep), _p32(out))
        if rc != 0:
            raise OracleError(f"profile failed ({rc})")
        return dep[:k], out[:k]

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_csa_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _single(fname, u, v, t, lam, nv, s, ts, *extra):
    u, v, t, lam = _conn(u, v, t, lam)
    out = np.empty(nv, dtype=np.int32)
    f = getattr(_load(), fname)
    rc = f(len(u), _p32(u), _p32(v), _p32(t), _p32(lam), int(nv), int(s), int(ts), *extra, _p32(out))
    if rc != 0:
        raise OracleError(f"{fname} failed ({rc})")
    return out


def brute_paths(u, v, t, lam, nv, s, ts, max_paths=2_000_000):
    return _single("oracle_brute_paths", u, v, t, lam, nv, s, ts, ctypes.c_int64(max_paths))


def brute_states(u, v, t, lam, nv, s, ts):
    return _single("oracle_brute_states", u, v, t, lam, nv, s, ts)


def te_dijkstra(u, v, t, lam, nv, s, ts):
    return _single("oracle_te_dijkstra", u, v, t, lam, nv, s, ts)


def td_dijkstra(u, v, t, lam, nv, s, ts):
    return _single("oracle_td_dijkstra", u, v, t, lam, nv, s, ts)


def certify(u, v, t, lam, nv, s, ts, arr):
    """0 if arr is the EAT answer, else 1 (source), 2 (closure) or 3 (witness)."""
    u, v, t, lam = _conn(u, v, t, lam)
    arr = _arr(arr)
    bad = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_certify(len(u), _p32(u), _p32(v), _p32(t), _p32(lam), int(nv),
                                int(s), int(ts), _p32(arr), _p32(bad))
    if rc < 0:
        raise OracleError("certify: invalid input")
    return rc


def parents(u, v, t, lam, nv, s, arr):
    """(par_u, par_t, par_lam): for each reached stop x != s, the connection
    into x realising arr[x] with the smallest tail, then the smallest duration;
    -1 elsewhere."""
    u, v, t, lam = _conn(u, v, t, lam)
    arr = _arr(arr)
    pu, pt, pl = (np.empty(nv, dtype=np.int32) for _ in range(3))
    rc = _load().oracle_parents(len(u), _p32(u), _p32(v), _p32(t), _p32(lam), int(nv), int(s), _p32(arr),
                                _p32(pu), _p32(pt), _p32(pl))
    if rc != 0:
        raise OracleError(f"parents failed ({rc}): arr is not an EAT answer")
    return pu, pt, pl


def brute_profile(u, v, t, lam, nv, s, t_lo, t_hi, max_paths=2_000_000):
    """Csa.profile computed by enumerating every journey (tiny inputs)."""
    u, v, t, lam = _conn(u, v, t, lam)
    lib = _load()
    n_dep = np.zeros(1, dtype=np.int32)
    args = (len(u), _p32(u), _p32(v), _p32(t), _p32(lam), int(nv), int(s), int(t_lo), int(t_hi),
            ctypes.c_int64(max_paths))
    rc = lib.oracle_brute_profile(*args, 0, None, _p32(n_dep), None)
    if rc not in (0, 3):
        raise OracleError(f"brute_profile failed ({rc})")
    k = int(n_dep[0])
    dep = np.empty(max(k, 1), dtype=np.int32)
    out = np.empty((max(k, 1), nv), dtype=np.int32)
    rc = lib.oracle_brute_profile(*args, k, _p32(dep), _p32(n_dep), _p32(out))
    if rc != 0:
        raise OracleError(f"brute_profile failed ({rc})")
    return dep[:k], out[:k]


def next_departure(deps, x):
    d = _arr(deps)
    return int(_load().oracle_next_departure(len(d), _p32(d), int(x)))
