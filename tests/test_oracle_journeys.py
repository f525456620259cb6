"""Pins for the oracle's query variants (Section I names them beside the
single-source problem): parent connections (journeys) and profiles.

The parents are checked as journeys against the state-closure brute force
(every reached stop's parent chain is a real time-respecting path from s that
arrives at the brute-force arrival), the profile of the scan oracle against
the enumeration of every journey, and both against hand-made cases.  Planted
mistakes in a copy of journeys.c must be caught."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import synth

INF = oracle.INF
ORACLE_DIR = os.path.dirname(oracle.__file__)


def _tt(rows, nv):
    a = np.array(rows, dtype=np.int32).reshape(-1, 4)
    return synth.Timetable("hand", nv, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), a[:, 3].copy(), -1, -1, -1)


def _check_journeys(tt, s, arr, pu, pt, pl):
    """Every reached stop's parent chain is a journey from s arriving at arr."""
    conns = set(zip(tt.u.tolist(), tt.v.tolist(), tt.t.tolist(), tt.lam.tolist()))
    for x in range(tt.n_vertices):
        if x == s or arr[x] == INF:
            assert pu[x] == pt[x] == pl[x] == -1
            continue
        assert (int(pu[x]), x, int(pt[x]), int(pl[x])) in conns
        assert pt[x] + pl[x] == arr[x]
        assert arr[pu[x]] <= pt[x]
        # walk back to s: arrivals strictly decrease, so the walk ends
        y, steps = x, 0
        while y != s:
            assert arr[pu[y]] < arr[y]
            y = int(pu[y])
            steps += 1
            assert steps <= tt.n_vertices


def test_parents_hand_case_smallest_tail_then_duration():
    # stop 3 is reached at 30 by three connections: from 2 (t=20, lam=10),
    # from 1 (t=25, lam=5) and from 1 (t=10, lam=20); the rule takes tail 1,
    # then the smaller duration 5.  Stop 4 is never reached.
    tt = _tt([[0, 1, 0, 5], [0, 2, 0, 10], [2, 3, 20, 10], [1, 3, 25, 5], [1, 3, 10, 20], [3, 0, 40, 1],
              [4, 0, 0, 1]], 5)
    arr = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, 5).query(0, 0)
    assert arr.tolist() == [0, 5, 10, 30, INF]
    pu, pt, pl = oracle.parents(tt.u, tt.v, tt.t, tt.lam, 5, 0, arr)
    assert pu.tolist() == [-1, 0, 0, 1, -1]
    assert pt.tolist() == [-1, 0, 0, 25, -1]
    assert pl.tolist() == [-1, 5, 10, 5, -1]
    _check_journeys(tt, 0, arr, pu, pt, pl)


def test_parents_are_journeys_on_random_timetables():
    rng = np.random.default_rng(91)
    for _ in range(400):
        tt = synth.random_tiny(rng)
        s = int(rng.integers(0, tt.n_vertices))
        ts = int(rng.integers(0, 32))
        arr = oracle.brute_states(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts)
        pu, pt, pl = oracle.parents(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, arr)
        _check_journeys(tt, s, arr, pu, pt, pl)


def test_parents_refuse_an_arrival_array_that_is_not_an_answer():
    tt = _tt([[0, 1, 0, 5], [1, 2, 5, 5]], 3)
    arr = np.array([0, 5, 10], dtype=np.int32)
    oracle.parents(tt.u, tt.v, tt.t, tt.lam, 3, 0, arr)
    arr[2] = 11  # no connection arrives at 11
    with pytest.raises(oracle.OracleError):
        oracle.parents(tt.u, tt.v, tt.t, tt.lam, 3, 0, arr)


def test_profile_hand_case():
    # s = 0.  Departures of s: 10 (to 1, arrive 20), 15 (to 2, arrive 18),
    # 30 (to 1, arrive 35).  1 -> 3 at 25 (arrive 40) and 2 -> 3 at 19
    # (arrive 50).  Profile over [0, 20]: stop 1: (10, 20) only -- leaving at
    # 30 is outside the interval but dominates nothing earlier; stop 2:
    # (15, 18); stop 3: leaving at 10 arrives 40, leaving at 15 arrives 50
    # (dominated by nothing later: kept), so both pairs are Pareto-optimal.
    tt = _tt([[0, 1, 10, 10], [0, 2, 15, 3], [0, 1, 30, 5], [1, 3, 25, 15], [2, 3, 19, 31]], 4)
    dep, arr = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, 4).profile(0, 0, 20)
    assert dep.tolist() == [10, 15]
    assert arr.tolist() == [[INF, 20, INF, 40], [INF, INF, 18, 50]]
    # widen to [0, 30]: leaving at 30 reaches 1 at 35 (kept); nothing changes before
    dep, arr = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, 4).profile(0, 0, 30)
    assert dep.tolist() == [10, 15, 30]
    assert arr[2].tolist() == [INF, 35, INF, INF]
    # a later departure that dominates: 0 -> 3 directly at 16, arriving 39,
    # beats leaving at 10 (arrive 40) and at 15 (arrive 50) for stop 3
    tt2 = _tt([[0, 1, 10, 10], [0, 2, 15, 3], [0, 1, 30, 5], [1, 3, 25, 15], [2, 3, 19, 31], [0, 3, 16, 23]], 4)
    dep, arr = oracle.Csa(tt2.u, tt2.v, tt2.t, tt2.lam, 4).profile(0, 0, 20)
    assert dep.tolist() == [10, 15, 16]
    assert arr[:, 3].tolist() == [INF, INF, 39]
    # the interval ends before the dominating departure: (10, 40) and (15, 50)
    # are still dominated by it (optimality is among all journeys after t_lo)
    dep, arr = oracle.Csa(tt2.u, tt2.v, tt2.t, tt2.lam, 4).profile(0, 0, 15)
    assert dep.tolist() == [10, 15]
    assert arr[:, 3].tolist() == [INF, INF]


def test_profile_scan_equals_journey_enumeration():
    rng = np.random.default_rng(92)
    for k in range(500):
        tt = synth.random_tiny(rng)
        s = int(rng.integers(0, tt.n_vertices))
        lo = int(rng.integers(0, 24))
        hi = lo + int(rng.integers(0, 20))
        dep, arr = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices).profile(s, lo, hi)
        dep2, arr2 = oracle.brute_profile(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, lo, hi)
        assert np.array_equal(dep, dep2), k
        assert np.array_equal(arr, arr2), k
        # every kept pair is a real journey: its arrival is EAT(s, dep) there,
        # and the kept arrivals of a stop increase with the departure
        for i, d in enumerate(dep):
            e = oracle.brute_states(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, int(d))
            kept = arr[i] != INF
            assert np.array_equal(arr[i][kept], e[kept])
        for x in range(tt.n_vertices):
            col = arr[:, x][arr[:, x] != INF]
            assert np.all(np.diff(col) > 0)


def test_profile_empty_interval_and_limits():
    tt = _tt([[0, 1, 10, 10]], 2)
    c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, 2)
    dep, arr = c.profile(0, 11, 100)  # no departure of s inside
    assert len(dep) == 0 and arr.shape == (0, 2)
    dep, arr = c.profile(1, 0, 100)  # s has no outgoing connection
    assert len(dep) == 0


MUTANTS = {
    "parents: strict boarding": ("a > t[i] ||", "a >= t[i] ||"),
    "parents: largest tail": ("u[i] < par_u[w] ||", "u[i] > par_u[w] ||"),
    "profile: keeps ties with the next row": ("!(row[x] < after[x])", "!(row[x] <= after[x])"),
    "profile: no scan after the interval": ("if (next != ORACLE_INF) rc", "if (0) rc"),
    "profile: interval end exclusive": ("t[i] >= lo && t[i] <= hi", "t[i] >= lo && t[i] < hi"),
    "profile: next departure taken at t_hi": ("t[i] > t_hi && t[i] < next", "t[i] >= t_hi && t[i] < next"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(ORACLE_DIR, "journeys.c")).read()
    assert old in src, f"mutation site for '{name}' not found"
    d = tmp_path / "m"
    d.mkdir()
    for f in ("oracle.h", "csa.c", "brute.c"):
        shutil.copy(os.path.join(ORACLE_DIR, f), d / f)
    (d / "journeys.c").write_text(src.replace(old, new, 1))
    so = d / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(d / "csa.c"), str(d / "brute.c"),
                    str(d / "journeys.c")], check=True)
    return ctypes.CDLL(str(so))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lib = _build_mutant(tmp_path, name, *MUTANTS[name])
    p = ctypes.POINTER(ctypes.c_int32)
    conn = [ctypes.c_int64, p, p, p, p, ctypes.c_int32]
    lib.oracle_parents.argtypes = conn + [ctypes.c_int32, p, p, p, p]
    lib.oracle_csa_new.argtypes = conn
    lib.oracle_csa_new.restype = ctypes.c_void_p
    lib.oracle_csa_free.argtypes = [ctypes.c_void_p]
    lib.oracle_profile.argtypes = [ctypes.c_int64, p, p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, p, p, p]
    P = lambda a: a.ctypes.data_as(p)
    rng = np.random.default_rng(93)
    for _ in range(1500):
        tt = synth.random_tiny(rng)
        nv = tt.n_vertices
        s = int(rng.integers(0, nv))
        cols = [np.ascontiguousarray(a, dtype=np.int32) for a in (tt.u, tt.v, tt.t, tt.lam)]
        if name.startswith("parents"):
            # the hand case first (it pins the choice among realising
            # connections), then the journey checks on random timetables
            if _ == 0:
                tt = _tt([[0, 1, 0, 5], [0, 2, 0, 10], [2, 3, 20, 10], [1, 3, 25, 5], [1, 3, 10, 20]], 4)
                nv, s = 4, 0
                cols = [np.ascontiguousarray(a, dtype=np.int32) for a in (tt.u, tt.v, tt.t, tt.lam)]
            ts = 0 if _ == 0 else int(rng.integers(0, 32))
            arr = oracle.brute_states(tt.u, tt.v, tt.t, tt.lam, nv, s, ts)
            got = [np.empty(nv, dtype=np.int32) for _ in range(3)]
            rc = lib.oracle_parents(len(tt.u), *map(P, cols), nv, s, P(arr), *map(P, got))
            if rc != 0:
                return  # caught: a reached stop without a parent
            if _ == 0 and got[0].tolist() != [-1, 0, 0, 1]:
                return  # caught by the hand case
            try:
                _check_journeys(tt, s, arr, *got)
            except AssertionError:
                return  # caught
        else:
            lo = int(rng.integers(0, 24))
            hi = lo + int(rng.integers(0, 20))
            dep2, arr2 = oracle.brute_profile(tt.u, tt.v, tt.t, tt.lam, nv, s, lo, hi)
            h = lib.oracle_csa_new(len(tt.u), *map(P, cols), nv)
            cap = 64
            dep = np.zeros(cap, dtype=np.int32)
            nd = np.zeros(1, dtype=np.int32)
            arr = np.zeros((cap, nv), dtype=np.int32)
            rc = lib.oracle_profile(len(tt.u), P(cols[0]), P(cols[2]), h, nv, s, lo, hi, cap, P(dep), P(nd), P(arr))
            lib.oracle_csa_free(h)
            k = int(nd[0])
            if rc != 0 or not np.array_equal(dep[:k], dep2) or not np.array_equal(arr[:k], arr2):
                return  # caught
    pytest.fail(f"mutant '{name}' survived")
