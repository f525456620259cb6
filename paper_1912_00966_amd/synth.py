"""Seeded synthetic public-transport timetables and query sets.

The paper measures on GTFS feeds (Table I); none ship with this project, so every
input here is synthetic, seeded and regenerated on demand.  This module holds no
part of the EAT method: it only draws stops, edges, connection types and
departure times, and it is the one module that both the GPU path and the CPU
oracle are fed from.

Shape of a timetable (Sections I-A and II-B): stops are points in the unit
square; every stop is linked both ways to its k nearest neighbours (an edge
(u, v) of Section II-E); each edge carries a few connection types (same u, v and
duration lam, Section II-B); the departures of a type follow an arithmetic
progression (first departure between 05:00 and 07:00, a headway h, ending no
later than 23:00) plus a fraction of irregular departures anywhere in the day.

Connection totals: the k-NN graphs carry more types than a full-day progression
per type would fit into the stated connection totals, so the number of
progression terms per type is drawn uniformly from 1 .. 2m-1 (capped by the
23:00 end), with m chosen so that the expected total matches the stated one
(``reading="S"``).  ``reading="F"`` runs every progression to its last term
before 23:00 instead (paper-like density, roughly four times the connections).

Numpy's Generator (PCG64) is used throughout; its distribution methods are not
guaranteed stable across numpy versions, so ``Timetable.digest`` records a
content hash that tests and benchmarks print next to their results.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional, Sequence

import numpy as np

DAY = 86400
AP_START_LO = 5 * 3600
AP_START_HI = 7 * 3600
AP_END_CAP = 23 * 3600


@dataclasses.dataclass
class Timetable:
    name: str
    n_vertices: int
    u: np.ndarray
    v: np.ndarray
    t: np.ndarray
    lam: np.ndarray
    n_edges: int
    n_types_drawn: int
    seed: int
    # vehicle trip of each connection (-1: none), for timetables drawn as lines
    trip: Optional[np.ndarray] = None

    @property
    def n_conn(self) -> int:
        return int(len(self.u))

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n_vertices).tobytes())
        for a in (self.u, self.v, self.t, self.lam):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


@dataclasses.dataclass
class Queries:
    s: np.ndarray
    ts: np.ndarray
    seed: int

    def __len__(self) -> int:
        return int(len(self.s))


def _knn_edges(pts: np.ndarray, k: int) -> np.ndarray:
    """Directed edge list (u, v) of the symmetric closure of the k-NN relation."""
    from scipy.spatial import cKDTree

    n = len(pts)
    k = min(k, n - 1)
    if k <= 0:
        return np.zeros((0, 2), dtype=np.int64)
    _, idx = cKDTree(pts).query(pts, k=k + 1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = idx[:, 1:].reshape(-1).astype(np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    both = np.concatenate([src * n + dst, dst * n + src])
    uniq = np.unique(both)
    return np.stack([uniq // n, uniq % n], axis=1)


def _draw_departures(rng, n_types, headway, irregular, conn_target, reading):
    """Per type: AP start, headway, term count and irregular count."""
    start = rng.integers(AP_START_LO, AP_START_HI + 1, size=n_types)
    if isinstance(headway, tuple):
        h = rng.integers(headway[0], headway[1] + 1, size=n_types)
    else:
        h = rng.choice(np.asarray(headway, dtype=np.int64), size=n_types)
    cap = (AP_END_CAP - start) // h + 1
    if reading == "F":
        n_ap = cap
    elif reading == "S":
        m = conn_target / (n_types * (1.0 + irregular))
        hi = max(1, int(round(2 * m - 1)))
        n_ap = np.minimum(rng.integers(1, hi + 1, size=n_types), cap)
    else:
        raise ValueError("reading must be 'S' or 'F'")
    n_irr = rng.binomial(n_ap, irregular)
    return start, h, n_ap, n_irr


def _assemble(rng, name, nv, edges, types_lo, types_hi, lam_lo, lam_hi,
              headway, irregular, conn_target, reading, seed,
              lam_override: Optional[np.ndarray] = None):
    n_e = len(edges)
    per_edge = rng.integers(types_lo, types_hi + 1, size=n_e)
    ty_edge = np.repeat(np.arange(n_e), per_edge)
    n_types = len(ty_edge)
    if lam_override is not None:
        lam_lo_t = lam_override[0][ty_edge]
        lam_hi_t = lam_override[1][ty_edge]
        lam_t = rng.integers(lam_lo_t, lam_hi_t + 1)
    else:
        lam_t = rng.integers(lam_lo, lam_hi + 1, size=n_types)
    start, h, n_ap, n_irr = _draw_departures(rng, n_types, headway, irregular,
                                             conn_target, reading)
    # arithmetic-progression departures: start + j*h, j = 0 .. n_ap-1
    tid = np.repeat(np.arange(n_types, dtype=np.int64), n_ap)
    first = np.cumsum(n_ap) - n_ap
    j = np.arange(len(tid), dtype=np.int64) - np.repeat(first, n_ap)
    t_ap = start[tid] + j * h[tid]
    # irregular departures uniform in the day
    tid_irr = np.repeat(np.arange(n_types, dtype=np.int64), n_irr)
    t_irr = rng.integers(0, DAY, size=len(tid_irr))
    tid_all = np.concatenate([tid, tid_irr])
    t_all = np.concatenate([t_ap, t_irr])
    del tid, j, t_ap, tid_irr, t_irr
    # a type is a set of departures: drop repeated (type, t) pairs
    key = np.unique(tid_all * (1 << 17) + t_all)
    del tid_all, t_all
    tid_all = key >> 17
    t_all = key & ((1 << 17) - 1)
    del key
    order = rng.permutation(len(tid_all))
    tid_all = tid_all[order]
    t_all = t_all[order]
    e_all = ty_edge[tid_all]
    u = edges[e_all, 0].astype(np.int32)
    v = edges[e_all, 1].astype(np.int32)
    lam = lam_t[tid_all].astype(np.int32)
    t = t_all.astype(np.int32)
    return Timetable(name=name, n_vertices=int(nv), u=u, v=v, t=t, lam=lam,
                     n_edges=int(n_e), n_types_drawn=int(n_types), seed=int(seed))


def transit_city(n_stops: int, knn: int, types: Sequence[int], lam: Sequence[int],
                 headway, irregular: float, conn_target: int, seed: int,
                 reading: str = "S", name: str = "city") -> Timetable:
    """Stops uniform in the unit square, k-NN edges both ways."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n_stops, 2))
    edges = _knn_edges(pts, knn)
    return _assemble(rng, name, n_stops, edges, types[0], types[1], lam[0], lam[1],
                     headway, irregular, conn_target, reading, seed)


def transit_region(n_stops: int, n_towns: int, knn: int, town_sigma: float,
                   near_towns: int, pairs_per_town_pair: int,
                   types: Sequence[int], lam: Sequence[int], lam_long: Sequence[int],
                   headway, irregular: float, conn_target: int, seed: int,
                   reading: str = "S", name: str = "region") -> Timetable:
    """Gaussian towns joined by a few long inter-town edges."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.05, 0.95, size=(n_towns, 2))
    town = np.repeat(np.arange(n_towns), n_stops // n_towns)
    town = np.concatenate([town, np.arange(n_stops - len(town)) % n_towns])
    pts = np.clip(centres[town] + rng.normal(0.0, town_sigma, size=(n_stops, 2)), 0.0, 1.0)
    local = _knn_edges(pts, knn)
    # inter-town edges: each town to its nearest towns, random stop pairs, both ways
    _, near = cKDTree(centres).query(centres, k=near_towns + 1)
    members = [np.flatnonzero(town == i) for i in range(n_towns)]
    src, dst = [], []
    for a in range(n_towns):
        for b in near[a, 1:]:
            sa = rng.choice(members[a], size=pairs_per_town_pair)
            sb = rng.choice(members[int(b)], size=pairs_per_town_pair)
            src.append(np.concatenate([sa, sb]))
            dst.append(np.concatenate([sb, sa]))
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    n = n_stops
    local_key = local[:, 0] * n + local[:, 1]
    long_key = np.unique(src.astype(np.int64) * n + dst)
    long_key = long_key[~np.isin(long_key, local_key)]
    long_key = long_key[(long_key // n) != (long_key % n)]
    all_key = np.concatenate([local_key, long_key])
    is_long = np.concatenate([np.zeros(len(local_key), bool), np.ones(len(long_key), bool)])
    order = np.argsort(all_key, kind="stable")
    all_key, is_long = all_key[order], is_long[order]
    edges = np.stack([all_key // n, all_key % n], axis=1)
    # per-edge duration range: long edges use lam_long
    lo = np.where(is_long, lam_long[0], lam[0]).astype(np.int64)
    hi = np.where(is_long, lam_long[1], lam[1]).astype(np.int64)
    return _assemble(rng, name, n_stops, edges, types[0], types[1], lam[0], lam[1],
                     headway, irregular, conn_target, reading, seed,
                     lam_override=(lo, hi))


def queries(n_vertices: int, n: int, seed: int) -> Queries:
    """Sources uniform over the stops, departure times uniform over the day."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n_vertices, size=n).astype(np.int32)
    ts = rng.integers(0, DAY, size=n).astype(np.int32)
    return Queries(s=s, ts=ts, seed=int(seed))


# ---------------------------------------------------------------------------
# Named workloads.  Each mirrors one benchmark configuration: stop count, edge
# rule, types per edge, duration range, headways, irregular share, connection
# total and query count.
# ---------------------------------------------------------------------------

SMALL_HEADWAYS = (300, 600, 900, 1200, 1800)


def city_1k(reading: str = "S", seed: int = 1) -> Timetable:
    """1,000 stops, 3-NN both ways, 1-3 types per edge, lam in [60,1800] s,
    headway in {5,10,15,20,30} min, 10% irregular, about 200k connections."""
    return transit_city(1000, 3, (1, 3), (60, 1800), SMALL_HEADWAYS, 0.10, 200_000,
                        seed, reading, name=f"city-1k-{reading}")


def city_50k(reading: str = "S", seed: int = 2) -> Timetable:
    """50,000 stops, 5-NN both ways, 1-4 types per edge, lam in [30,3600] s,
    headway 120-3600 s, 15% irregular, about 12M connections."""
    return transit_city(50_000, 5, (1, 4), (30, 3600), (120, 3600), 0.15, 12_000_000,
                        seed, reading, name=f"city-50k-{reading}")


def region_500k(reading: str = "S", seed: int = 3) -> Timetable:
    """500,000 stops in 20 Gaussian towns, 5-NN inside towns plus long
    inter-town edges (lam 1800-7200 s), 80% of departures on progressions,
    about 120M connections."""
    return transit_region(500_000, 20, 5, 0.02, 3, 8, (1, 4), (30, 3600), (1800, 7200),
                          (120, 3600), 0.25, 120_000_000, seed, reading,
                          name=f"region-500k-{reading}")


def scaled_city(n_stops: int, seed: int, reading: str = "S") -> Timetable:
    """A city of any size at the densities above: below 10k stops the 1k-stop
    recipe (200 connections per stop), from 10k stops the 50k-stop recipe (240
    connections per stop)."""
    if n_stops < 10_000:
        return transit_city(n_stops, 3, (1, 3), (60, 1800), SMALL_HEADWAYS, 0.10,
                            200 * n_stops, seed, reading, name=f"city-{n_stops}-{reading}")
    return transit_city(n_stops, 5, (1, 4), (30, 3600), (120, 3600), 0.15, 240 * n_stops,
                        seed, reading, name=f"city-{n_stops}-{reading}")


def transit_lines(n_stops: int, knn: int, n_lines: int, stops_per_line: Sequence[int],
                  segment: Sequence[int], dwell: Sequence[int], headway: Sequence[int], seed: int,
                  name: str = "lines") -> Timetable:
    """A timetable made of vehicle trips (the trips of Section II-G).  Stops
    are uniform in the unit square with k-NN neighbours; a line is a walk of
    distinct neighbouring stops, served in both directions; every segment of a
    line has a running time and every intermediate stop a dwell time, the same
    for all its trips; a direction's trips leave the first stop every headway
    from a start in [05:00, 07:00] until 23:00.  A trip's connection i leaves
    stop i at t_i and reaches stop i+1 at t_i + lam_i <= t_{i+1}.
    ``trip`` numbers each connection's trip."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n_stops, 2))
    k = min(knn, n_stops - 1)
    _, nbr = cKDTree(pts).query(pts, k=k + 1)
    nbr = nbr[:, 1:]
    us, vs, ts, ls, trips = [], [], [], [], []
    next_trip = 0
    for _ in range(n_lines):
        want = int(rng.integers(stops_per_line[0], stops_per_line[1] + 1))
        walk = [int(rng.integers(0, n_stops))]
        seen = {walk[0]}
        while len(walk) < want:
            cand = [int(x) for x in nbr[walk[-1]] if int(x) not in seen]
            if not cand:
                break
            nxt = cand[int(rng.integers(0, len(cand)))]
            walk.append(nxt)
            seen.add(nxt)
        if len(walk) < 2:
            continue
        run = rng.integers(segment[0], segment[1] + 1, size=len(walk) - 1)
        stay = rng.integers(dwell[0], dwell[1] + 1, size=len(walk))
        h = int(rng.integers(headway[0], headway[1] + 1))
        for stops, seg, dw in ((walk, run, stay), (walk[::-1], run[::-1], stay[::-1])):
            start = int(rng.integers(AP_START_LO, AP_START_HI + 1))
            # departure offsets of the trip's connections from its first departure
            off = np.zeros(len(stops) - 1, dtype=np.int64)
            for i in range(1, len(stops) - 1):
                off[i] = off[i - 1] + seg[i - 1] + dw[i]
            n_trips = (AP_END_CAP - start) // h + 1
            first = start + h * np.arange(n_trips, dtype=np.int64)
            t = (first[:, None] + off[None, :]).reshape(-1)
            us.append(np.tile(np.asarray(stops[:-1], np.int64), n_trips))
            vs.append(np.tile(np.asarray(stops[1:], np.int64), n_trips))
            ts.append(t)
            ls.append(np.tile(np.asarray(seg, np.int64), n_trips))
            trips.append(np.repeat(np.arange(next_trip, next_trip + n_trips, dtype=np.int64), len(stops) - 1))
            next_trip += n_trips
    u = np.concatenate(us).astype(np.int32)
    v = np.concatenate(vs).astype(np.int32)
    t = np.concatenate(ts).astype(np.int32)
    lam = np.concatenate(ls).astype(np.int32)
    trip = np.concatenate(trips).astype(np.int32)
    order = rng.permutation(len(u))  # no order is implied by position
    n_edges = len(np.unique(u.astype(np.int64) * n_stops + v))
    return Timetable(name=name, n_vertices=int(n_stops), u=u[order], v=v[order], t=t[order], lam=lam[order],
                     n_edges=int(n_edges), n_types_drawn=-1, seed=int(seed), trip=trip[order])


def lines_city(n_stops: int = 10_000, seed: int = 601) -> Timetable:
    """A city served by bus lines: k = 5 neighbours, lines of 8..40 stops (one
    per 8 stops, both directions), 60..600 s segments, 0..60 s dwell, headway
    5..30 min."""
    return transit_lines(n_stops, 5, n_stops // 8, (8, 40), (60, 600), (0, 60), (300, 1800), seed,
                         name=f"lines-{n_stops}")


MIXED_BATCH_SIZES = (2_000, 5_000, 10_000, 20_000, 50_000, 100_000, 200_000, 500_000)
SERVE_SIZES = (10_000, 50_000, 500_000)

WORKLOADS = {
    # name: (timetable factory, query count, query seed)
    "city-1k": (lambda r="S": city_1k(r), 16, 10001),
    "city-50k": (lambda r="S": city_50k(r), 256, 10002),
    "region-500k": (lambda r="S": region_500k(r), 64, 10003),
}


def workload(name: str, reading: str = "S"):
    """(timetable, queries) of a named single-graph workload."""
    make, nq, qseed = WORKLOADS[name]
    tt = make(reading)
    return tt, queries(tt.n_vertices, nq, qseed)


def cities(sizes: Sequence[int], first_seed: int, reading: str = "S", workers: int = 8):
    """scaled_city(sizes[i], first_seed + i) for every i, drawn on a few threads
    (each city has its own seeded generator, so the result does not depend on
    the thread count)."""
    from concurrent.futures import ThreadPoolExecutor

    jobs = list(enumerate(sizes))
    if workers <= 1:
        return [scaled_city(n, first_seed + i, reading) for i, n in jobs]
    with ThreadPoolExecutor(min(workers, len(jobs))) as ex:
        return list(ex.map(lambda j: scaled_city(j[1], first_seed + j[0], reading), jobs))


def mixed_batch(reading: str = "S", workers: int = 8):
    """Eight cities of uneven size with 512 queries each."""
    graphs = cities(MIXED_BATCH_SIZES, 401, reading, workers)
    qs = [queries(n, 512, 10401 + i) for i, n in enumerate(MIXED_BATCH_SIZES)]
    return graphs, qs


def serving_cities(reading: str = "S", workers: int = 8):
    """The three resident cities of the serving workload (10k, 50k, 500k stops)."""
    return cities(SERVE_SIZES, 501, reading, workers)


def random_tiny(rng: np.random.Generator, max_v: int = 7, max_c: int = 20,
                max_t: int = 30, max_lam: int = 5) -> Timetable:
    """A tiny random timetable with many equal times and short durations, for
    brute-force comparisons."""
    nv = int(rng.integers(1, max_v + 1))
    n = int(rng.integers(0, max_c + 1))
    u = rng.integers(0, nv, size=n).astype(np.int32)
    v = rng.integers(0, nv, size=n).astype(np.int32)
    t = rng.integers(0, max_t + 1, size=n).astype(np.int32)
    lam = rng.integers(1, max_lam + 1, size=n).astype(np.int32)
    return Timetable(name="tiny", n_vertices=nv, u=u, v=v, t=t, lam=lam,
                     n_edges=-1, n_types_drawn=-1, seed=-1)
