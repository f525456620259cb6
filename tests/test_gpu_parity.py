"""GPU parity: libeat's HIP path against the CPU oracle, element by element,
bit-exact (the EAT answer is a unique int32 array).  Every call goes through the
C ABI (ctypes binding); the oracle is the plain connection scan (Algorithm 1)
plus the certificate."""
import functools
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_examples.json")))
INF = oracle.INF

LAYOUTS = {"hybrid": eat.EAT_LAYOUT_HYBRID, "flat": eat.EAT_LAYOUT_FLAT}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eat.lib()  # the native library must load; there is no fallback


@functools.lru_cache(maxsize=None)
def _workload(name):
    return synth.workload(name)


@functools.lru_cache(maxsize=None)
def _csa(name):
    tt, _ = _workload(name)
    return oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)


@functools.lru_cache(maxsize=None)
def _expected(name):
    tt, q = _workload(name)
    return _csa(name).query_many(q.s, q.ts)


@functools.lru_cache(maxsize=None)
def _graph(name, layout, cw=0):
    tt, _ = _workload(name)
    return eat.eat_graph_build(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, layout=LAYOUTS[layout],
                               cluster_seconds=cw)


def _query(g, s, ts, **opt):
    out = torch.full((g.n_vertices,), -7, dtype=torch.int32, device="cuda")
    st = eat.eat_query(g, s, ts, out, options=opt or None, stats=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st


# ------------------------------------------------------------- next departure

def _types_of(view):
    """(u, v, lam) of every layout type, in layout order."""
    vt = view["vt"]
    u = np.empty(len(view["ty"]), dtype=np.int64)
    for stop in range(len(vt)):
        u[vt[stop, 0]: vt[stop, 0] + vt[stop, 1]] = stop
    return u, view["ty"][:, 0], view["ty"][:, 1]


@pytest.mark.parametrize("layout,cw,headers", [
    ("hybrid", 0, eat.EAT_HEADERS_GRID), ("hybrid", 0, eat.EAT_HEADERS_COMPACT),
    ("hybrid", 1800, eat.EAT_HEADERS_GRID), ("hybrid", 1800, eat.EAT_HEADERS_COMPACT),
    ("flat", 0, eat.EAT_HEADERS_AUTO)])
def test_next_departure_matches_definition(layout, cw, headers):
    """Per-type lookup (Sections II-B..II-D, Algorithm 6) vs min{t >= x} computed
    from the raw connection list, for every connection type of the 1k-stop
    city, for both device forms of the hybrid layout
    (header grid, compact headers) and the flat layout; 1800-s clusters give 48
    clusters per type (occupancy bits above 32)."""
    tt, _ = _workload("city-1k")
    _say(f"next_departure city-1k {layout} cw={cw} headers={headers}")
    lay = eat.eat_layout_build(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, layout=LAYOUTS[layout],
                               cluster_seconds=cw)
    view = lay.view()
    tu, tv, tl = _types_of(view)
    # departures of every (u, v, lam) from the raw input
    order = np.lexsort((tt.t, tt.lam, tt.v, tt.u))
    key = np.stack([tt.u[order], tt.v[order], tt.lam[order]], 1)
    starts = np.flatnonzero(np.r_[True, (np.diff(key, axis=0) != 0).any(1)])
    bounds = np.r_[starts, len(order)]
    index = {tuple(key[s]): (bounds[i], bounds[i + 1]) for i, s in enumerate(starts)}
    rng = np.random.default_rng(11)
    g = _graph("city-1k", layout, cw)
    if layout == "hybrid":
        assert g.info.n_grid_entries == g.info.n_types * g.info.n_clusters
    # every connection type of the city, each probed around its departures,
    # at cluster boundaries and at random times; a few at every second of the day
    picks = np.arange(len(tu))
    ids, xs, segs = [], [], []
    n_probe = 0
    for j in list(picks) + list(rng.choice(len(tu), size=4, replace=False)):
        b, e = index[(tu[j], tv[j], tl[j])]
        d = tt.t[order[b:e]]
        if len(segs) < len(picks):
            probe = np.unique(np.concatenate([d - 1, d, d + 1, np.arange(0, 90001, 3600) - 1,
                                              np.arange(0, 90001, 3600), rng.integers(0, 90000, 20),
                                              [0, int(tt.t.max()) + 1, 2**31 - 2]]))
            probe = probe[probe >= 0]
        else:
            probe = np.arange(90001)
        ids.append(np.full(len(probe), j))
        xs.append(probe)
        segs.append((j, n_probe, n_probe + len(probe)))
        n_probe += len(probe)
    ids = np.concatenate(ids).astype(np.int32)
    xs = np.concatenate(xs).astype(np.int32)
    _say(f"  {len(picks)} types, {len(ids)} probes")
    out = torch.empty(len(ids), dtype=torch.int32, device="cuda")
    eat.eat_next_departure(g, torch.from_numpy(ids).cuda(), torch.from_numpy(xs).cuda(), out,
                           headers=headers)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    # expected: definition on the raw departures of each probed type
    exp = np.empty_like(got)
    for j, p0, p1 in segs:
        b, e = index[(tu[j], tv[j], tl[j])]
        d = np.sort(tt.t[order[b:e]])
        pos = np.searchsorted(d, xs[p0:p1], side="left")
        exp[p0:p1] = np.where(pos < len(d), d[np.minimum(pos, len(d) - 1)], INF)
    # spot-check the numpy expectation against the oracle's own definition
    for k in rng.choice(len(ids), size=300, replace=False):
        j = ids[k]
        b, e = index[(tu[j], tv[j], tl[j])]
        assert exp[k] == oracle.next_departure(tt.t[order[b:e]], int(xs[k]))
    assert np.array_equal(got, exp)


# ------------------------------------------------------------- single queries

@pytest.mark.parametrize("layout", ["hybrid", "flat"])
@pytest.mark.parametrize("tpv", [0, 1, 4, 16, 64])
def test_single_queries_city_1k_bit_exact(layout, tpv):
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = _graph("city-1k", layout)
    _say(f"single city-1k {layout} tpv={tpv}")
    for i, (s, ts) in enumerate(zip(q.s, q.ts)):
        got, st = _query(g, s, ts, threads_per_vertex=tpv)
        assert st["status"] == 0
        assert np.array_equal(got, exp[i]), (i, s, ts, np.flatnonzero(got != exp[i])[:10])


@pytest.mark.parametrize("tpv", [0, 8])
@pytest.mark.parametrize("cw", [0, 1800])
def test_compact_headers_are_exact(tpv, cw):
    """The hybrid layout's compact headers (one per non-empty cluster) give the
    same answers as the header grid, which AUTO picks when the graph has one."""
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = _graph("city-1k", "hybrid", cw)
    _say(f"compact headers city-1k tpv={tpv} cw={cw}")
    for i, (s, ts) in enumerate(zip(q.s, q.ts)):
        got, st = _query(g, s, ts, threads_per_vertex=tpv, headers=eat.EAT_HEADERS_COMPACT)
        assert np.array_equal(got, exp[i]), (i, s, ts)
        got2, st2 = _query(g, s, ts, threads_per_vertex=tpv, headers=eat.EAT_HEADERS_GRID)
        assert np.array_equal(got2, exp[i]), (i, s, ts)


def test_graph_without_grid_uses_compact_headers():
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = eat.graph_from_timetable(tt, header_grid=-1)
    assert g.info.n_grid_entries == 0
    got, _ = _query(g, int(q.s[0]), int(q.ts[0]))
    assert np.array_equal(got, exp[0])
    out = torch.empty(g.n_vertices, dtype=torch.int32, device="cuda")
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query(g, 0, 0, out, options={"headers": eat.EAT_HEADERS_GRID})
    assert ei.value.status == eat.EAT_ERR_UNSUPPORTED
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query(g, 0, 0, out, options={"headers": 7})
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("mode", [eat.EAT_MODE_TOPOLOGY, eat.EAT_MODE_FRONTIER])
@pytest.mark.parametrize("fcap", [64, 0])
@pytest.mark.parametrize("table", [0, -1, 64])
def test_modes_stores_and_overflows_are_exact(mode, fcap, table):
    """Frontier / topology rounds (topology rounds sweep every round), arrivals
    in the on-chip table, in the slab, and a table too small (spill to the
    slab).  Frontier-list overflow on a larger graph:
    test_small_lists_overflow_into_sweeps_city_50k."""
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = _graph("city-1k", "hybrid")
    _say(f"modes city-1k mode={mode} fcap={fcap} table={table}")
    sweeps = spills = 0
    for i, (s, ts) in enumerate(zip(q.s, q.ts)):
        got, st = _query(g, s, ts, mode=mode, frontier_cap=fcap, table_cap=table)
        sweeps += st["sweep_rounds"]
        spills += st["spilled"]
        assert st["reached"] == int((exp[i] < INF).sum())
        assert np.array_equal(got, exp[i]), (i, s, ts)
    if mode == eat.EAT_MODE_TOPOLOGY:
        assert sweeps > 0  # the sweep path really ran
    if table == 64:
        assert spills > 0  # some queries reach more than 48 stops: the spill path ran
    else:
        assert spills == 0


@pytest.mark.parametrize("window", [-1, 1, 60, 600, 7200])
@pytest.mark.parametrize("tpv", [0, 16])
def test_time_windows_are_exact(window, tpv):
    """Rounds that expand only the stops below the smallest pushed arrival plus a
    window (deferring the rest) reach the same fixpoint; -1 = every listed stop
    every round."""
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = _graph("city-1k", "hybrid")
    _say(f"time window {window} tpv={tpv}")
    for i, (s, ts) in enumerate(zip(q.s, q.ts)):
        got, st = _query(g, s, ts, time_window=window, threads_per_vertex=tpv)
        assert st["status"] == 0
        assert np.array_equal(got, exp[i]), (i, s, ts)
    # with overflowing lists (sweeps) and the topology schedule as well
    for opts in ({"frontier_cap": 64}, {"mode": eat.EAT_MODE_TOPOLOGY}, {"table_cap": -1}):
        for i in (0, 5, 11):
            got, _ = _query(g, int(q.s[i]), int(q.ts[i]), time_window=window, threads_per_vertex=tpv, **opts)
            assert np.array_equal(got, exp[i]), (i, opts)


@pytest.mark.parametrize("threads", [512, 768, 384, 256])
@pytest.mark.parametrize("opts", [{}, {"table_cap": 64}, {"time_window": -1}, {"types_per_lane": 2},
                                  {"headers": eat.EAT_HEADERS_COMPACT}, {"mode": eat.EAT_MODE_TOPOLOGY},
                                  {"frontier_cap": 64}])
def test_two_queries_per_cu_are_exact(threads, opts):
    """Several queries per CU (512- or 768-thread work-groups with half the LDS
    each, 384 with a quarter, 256 with a sixth) give the same answers, also
    when the smaller table overflows."""
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = _graph("city-1k", "hybrid")
    _say(f"{threads} threads {opts}")
    if threads != 512 and opts.get("types_per_lane", 1) > 1:
        # 256-, 384- and 768-thread queries run at 80 VGPRs: only one type per lane fits
        out = torch.empty(g.n_vertices, dtype=torch.int32, device="cuda")
        with pytest.raises(eat.EatError) as ei:
            eat.eat_query(g, int(q.s[0]), int(q.ts[0]), out, options=dict(opts, threads_per_query=threads))
        assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
        return
    for i, (s, ts) in enumerate(zip(q.s, q.ts)):
        got, st = _query(g, s, ts, threads_per_query=threads, **opts)
        assert st["status"] == 0
        assert np.array_equal(got, exp[i]), (i, s, ts)


def test_512_threads_need_wave_claims():
    g = _graph("city-1k", "hybrid")
    out = torch.empty(g.n_vertices, dtype=torch.int32, device="cuda")
    for bad in ({"threads_per_query": 512, "threads_per_vertex": 16}, {"threads_per_query": 768, "threads_per_vertex": 4},
                {"threads_per_query": 384, "threads_per_vertex": 8}, {"threads_per_query": 640}):
        with pytest.raises(eat.EatError) as ei:
            eat.eat_query(g, 0, 0, out, options=bad)
        assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT


def test_small_work_groups_and_the_lds_bitmap_limit():
    """384- and 256-thread queries run a 70,000-stop graph; a 300,000-stop one,
    whose activity bitmap does not fit their share of the LDS, is refused
    before any launch (arr untouched), alone and in a batch with a small
    graph; 768 threads run it."""
    small = _graph("city-1k", "hybrid")
    out_small = torch.full((small.n_vertices,), -7, dtype=torch.int32, device="cuda")
    mid = eat.eat_graph_build(np.array([0, 1]), np.array([1, 2]), np.array([10, 20]), np.array([5, 5]), 70000)
    for th in (384, 256):
        got, _ = _query(mid, 0, 0, threads_per_query=th)
        assert got[:3].tolist() == [0, 15, 25] and np.all(got[3:] == oracle.INF)
    n = 300000
    big = eat.eat_graph_build(np.array([0, 1]), np.array([1, 2]), np.array([10, 20]), np.array([5, 5]), n)
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    for th in (384, 256):
        with pytest.raises(eat.EatError) as ei:
            eat.eat_query(big, 0, 0, out, options={"threads_per_query": th})
        assert ei.value.status == eat.EAT_ERR_UNSUPPORTED
        with pytest.raises(eat.EatError) as ei:
            eat.eat_query_batch([small, big], np.array([0, 1], np.int32), np.array([0, 0], np.int32),
                                np.array([0, 0], np.int32), [out_small, out], options={"threads_per_query": th})
        assert ei.value.status == eat.EAT_ERR_UNSUPPORTED
    assert torch.all(out == -7) and torch.all(out_small == -7)
    got, _ = _query(big, 0, 0, threads_per_query=768)
    assert got[:3].tolist() == [0, 15, 25] and np.all(got[3:] == oracle.INF)


def test_certificate_holds_for_gpu_answers():
    tt, q = _workload("city-1k")
    g = _graph("city-1k", "hybrid")
    for s, ts in zip(q.s, q.ts):
        got, _ = _query(g, s, ts)
        assert oracle.certify(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts, got) == 0


def test_repeated_runs_are_identical():
    tt, q = _workload("city-1k")
    g = _graph("city-1k", "hybrid")
    s, ts = int(q.s[0]), int(q.ts[0])
    first, _ = _query(g, s, ts)
    for tpv in (0, 2, 8, 32):
        for _ in range(5):
            again, _ = _query(g, s, ts, threads_per_vertex=tpv)
            assert np.array_equal(first, again)
    for ub in (1, 2, 3):
        again, _ = _query(g, s, ts, types_per_lane=ub)
        assert np.array_equal(first, again)


# ------------------------------------------------------------- batches

def _batch(graphs, q_graph, q_src, q_ts, **opt):
    outs = [torch.full((graphs[gi].n_vertices,), -7, dtype=torch.int32, device="cuda") for gi in q_graph]
    st = eat.eat_query_batch(graphs, q_graph, q_src, q_ts, outs, options=opt or None, stats=True)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], st


@pytest.mark.parametrize("layout", ["hybrid", "flat"])
def test_batch_city_1k_equals_oracle(layout):
    tt, q = _workload("city-1k")
    exp = _expected("city-1k")
    g = _graph("city-1k", layout)
    _say(f"batch city-1k {layout}")
    outs, st = _batch([g], np.zeros(len(q), np.int32), q.s, q.ts)
    for i in range(len(q)):
        assert st[i]["status"] == 0
        assert np.array_equal(outs[i], exp[i]), i


@pytest.mark.parametrize("layout,headers,threads", [("hybrid", eat.EAT_HEADERS_GRID, 1024),
                                                    ("hybrid", eat.EAT_HEADERS_GRID, 512),
                                                    ("hybrid", eat.EAT_HEADERS_GRID, 768),
                                                    ("hybrid", eat.EAT_HEADERS_GRID, 384),
                                                    ("hybrid", eat.EAT_HEADERS_GRID, 256),
                                                    ("hybrid", eat.EAT_HEADERS_COMPACT, 1024),
                                                    ("flat", eat.EAT_HEADERS_AUTO, 512)])
def test_batch_city_50k_all_256_queries_bit_exact(layout, headers, threads):
    tt, q = _workload("city-50k")
    _say(f"batch city-50k {layout} headers={headers}: building graph")
    g = _graph("city-50k", layout)
    _say("  running batch")
    V = tt.n_vertices
    slab = torch.full((len(q), V), -7, dtype=torch.int32, device="cuda")
    b = eat.Batch([g], np.zeros(len(q), np.int32), q.s, q.ts, [slab[i] for i in range(len(q))],
                  options={"headers": headers, "threads_per_query": threads})
    b.run()
    st = b.wait(stats=True)
    got = slab.cpu().numpy()
    _say("  oracle")
    exp = _expected("city-50k")
    bad = [i for i in range(len(q)) if not np.array_equal(got[i], exp[i])]
    assert not bad, bad[:10]
    assert all(x["status"] == 0 for x in st)
    # repeat the prepared batch: the counters re-arm themselves
    slab.fill_(-7)
    b.run()
    b.wait()
    assert np.array_equal(slab.cpu().numpy(), exp)
    for i in (0, 17, 101):
        assert oracle.certify(tt.u, tt.v, tt.t, tt.lam, V, q.s[i], q.ts[i], got[i]) == 0


@pytest.mark.parametrize("opts", [{}, {"time_window": -1}, {"threads_per_vertex": 16}, {"table_cap": -1},
                                  {"threads_per_query": 512}, {"threads_per_query": 768},
                                  {"threads_per_query": 768, "table_cap": -1}, {"types_per_lane": 2},
                                  {"threads_per_query": 384}, {"threads_per_query": 256},
                                  {"mode": eat.EAT_MODE_TOPOLOGY}, {"mode": eat.EAT_MODE_TOPOLOGY, "time_window": 1800},
                                  {"mode": eat.EAT_MODE_TOPOLOGY, "threads_per_query": 384, "table_cap": -1},
                                  {"mode": eat.EAT_MODE_TOPOLOGY, "threads_per_query": 768},
                                  {"mode": eat.EAT_MODE_TOPOLOGY, "threads_per_query": 256},
                                  {"mode": eat.EAT_MODE_TOPOLOGY, "threads_per_query": 512, "table_cap": -1}])
def test_small_lists_overflow_into_sweeps_city_50k(opts):
    """64-entry frontier lists (the smallest): rounds whose pushes overflow the
    list sweep the activity flags in chunks of up to 64 items instead; every
    answer stays exact, with arrivals in the table or in the slab.  The
    topology cases sweep every round, so every work-group size starts many
    chunks close to the end of its group cursor."""
    tt, q = _workload("city-50k")
    g = _graph("city-50k", "hybrid")
    exp = _expected("city-50k")
    V, Q = tt.n_vertices, len(q)
    _say(f"city-50k frontier_cap 64 {opts}")
    slab = torch.full((Q, V), -7, dtype=torch.int32, device="cuda")
    b = eat.Batch([g], np.zeros(Q, np.int32), q.s, q.ts, [slab[i] for i in range(Q)],
                  options=dict(opts, frontier_cap=64))
    b.run()
    st = b.wait(stats=True)
    got = slab.cpu().numpy()
    b.free()
    bad = [i for i in range(Q) if not np.array_equal(got[i], exp[i])]
    assert not bad, bad[:10]
    assert all(x["status"] == 0 for x in st)
    assert sum(x["sweep_rounds"] for x in st) > 0
    assert all(x["reached"] == int((exp[i] < INF).sum()) for i, x in enumerate(st))


def test_batch_run_replays_from_a_captured_hip_graph():
    """A prepared batch's run is one persistent kernel launch on the caller's
    stream, with no memset or copy (its counters re-arm on the device), so it
    can be captured into a HIP graph and replayed.  Every replay -- with eager
    work and synchronisations between the replays -- gives the oracle's
    answers, and the batch still runs eagerly afterwards."""
    tt, q = _workload("city-50k")
    g = _graph("city-50k", "hybrid")
    exp = _expected("city-50k")
    V, Q = tt.n_vertices, len(q)
    _say("city-50k batch in a captured HIP graph")
    slab = torch.full((Q, V), -7, dtype=torch.int32, device="cuda")
    b = eat.Batch([g], np.zeros(Q, np.int32), q.s, q.ts, [slab[i] for i in range(Q)],
                  options={"threads_per_query": 512})
    b.run()
    b.wait()  # an eager run first
    assert np.array_equal(slab.cpu().numpy(), exp)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        b.run()  # on the capturing stream
    torch.cuda.synchronize()
    for rep in range(4):
        slab.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(slab.cpu().numpy(), exp), rep
    del graph
    slab.fill_(-7)
    b.run()
    b.wait()
    assert np.array_equal(slab.cpu().numpy(), exp)
    b.free()


def test_graph_built_on_a_stream_while_another_stream_runs():
    """eat_graph_build on a stream of its own (uploads, the grid build and the
    final wait on that stream) while a batch on another graph runs on a second
    stream: both answers equal the scan's."""
    tt, q = _workload("city-1k")
    g1 = _graph("city-1k", "hybrid")
    busy = torch.cuda.Stream()
    slab = torch.full((len(q), tt.n_vertices), -7, dtype=torch.int32, device="cuda")
    b = eat.Batch([g1], np.zeros(len(q), np.int32), q.s, q.ts, [slab[i] for i in range(len(q))])
    b.run(busy)
    tt2 = synth.scaled_city(5000, seed=403)
    side = torch.cuda.Stream()
    g2 = eat.eat_graph_build(tt2.u, tt2.v, tt2.t, tt2.lam, tt2.n_vertices, stream=side)
    q2 = synth.queries(tt2.n_vertices, 8, 778)
    c2 = oracle.Csa(tt2.u, tt2.v, tt2.t, tt2.lam, tt2.n_vertices)
    for i in range(len(q2.s)):
        got, _ = _query(g2, int(q2.s[i]), int(q2.ts[i]))
        assert np.array_equal(got, c2.query(int(q2.s[i]), int(q2.ts[i]))), i
    b.wait()
    assert np.array_equal(slab.cpu().numpy(), _expected("city-1k"))
    b.free()


def test_batch_equals_single_queries_and_mixed_graphs():
    """Alone == batched, with two graphs of different size in one launch."""
    tt1, q1 = _workload("city-1k")
    g1 = _graph("city-1k", "hybrid")
    tt2 = synth.scaled_city(5000, seed=402)
    g2 = eat.graph_from_timetable(tt2)
    q2 = synth.queries(tt2.n_vertices, 24, 777)
    c2 = oracle.Csa(tt2.u, tt2.v, tt2.t, tt2.lam, tt2.n_vertices)
    qg = np.r_[np.zeros(len(q1), np.int32), np.ones(len(q2), np.int32)]
    qs = np.r_[q1.s, q2.s]
    qt = np.r_[q1.ts, q2.ts]
    perm = np.random.default_rng(1).permutation(len(qg))
    outs, st = _batch([g1, g2], qg[perm], qs[perm], qt[perm])
    exp1 = _expected("city-1k")
    for k, i in enumerate(perm):
        exp = exp1[i] if i < len(q1) else c2.query(qs[i], qt[i])
        assert np.array_equal(outs[k], exp), (k, i)
        alone, _ = _query(g1 if qg[i] == 0 else g2, qs[i], qt[i])
        assert np.array_equal(alone, outs[k])



@pytest.mark.parametrize("order", [eat.EAT_ORDER_AUTO, eat.EAT_ORDER_LOCALITY, eat.EAT_ORDER_LONGEST_FIRST,
                                   eat.EAT_ORDER_BANDED])
def test_query_orders_change_nothing_but_the_schedule(order):
    """The order in which work-groups take a batch's queries is a schedule
    only: on two graphs with more queries than work-groups in flight (1,200 on
    a 1k-stop city, 300 on a 5k-stop one, shuffled), every answer equals the
    scan's and every query's statistics land at its own index."""
    tt1, _ = _workload("city-1k")
    g1 = _graph("city-1k", "hybrid")
    tt2 = synth.scaled_city(5000, seed=402)
    g2 = eat.graph_from_timetable(tt2)
    qa = synth.queries(tt1.n_vertices, 1200, 901)
    qb = synth.queries(tt2.n_vertices, 300, 902)
    qg = np.r_[np.zeros(len(qa.s), np.int32), np.ones(len(qb.s), np.int32)]
    qs = np.r_[qa.s, qb.s]
    qt = np.r_[qa.ts, qb.ts]
    perm = np.random.default_rng(order).permutation(len(qg))
    qg, qs, qt = qg[perm], qs[perm], qt[perm]
    _say(f"order {order}: {len(qg)} queries over two graphs")
    outs, st = _batch([g1, g2], qg, qs, qt, query_order=order, threads_per_query=768)
    c1 = _csa("city-1k")
    c2 = oracle.Csa(tt2.u, tt2.v, tt2.t, tt2.lam, tt2.n_vertices)
    for k in range(len(qg)):
        exp = (c1 if qg[k] == 0 else c2).query(int(qs[k]), int(qt[k]))
        assert np.array_equal(outs[k], exp), (order, k)
        assert st[k]["status"] == 0
        if st[k]["spilled"] == 0:  # the on-chip table counts the stops it holds
            assert st[k]["reached"] == int(np.count_nonzero(exp != oracle.INF)), (order, k)


def test_unknown_query_order_is_refused():
    tt, q = _workload("city-1k")
    g = _graph("city-1k", "hybrid")
    out = torch.full((tt.n_vertices,), -7, dtype=torch.int32, device="cuda")
    for bad in (-1, 4):
        with pytest.raises(eat.EatError) as ei:
            eat.eat_query_batch([g], np.zeros(1, np.int32), q.s[:1], q.ts[:1], [out], options={"query_order": bad})
        assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    assert torch.all(out == -7)


# ------------------------------------------------------------- edge cases

def test_racing_candidates_keep_the_minimum():
    """Section III-C: concurrent candidates 3 and 6 for one stop must leave 3."""
    ex = GOLDEN["racing_updates"]
    rng = np.random.default_rng(0)
    # 64 connection types 0 -> 1 departing at 0, all relaxed in the same round
    lam = np.r_[ex["candidates"], rng.integers(4, 500, 62)].astype(np.int32)
    n = len(lam)
    g = eat.eat_graph_build(np.zeros(n), np.ones(n), np.zeros(n), lam, 2)
    for tpv in (1, 64):
        got, _ = _query(g, 0, 0, threads_per_vertex=tpv)
        assert got.tolist() == [0, ex["result"]]


def _check_tt(tt, queries, layout="hybrid", cw=0, **opt):
    c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    g = eat.eat_graph_build(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, layout=LAYOUTS[layout],
                            cluster_seconds=cw)
    for s, ts in queries:
        got, st = _query(g, s, ts, **opt)
        assert np.array_equal(got, c.query(s, ts)), (s, ts)


def _hub_timetable(hub_types, seed):
    """Stop 0 with `hub_types` connection types (one per head stop 1..hub_types,
    three departures each), behind it a sparse random network over all stops,
    so one round holds the hub's types and later rounds are ordinary."""
    rng = np.random.default_rng(seed)
    V = hub_types + 3000
    heads = np.arange(1, hub_types + 1, dtype=np.int32)
    u = [np.zeros(3 * hub_types, np.int32)]
    v = [np.repeat(heads, 3)]
    t = [np.tile(np.array([3600, 5400, 9000], np.int32), hub_types) + rng.integers(0, 600, 3 * hub_types)]
    lam = [np.repeat(rng.integers(60, 3000, hub_types), 3)]
    m = 8 * V
    u.append(rng.integers(1, V, m))
    v.append(rng.integers(0, V, m))
    t.append(rng.integers(3600, 80000, m))
    lam.append(rng.integers(30, 1800, m))
    cat = lambda xs: np.concatenate(xs).astype(np.int32)
    u, v, t, lam = cat(u), cat(v), cat(t), cat(lam)
    keep = u != v
    return synth.Timetable(f"hub{hub_types}", V, u[keep], v[keep], t[keep], lam[keep], 0, 0, 0)


@pytest.mark.parametrize("hub_types", [5000, 9000])
def test_high_degree_stop(hub_types):
    """A stop with thousands of connection types: one entry whose types span
    up to 79 windows of 64 (5,000 types), and a round of more than 128 windows
    (9,000 types), which the kernels relax by claims of whole entries instead;
    with tables that hold the round and tables that overflow into the slab."""
    tt = _hub_timetable(hub_types, 11 + hub_types)
    c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    g = eat.eat_graph_build(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    src = np.array([0, 0, 0, 17, 1234], np.int32)
    ts = np.array([0, 5000, 8000, 3000, 3600], np.int32)
    exp = [c.query(int(s_), int(t_)) for s_, t_ in zip(src, ts)]
    for opts in ({}, {"threads_per_query": 768}, {"threads_per_query": 384}, {"threads_per_query": 256},
                 {"types_per_lane": 2}, {"types_per_lane": 3}, {"table_cap": -1}, {"time_window": -1},
                 {"threads_per_query": 768, "frontier_cap": 64}):
        _say(f"hub {hub_types}: {opts}")
        outs, st = _batch([g], np.zeros(len(src), np.int32), src, ts, **opts)
        for i in range(len(src)):
            assert st[i]["status"] == 0
            assert np.array_equal(outs[i], exp[i]), (opts, i)
    got, _ = _query(g, 0, 0)
    assert np.array_equal(got, exp[0])


def test_edge_cases():
    _say("edge cases")
    rng = np.random.default_rng(5)
    # isolated source, departure after the last connection, ts = 0
    tt, q = _workload("city-1k")
    _check_tt(tt, [(0, int(tt.t.max()) + 1), (int(q.s[0]), 0), (5, 86399)])
    # single vertex, no connections
    _check_tt(synth.Timetable("one", 1, *[np.zeros(0, np.int32)] * 4, 0, 0, 0), [(0, 0), (0, 12345)])
    # times near the int32 limit
    big = 2**31 - 1000
    tt2 = synth.Timetable("late", 3, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                          np.array([big, big + 10], np.int32), np.array([10, 998 - 11], np.int32),
                          0, 0, 0)
    _check_tt(tt2, [(0, big), (0, big - 5), (1, big + 10)], layout="flat")
    # a horizon of 50 hours (cluster bits above 31) in the hybrid layout
    tt3 = synth.random_tiny(rng, max_v=40, max_c=3000, max_t=50 * 3600 - 1, max_lam=4000)
    _check_tt(tt3, [(int(rng.integers(0, tt3.n_vertices)), int(rng.integers(0, 50 * 3600))) for _ in range(20)])
    # small clusters (30 min) and a dense random graph with many equal times
    tt4 = synth.random_tiny(rng, max_v=200, max_c=20000, max_t=1800 * 40, max_lam=600)
    c4 = [(int(rng.integers(0, tt4.n_vertices)), int(rng.integers(0, 72000))) for _ in range(20)]
    _check_tt(tt4, c4, cw=1800)
    _check_tt(tt4, c4, cw=1800, mode=eat.EAT_MODE_TOPOLOGY, threads_per_vertex=64)
    _check_tt(tt4, c4, layout="flat", frontier_cap=64)


def test_round_limit_reports_not_converged():
    tt, q = _workload("city-1k")
    g = _graph("city-1k", "hybrid")
    exp = _expected("city-1k")
    i = int(np.argmax((exp < INF).sum(1)))  # a query that needs several rounds
    out = torch.empty(tt.n_vertices, dtype=torch.int32, device="cuda")
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query(g, int(q.s[i]), int(q.ts[i]), out, options={"max_rounds": 2}, stats=True)
    assert ei.value.status == eat.EAT_ERR_NOT_CONVERGED
    # without stats the call is asynchronous; the graph counts the failure
    g2 = eat.graph_from_timetable(tt)
    assert g2.failures() == 0
    eat.eat_query(g2, int(q.s[i]), int(q.ts[i]), out)  # converges
    eat.eat_query(g2, int(q.s[i]), int(q.ts[i]), out, options={"max_rounds": 2})
    eat.eat_query(g2, int(q.s[i]), int(q.ts[i]), out, options={"max_rounds": 3})
    torch.cuda.synchronize()
    assert g2.failures() == 2


def test_invalid_query_arguments_leave_arr_untouched():
    g = _graph("city-1k", "hybrid")
    out = torch.full((g.n_vertices,), -7, dtype=torch.int32, device="cuda")
    for s, ts in ((-1, 0), (g.n_vertices, 0), (0, -1)):
        with pytest.raises(eat.EatError) as ei:
            eat.eat_query(g, s, ts, out)
        assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    with pytest.raises(eat.EatError):
        eat.eat_query(g, 0, 0, out, options={"threads_per_vertex": 3})
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == -7).all()


def test_autotuner_on_the_product_path():
    """The library's autotuner times every candidate on the 50k-stop city's
    256-query batch (all must agree on the device); a batch created afterwards
    without run options uses the tuned options and stays bit-exact; a batch of
    another size has no record and takes the defaults."""
    from paper_1912_00966_amd import autotune
    tt, q = _workload("city-50k")
    g = _graph("city-50k", "hybrid")
    exp = _expected("city-50k")
    V, Q = tt.n_vertices, len(q)
    slab = torch.full((Q, V), -7, dtype=torch.int32, device="cuda")
    _say("autotune city-50k")
    best, results = autotune.tune([g], np.zeros(Q, np.int32), q.s, q.ts, [slab[i] for i in range(Q)],
                                  reps=2, streams=2, verbose=True)
    assert len(results) >= 8 and best in [o for o, _ in results]
    assert min(ms for _, ms in results) == [ms for o, ms in results if o == best][0]
    assert np.array_equal(slab.cpu().numpy(), exp)  # the tuner leaves the answers in the slabs
    slab.fill_(-7)
    b = eat.Batch([g], np.zeros(Q, np.int32), q.s, q.ts, [slab[i] for i in range(Q)], options=None)
    assert b.options() == best
    b.run()
    b.wait()
    assert np.array_equal(slab.cpu().numpy(), exp)
    b.free()
    b2 = eat.Batch([g], np.zeros(17, np.int32), q.s[:17], q.ts[:17], [slab[i] for i in range(17)])
    assert b2.options()["threads_per_query"] == 0  # no record for 17 queries: the defaults
    b2.run()
    b2.wait()
    assert np.array_equal(slab[:17].cpu().numpy(), exp[:17])
    b2.free()


def test_concurrent_batches_on_several_streams():
    """Prepared batches of the same graph run concurrently on four streams (the
    way bench.py overlaps steps); every stream's slabs stay exact."""
    tt, q = _workload("city-50k")
    g = _graph("city-50k", "hybrid")
    exp = _expected("city-50k")
    V, Q = tt.n_vertices, len(q)
    slabs = [torch.full((Q, V), -7, dtype=torch.int32, device="cuda") for _ in range(4)]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(3)]
    batches = [eat.Batch([g], np.zeros(Q, np.int32), q.s, q.ts, [sl[i] for i in range(Q)],
                         options={"threads_per_query": (1024, 768, 512)[k % 3]}) for k, sl in enumerate(slabs)]
    _say("concurrent batches on 4 streams")
    for i in range(12):
        batches[i % 4].run(streams[i % 4])
    torch.cuda.synchronize()
    for b, sl in zip(batches, slabs):
        assert b.wait(stats=True) is not None
        assert np.array_equal(sl.cpu().numpy(), exp)
        b.free()
