"""Parity at full size: the 500,000-stop region (about 120M connections, 64
queries; every answer checked with the exact O(|C|) certificate -- source,
closure, witness -- which the oracle tests pin against the scan, and sampled
answers against the scan itself) and the mixed batch of eight cities (2k..500k
stops, 4,096 queries in one launch; every answer against the scan)."""
import functools
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eat.lib()


def _say(m):
    print(m, flush=True)


@functools.lru_cache(maxsize=None)
def _region():
    t0 = time.time()
    tt, q = synth.workload("region-500k")
    _say(f"region-500k generated in {time.time() - t0:.0f}s: {tt.n_conn} connections")
    g = eat.graph_from_timetable(tt)
    return tt, q, g


def _certify(tt, s, ts, arr):
    return oracle.certify(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, int(s), int(ts), arr)


def test_region_500k_batch_certified():
    tt, q, g = _region()
    V = tt.n_vertices
    slab = torch.full((len(q), V), -7, dtype=torch.int32, device="cuda")
    b = eat.Batch([g], np.zeros(len(q), np.int32), q.s, q.ts, [slab[i] for i in range(len(q))])
    b.run()
    st = b.wait(stats=True)
    got = slab.cpu().numpy()
    assert all(x["status"] == 0 for x in st)
    _say(f"region-500k: spilled {sum(x['spilled'] for x in st)} of {len(q)}, "
         f"max reached {max(x['reached'] for x in st)}")
    n_thr = max(1, min(len(os.sched_getaffinity(0)), 16))
    with ThreadPoolExecutor(n_thr) as ex:
        rc = list(ex.map(lambda i: _certify(tt, q.s[i], q.ts[i], got[i]), range(len(q))))
    for i in range(len(q)):
        assert (got[i] >= 0).all()
        assert rc[i] == 0, i
        assert st[i]["reached"] == int((got[i] < oracle.INF).sum())
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    with ThreadPoolExecutor(n_thr) as ex:
        exp = list(ex.map(lambda i: csa.query(int(q.s[i]), int(q.ts[i])), range(0, len(q), 4)))
    for k, i in enumerate(range(0, len(q), 4)):
        assert np.array_equal(got[i], exp[k]), i


def test_region_500k_modes_agree():
    """Frontier vs topology rounds, on-chip table vs slab, on sampled queries."""
    tt, q, g = _region()
    for i in (0, 7, 33):
        ref = g.query(int(q.s[i]), int(q.ts[i])).cpu().numpy()
        for opts in ({"mode": eat.EAT_MODE_TOPOLOGY}, {"table_cap": -1}, {"threads_per_vertex": 16}):
            alt = g.query(int(q.s[i]), int(q.ts[i]), options=opts).cpu().numpy()
            assert np.array_equal(ref, alt), (i, opts)
        assert _certify(tt, q.s[i], q.ts[i], ref) == 0


def test_mixed_batch_4096_queries_one_launch():
    """All 4,096 answers of the eight-city batch (2k..500k stops, one launch),
    element by element against the connection scan, graph by graph, with the
    oracle's queries spread over a thread pool (each query is one native call
    that releases the interpreter lock)."""
    t0 = time.time()
    graphs_tt, qsets = synth.mixed_batch()
    _say(f"mixed batch generated in {time.time() - t0:.0f}s")
    graphs = [eat.graph_from_timetable(t) for t in graphs_tt]
    qg = np.concatenate([np.full(len(qs), i, np.int32) for i, qs in enumerate(qsets)])
    qsrc = np.concatenate([qs.s for qs in qsets])
    qts = np.concatenate([qs.ts for qs in qsets])
    perm = np.random.default_rng(4).permutation(len(qg))  # interleave the graphs
    qg, qsrc, qts = qg[perm], qsrc[perm], qts[perm]
    outs = [torch.full((graphs[gi].n_vertices,), -7, dtype=torch.int32, device="cuda") for gi in qg]
    st = eat.eat_query_batch(graphs, qg, qsrc, qts, outs, stats=True)
    torch.cuda.synchronize()
    assert len(st) == 4096 and all(x["status"] == 0 for x in st)
    _say(f"batch done; checking every answer ({time.time() - t0:.0f}s)")
    n_thr = max(1, min(len(os.sched_getaffinity(0)), 16))
    checked = 0
    with ThreadPoolExecutor(n_thr) as ex:
        for gi, t in enumerate(graphs_tt):
            csa = oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices)
            ks = np.flatnonzero(qg == gi)
            for c0 in range(0, len(ks), 64):  # bounded host memory per chunk
                chunk = ks[c0:c0 + 64]
                exp = list(ex.map(lambda k: csa.query(int(qsrc[k]), int(qts[k])), chunk))
                for k, e in zip(chunk, exp):
                    got = outs[k].cpu().numpy()
                    assert np.array_equal(got, e), (int(k), gi, int(qsrc[k]), int(qts[k]))
                    assert st[k]["reached"] == int((e < oracle.INF).sum())
                    checked += 1
            csa.close()
            _say(f"  graph {gi} ({t.n_vertices} stops): {len(ks)} answers bit-exact ({time.time() - t0:.0f}s)")
    assert checked == 4096


@functools.lru_cache(maxsize=None)
def _mixed_city(i):
    """City i of the mixed batch (its generator seed) and 128 of its queries."""
    n = synth.MIXED_BATCH_SIZES[i]
    tt = synth.scaled_city(n, 401 + i)
    q = synth.queries(n, 512, 10401 + i)
    return tt, q.s[:128], q.ts[:128], eat.graph_from_timetable(tt)


@functools.lru_cache(maxsize=None)
def _mixed_city_scan(i):
    tt, s, ts, _ = _mixed_city(i)
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    n_thr = max(1, min(len(os.sched_getaffinity(0)), 16))
    with ThreadPoolExecutor(n_thr) as ex:
        exp = list(ex.map(lambda k: csa.query(int(s[k]), int(ts[k])), range(len(s))))
    csa.close()
    return exp


@pytest.mark.parametrize("fcap", [0, 64])
@pytest.mark.parametrize("th,city", [(384, 6), (256, 5)])
def test_small_work_groups_on_large_cities(th, city, fcap):
    """Four and six queries per CU (384 and 256 threads) on the mixed batch's
    200,000- and 100,000-stop cities, 128 queries in one launch, with default
    lists and with lists of 64 entries (most rounds then sweep the table in
    chunks): every answer equals the scan's."""
    tt, s, ts, g = _mixed_city(city)
    _say(f"{tt.n_vertices} stops, {th} threads, frontier_cap {fcap}")
    outs = [torch.full((tt.n_vertices,), -7, dtype=torch.int32, device="cuda") for _ in range(len(s))]
    st = eat.eat_query_batch([g], np.zeros(len(s), np.int32), s, ts, outs, stats=True,
                             options={"threads_per_query": th, "frontier_cap": fcap})
    torch.cuda.synchronize()
    assert all(x["status"] == 0 for x in st)
    if fcap:
        assert sum(x["sweep_rounds"] for x in st) > 0
    exp = _mixed_city_scan(city)
    for k in range(len(s)):
        assert np.array_equal(outs[k].cpu().numpy(), exp[k]), (k, int(s[k]), int(ts[k]))


@functools.lru_cache(maxsize=None)
def _lines_1500k():
    """1.5M stops served by 12,000 bus lines (about 23M connections): the stop
    bitmap (188 KB) does not fit the LDS, so slab-mode activity bits live in
    HBM.  Sources are stops with departures, leaving between 05:00 and 09:00
    (some queries reach over 100 stops: a 64-slot table overflows)."""
    tt = synth.transit_lines(1_500_000, 5, 12_000, (20, 40), (60, 300), (0, 30), (900, 1800), 703,
                             name="lines-1.5M")
    rng = np.random.default_rng(704)
    q = synth.Queries(s=rng.choice(np.unique(tt.u), 64).astype(np.int32),
                      ts=rng.integers(5 * 3600, 9 * 3600, 64).astype(np.int32), seed=704)
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    return tt, q, csa.query_many(q.s, q.ts)


def test_graph_beyond_the_lds_bitmap_limit():
    tt, q, exp = _lines_1500k()
    g = eat.graph_from_timetable(tt)
    V, Q = tt.n_vertices, len(q)
    _say(f"lines 1.5M: {tt.n_conn} connections, max reach {int((exp < oracle.INF).sum(1).max())}")
    slab = torch.full((Q, V), -7, dtype=torch.int32, device="cuda")
    for opts in (None, {"table_cap": -1}, {"table_cap": -1, "mode": eat.EAT_MODE_TOPOLOGY},
                 {"table_cap": 64}):
        slab.fill_(-7)
        st = eat.eat_query_batch([g], np.zeros(Q, np.int32), q.s, q.ts, [slab[i] for i in range(Q)],
                                 options=opts, stats=True)
        got = slab.cpu().numpy()
        bad = [i for i in range(Q) if not np.array_equal(got[i], exp[i])]
        assert not bad, (opts, bad[:5])
        assert all(x["status"] == 0 for x in st)
        if opts and opts.get("table_cap") == 64:
            assert sum(x["spilled"] for x in st) > 0  # table overflow fell back to HBM bits
    # single queries: the bits take a stream-ordered region of HBM
    for i in (0, 5, 9):
        out = torch.full((V,), -7, dtype=torch.int32, device="cuda")
        eat.eat_query(g, int(q.s[i]), int(q.ts[i]), out, options={"table_cap": -1})
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), exp[i])
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query(g, 0, 0, slab[0], options={"threads_per_query": 768})
    assert ei.value.status == eat.EAT_ERR_UNSUPPORTED
    # a serving session with slab-mode queries
    sess = eat.Session([g], pool_bytes=64 * V * 4, options={"table_cap": -1})
    slots = [sess.admit(0, int(q.s[i]), int(q.ts[i])) for i in range(16)]
    assert sess.step() == 16
    sess.sync()
    assert sorted(sess.poll()) == sorted(slots)
    for i, s_ in enumerate(slots):
        assert np.array_equal(sess.result(s_).cpu().numpy(), exp[i])
    sess.free()
    for i in range(0, Q, 16):
        assert _certify(tt, q.s[i], q.ts[i], exp[i]) == 0
