"""Serving sessions on the GPU: continuous batching over two resident graphs.
Every served answer must equal the same query run alone and the oracle,
bit-exact (tolerance 0)."""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, serve, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eat.lib()


@functools.lru_cache(maxsize=None)
def _two_graphs():
    tt1, _ = synth.workload("city-1k")
    tt2 = synth.scaled_city(5000, seed=402)
    return [tt1, tt2], [eat.graph_from_timetable(tt1), eat.graph_from_timetable(tt2)]


def _run(pool_bytes, rate, n, seed, n_streams=2):
    tts, graphs = _two_graphs()
    sess = eat.Session(graphs, pool_bytes=pool_bytes, n_streams=n_streams)
    reqs = serve.poisson_requests(rate, n, [g.n_vertices for g in graphs], seed=seed)
    got = {}

    def on_done(r, slot):
        got[r.id] = sess.result(slot).cpu().numpy()  # synchronous copy before the slot is released

    print(f"serving {n} requests at {rate} qps, pool {pool_bytes} B", flush=True)
    rep = serve.serve(sess, reqs, on_done=on_done, min_batch=16, max_delay_s=20e-6)
    sess.free()
    return tts, graphs, reqs, got, rep


def test_served_answers_equal_alone_and_oracle():
    tts, graphs, reqs, got, rep = _run(pool_bytes=0, rate=20_000, n=400, seed=5)
    assert rep.n == 400 and len(got) == 400
    csa = [oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices) for t in tts]
    for r in reqs:
        alone = graphs[r.graph].query(r.s, r.ts).cpu().numpy()
        assert np.array_equal(got[r.id], alone), r
        if r.id % 4 == 0:
            assert np.array_equal(got[r.id], csa[r.graph].query(r.s, r.ts)), r
    assert rep.steps >= 2


def test_tiny_pool_admits_as_slots_free_up():
    # room for about three 5k-stop slots: admission must wait and still finish all
    tts, graphs, reqs, got, rep = _run(pool_bytes=64 * 1024, rate=200_000, n=120, seed=6, n_streams=3)
    assert rep.n == 120 and rep.busy_waits > 0
    csa = [oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices) for t in tts]
    for r in reqs[::3]:
        assert np.array_equal(got[r.id], csa[r.graph].query(r.s, r.ts)), r


def test_session_api_errors_and_stats():
    tts, graphs = _two_graphs()
    sess = eat.Session(graphs, pool_bytes=1 << 20)
    with pytest.raises(eat.EatError):
        sess.admit(2, 0, 0)           # no such graph
    with pytest.raises(eat.EatError):
        sess.admit(0, 10_000, 0)      # source out of range
    slot = sess.admit(1, 7, 30_000)
    with pytest.raises(eat.EatError):
        sess.result(slot)             # not finished
    assert sess.step() == 1
    sess.sync()
    assert sess.poll() == [slot]
    st = sess.stats(slot)
    assert st["status"] == 0 and st["rounds"] >= 1 and st["elapsed_ns"] > 0
    exp = oracle.Csa(tts[1].u, tts[1].v, tts[1].t, tts[1].lam, tts[1].n_vertices).query(7, 30_000)
    assert np.array_equal(sess.result(slot).cpu().numpy(), exp)
    sess.release(slot)
    with pytest.raises(eat.EatError):
        sess.release(slot)            # already free
    # an admitted but never launched slot can be cancelled
    s2 = sess.admit(0, 3, 100)
    sess.release(s2)
    assert sess.step() == 0
    sess.free()


@functools.lru_cache(maxsize=None)
def _serve_graphs():
    """The three resident cities of the serving workload: 10k, 50k and 500k stops."""
    tts = synth.serving_cities()
    return tts, [eat.graph_from_timetable(t) for t in tts]


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_serving_on_the_10k_50k_500k_cities():
    """Poisson arrivals over the 10k/50k/500k-stop cities: at least 200 served
    answers per graph; on the 10k and 50k cities every one of them against
    the connection scan, on the 500k city every one of them certified (source,
    closure, witness; exact, O(|C|)); a sample also against the query alone."""
    import os
    import time
    from concurrent.futures import ThreadPoolExecutor

    t0 = time.time()
    tts, graphs = _serve_graphs()
    print(f"serving cities built in {time.time() - t0:.0f}s", flush=True)
    sess = eat.Session(graphs, pool_bytes=1 << 30, n_streams=2)
    reqs = serve.poisson_requests(20_000, 900, [g.n_vertices for g in graphs], seed=599)
    got = {}

    def on_done(r, slot):
        got[r.id] = sess.result(slot).cpu().numpy()

    rep = serve.serve(sess, reqs, on_done=on_done, min_batch=64, max_delay_s=50e-6)
    sess.free()
    assert rep.n == len(reqs) and len(got) == len(reqs)
    print(f"served {rep.n} in {rep.wall_s:.3f}s, p50 {rep.percentile_ms(50):.3f} ms, "
          f"p99 {rep.percentile_ms(99):.3f} ms", flush=True)
    n_thr = max(1, min(len(os.sched_getaffinity(0)), 16))
    with ThreadPoolExecutor(n_thr) as ex:
        for gi, t in enumerate(tts):
            mine = [r for r in reqs if r.graph == gi]
            assert len(mine) >= 200, (gi, len(mine))
            if t.n_vertices <= 100_000:
                csa = oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices)
                exp = list(ex.map(lambda r: csa.query(r.s, r.ts), mine))
                for r, e in zip(mine, exp):
                    assert np.array_equal(got[r.id], e), r
            else:
                rc = list(ex.map(lambda r: oracle.certify(t.u, t.v, t.t, t.lam, t.n_vertices, r.s, r.ts,
                                                          got[r.id]), mine))
                assert all(x == 0 for x in rc), [r for r, x in zip(mine, rc) if x][:3]
            for r in mine[::25]:
                alone = graphs[gi].query(r.s, r.ts).cpu().numpy()
                assert np.array_equal(got[r.id], alone), r
            print(f"  city {t.n_vertices}: {len(mine)} served answers exact ({time.time() - t0:.0f}s)",
                  flush=True)


def test_a_query_retires_before_its_step_launch_ends():
    """Each query of a step writes its own completion word: a query that ends
    in one round is reported by poll while a long query of the same launch is
    still running (tried a few times: it is a race the short query should win
    by hundreds of microseconds)."""
    import time
    tt, q = synth.workload("city-50k")
    g = eat.graph_from_timetable(tt)
    exp = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices).query_many(q.s, q.ts)
    heavy = int(np.argmax((exp < oracle.INF).sum(1)))
    late = int(tt.t.max()) + 1  # departs after the last connection: one round
    sess = eat.Session([g], pool_bytes=64 << 20, n_streams=2)
    early = False
    for attempt in range(5):
        sh = sess.admit(0, int(q.s[heavy]), int(q.ts[heavy]))
        sq = sess.admit(0, 3, late)
        assert sess.step() == 2
        order = []
        t_end = time.perf_counter() + 5.0
        while len(order) < 2 and time.perf_counter() < t_end:
            order += sess.poll()
        assert sorted(order) == sorted([sh, sq])
        assert np.array_equal(sess.result(sh).cpu().numpy(), exp[heavy])
        quick = sess.result(sq).cpu().numpy()
        assert quick[3] == late and (np.delete(quick, 3) == oracle.INF).all()
        sess.release(sh)
        sess.release(sq)
        if order[0] == sq:
            early = True
            break
    sess.free()
    assert early


def test_steps_are_refused_not_blocked_when_every_launch_is_in_flight():
    """With one launch slot, a second step while the first is in flight
    returns busy (nothing launched) instead of waiting."""
    tts, graphs = _two_graphs()
    sess = eat.Session(graphs, pool_bytes=8 << 20, n_streams=1)
    q = synth.queries(graphs[1].n_vertices, 64, 31)
    slots = [sess.admit(1, int(s), int(t)) for s, t in zip(q.s, q.ts)]
    assert sess.step() == 64
    extra = sess.admit(0, 1, 30_000)
    refused = sess.step()  # the 64-query launch is very likely still running
    sess.sync()
    if refused is None:
        assert sess.step() == 1
        sess.sync()
    done = set(sess.poll())
    assert done == set(slots) | {extra}
    exp = oracle.Csa(tts[1].u, tts[1].v, tts[1].t, tts[1].lam, tts[1].n_vertices)
    for s_, (src, t) in zip(slots[:8], zip(q.s, q.ts)):
        assert np.array_equal(sess.result(s_).cpu().numpy(), exp.query(int(src), int(t)))
    sess.free()


@pytest.mark.parametrize("pool_bytes,rate,n_streams", [(0, 50_000, 4), (64 * 1024, 400_000, 3)],
                         ids=["roomy-pool", "tiny-pool"])
def test_native_request_loop_serves_every_request_exactly(pool_bytes, rate, n_streams):
    """eat_session_serve runs the open-loop stream in native code: every
    request's copied answer equals the scan's, every latency is positive, and a
    pool with room for about three 5k-stop slots still serves them all."""
    tts, graphs = _two_graphs()
    sess = eat.Session(graphs, pool_bytes=pool_bytes, n_streams=n_streams)
    reqs = serve.poisson_requests(rate, 300, [g.n_vertices for g in graphs], seed=17)
    reqs = sorted(reqs, key=lambda r: r.arrival)
    gi = np.array([r.graph for r in reqs], np.int32)
    dst = [torch.full((graphs[int(g)].n_vertices,), -7, dtype=torch.int32, device="cuda") for g in gi]
    side = torch.cuda.Stream()
    print(f"native loop: {len(reqs)} requests at {rate} qps", flush=True)
    lat, rep = sess.serve(gi, [r.s for r in reqs], [r.ts for r in reqs], [r.arrival for r in reqs],
                          min_batch=16, max_delay_s=20e-6, copy_dst=dst, copy_stream=side)
    side.synchronize()
    assert rep["launched"] == len(reqs) and rep["steps"] >= 1
    assert np.all(lat > 0)
    csa = [oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices) for t in tts]
    for k, r in enumerate(reqs):
        assert np.array_equal(dst[k].cpu().numpy(), csa[r.graph].query(r.s, r.ts)), k
    # the session is empty again: a second stream of requests runs on it
    lat2, rep2 = sess.serve(gi[:20], [r.s for r in reqs[:20]], [r.ts for r in reqs[:20]],
                            [r.arrival for r in reqs[:20]])
    assert rep2["launched"] == 20 and np.all(lat2 > 0)
    sess.free()


def test_native_request_loop_checks_its_requests():
    tts, graphs = _two_graphs()
    sess = eat.Session(graphs, n_streams=2)
    V0 = graphs[0].n_vertices
    cases = [([0, 0], [1, 2], [0, 0], [0.001, 0.0]),   # arrivals out of order
             ([0, 2], [1, 2], [0, 0], [0.0, 0.001]),   # no graph 2
             ([0], [V0], [0], [0.0]),                  # source out of range
             ([0], [1], [-5], [0.0])]                  # negative departure time
    for g, s, t, a in cases:
        with pytest.raises(eat.EatError) as ei:
            sess.serve(g, s, t, a)
        assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    small = eat.Session(graphs, pool_bytes=8 * 1024, n_streams=1)  # no room for a 5k-stop slot
    with pytest.raises(eat.EatError) as ei:
        small.serve([1], [1], [0], [0.0])
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    small.free()
    slot = sess.admit(0, 1, 0)  # an admitted query left in the session
    with pytest.raises(eat.EatError) as ei:
        sess.serve([0], [1], [0], [0.0])
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    sess.release(slot)
    lat, rep = sess.serve([0], [1], [0], [0.0])
    assert rep["launched"] == 1
    sess.free()
