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
