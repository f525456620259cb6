"""The entry point that allocates nothing (eat_query_batch_static) against the
allocating one (eat_query_batch) and the oracle, through the C ABI: two calls
in a row, the second with a smaller input, so a second call cannot lean on
what the first left in the shared scratch array."""
import functools

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eat.lib()


@functools.lru_cache(maxsize=None)
def _graphs():
    tt1, q1 = synth.workload("city-1k")
    tt2 = synth.scaled_city(20_000, seed=404)
    q2 = synth.queries(tt2.n_vertices, 200, 777)
    return (tt1, q1, eat.graph_from_timetable(tt1)), (tt2, q2, eat.graph_from_timetable(tt2))


def _both(graphs, qg, qs, qt):
    """Answers and statistics of both entry points on the same queries."""
    outs_a = [torch.full((graphs[gi].n_vertices,), -7, dtype=torch.int32, device="cuda") for gi in qg]
    outs_b = [torch.full((graphs[gi].n_vertices,), -9, dtype=torch.int32, device="cuda") for gi in qg]
    st_a = eat.eat_query_batch(graphs, qg, qs, qt, outs_a, stats=True)
    st_b = eat.eat_query_batch_static(graphs, qg, qs, qt, outs_b, stats=True)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs_a], st_a, [o.cpu().numpy() for o in outs_b], st_b


def test_static_batch_equals_the_allocating_batch_twice():
    (tt1, q1, g1), (tt2, q2, g2) = _graphs()
    c1 = oracle.Csa(tt1.u, tt1.v, tt1.t, tt1.lam, tt1.n_vertices)
    c2 = oracle.Csa(tt2.u, tt2.v, tt2.t, tt2.lam, tt2.n_vertices)
    # first call: two graphs, 216 queries interleaved
    qg = np.r_[np.zeros(len(q1), np.int32), np.ones(len(q2), np.int32)]
    qs = np.r_[q1.s, q2.s]
    qt = np.r_[q1.ts, q2.ts]
    perm = np.random.default_rng(3).permutation(len(qg))
    qg, qs, qt = qg[perm], qs[perm], qt[perm]
    print(f"static batch, call 1: {len(qg)} queries over 2 graphs", flush=True)
    a, st_a, b, st_b = _both([g1, g2], qg, qs, qt)
    for k in range(len(qg)):
        exp = (c1 if qg[k] == 0 else c2).query(int(qs[k]), int(qt[k]))
        assert np.array_equal(a[k], exp), k
        assert np.array_equal(b[k], exp), k
        assert st_b[k]["status"] == st_a[k]["status"] == 0
        assert st_b[k]["reached"] == st_a[k]["reached"] == int((exp < oracle.INF).sum())
    # second call: a smaller input, one graph, other queries
    print("static batch, call 2: 5 queries on one graph", flush=True)
    q3 = synth.queries(tt1.n_vertices, 5, 4242)
    a, st_a, b, st_b = _both([g1], np.zeros(5, np.int32), q3.s, q3.ts)
    for k in range(5):
        exp = c1.query(int(q3.s[k]), int(q3.ts[k]))
        assert np.array_equal(a[k], exp) and np.array_equal(b[k], exp), k
        assert st_b[k]["reached"] == st_a[k]["reached"]
    # without statistics, and with explicit options
    outs = [torch.full((tt1.n_vertices,), -5, dtype=torch.int32, device="cuda") for _ in range(5)]
    eat.eat_query_batch_static([g1], np.zeros(5, np.int32), q3.s, q3.ts, outs,
                               options={"threads_per_query": 512})
    torch.cuda.synchronize()
    for k in range(5):
        assert np.array_equal(outs[k].cpu().numpy(), c1.query(int(q3.s[k]), int(q3.ts[k])))


def test_static_batch_limits_and_errors():
    (tt1, q1, g1), _ = _graphs()
    out = torch.empty(tt1.n_vertices, dtype=torch.int32, device="cuda")
    n = 8193  # one more than the scratch array holds
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query_batch_static([g1], np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                                   [out] * n)
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query_batch_static([g1] * 65, np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.int32),
                                   [out])
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query_batch_static([g1], np.zeros(1, np.int32), np.array([tt1.n_vertices], np.int32),
                                   np.zeros(1, np.int32), [out])
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    # the round limit is reported like the allocating entry point does
    exp = oracle.Csa(tt1.u, tt1.v, tt1.t, tt1.lam, tt1.n_vertices).query_many(q1.s, q1.ts)
    i = int(np.argmax((exp < oracle.INF).sum(1)))
    with pytest.raises(eat.EatError) as ei:
        eat.eat_query_batch_static([g1], np.zeros(1, np.int32), q1.s[i:i + 1], q1.ts[i:i + 1], [out],
                                   options={"max_rounds": 2})
    assert ei.value.status == eat.EAT_ERR_NOT_CONVERGED
    # and a following call is clean again
    eat.eat_query_batch_static([g1], np.zeros(1, np.int32), q1.s[i:i + 1], q1.ts[i:i + 1], [out])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), exp[i])
