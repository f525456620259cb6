"""Pins for the CPU oracle: the connection scan (Algorithm 1) is checked against
answers that do not come from it -- brute force from the definition of the EAT
problem (Section I), Dijkstra on the time-expanded and time-dependent models,
hand-derived cases, the certificate, and invariants of the problem."""
import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import synth

INF = oracle.INF


def _run_all(tt, s, ts):
    args = (tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts)
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices).query(s, ts)
    return csa, args


# ---------------------------------------------------------------- hand cases

def _tt(rows, nv):
    a = np.array(rows, dtype=np.int32).reshape(-1, 4)
    return synth.Timetable("hand", nv, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(),
                           a[:, 3].copy(), -1, -1, -1)


def test_hand_chain_with_wait_and_missed_connection():
    # 0 -(t=10,lam=5)-> 1 at 15; 1 -(t=14)-> 2 is missed (departs before 15);
    # 1 -(t=20,lam=3)-> 2 at 23; 2 -(t=23,lam=1)-> 3 at 24 (boarding at the
    # arrival second is allowed: e[u] <= t, Algorithm 1).
    tt = _tt([[0, 1, 10, 5], [1, 2, 14, 2], [1, 2, 20, 3], [2, 3, 23, 1]], 5)
    csa, args = _run_all(tt, 0, 10)
    assert csa.tolist() == [10, 15, 23, 24, INF]
    # leaving one second later misses the first connection entirely
    csa2, _ = _run_all(tt, 0, 11)
    assert csa2.tolist() == [11, INF, INF, INF, INF]


def test_hand_faster_later_connection_wins():
    # a slow early trip (arrive 100) and a fast later one (arrive 50)
    tt = _tt([[0, 1, 0, 100], [0, 1, 40, 10], [0, 1, 60, 1]], 2)
    csa, _ = _run_all(tt, 0, 0)
    assert csa.tolist() == [0, 50]
    csa, _ = _run_all(tt, 0, 41)
    assert csa.tolist() == [41, 61]


def test_hand_cycle_back_to_source_keeps_ts():
    tt = _tt([[0, 1, 5, 1], [1, 0, 6, 1], [0, 2, 7, 1]], 3)
    csa, _ = _run_all(tt, 0, 5)
    # returning to 0 at 7 does not change arr[0]; 0 -> 2 boards at 7 from ts=5
    assert csa.tolist() == [5, 6, 8]


def test_hand_two_hop_beats_direct():
    tt = _tt([[0, 2, 0, 100], [0, 1, 0, 10], [1, 2, 10, 10]], 3)
    csa, _ = _run_all(tt, 0, 0)
    assert csa.tolist() == [0, 10, 20]


# ------------------------------------------------------------ brute force pins

def test_csa_equals_brute_force_and_dijkstras_on_tiny_graphs():
    rng = np.random.default_rng(12345)
    n_checked = 0
    for _ in range(6000):
        tt = synth.random_tiny(rng)
        s = int(rng.integers(0, tt.n_vertices))
        ts = int(rng.integers(0, 32))
        csa, args = _run_all(tt, s, ts)
        st = oracle.brute_states(*args)
        assert np.array_equal(csa, st), (tt.u, tt.v, tt.t, tt.lam, s, ts)
        try:
            bp = oracle.brute_paths(*args, max_paths=200_000)
            assert np.array_equal(csa, bp)
        except oracle.OracleError:
            pass  # too many paths for the enumeration; the state closure still checked it
        assert np.array_equal(csa, oracle.te_dijkstra(*args))
        assert np.array_equal(csa, oracle.td_dijkstra(*args))
        assert oracle.certify(*args, csa) == 0
        n_checked += 1
    assert n_checked == 6000


def test_csa_equals_brute_states_on_denser_small_graphs():
    rng = np.random.default_rng(777)
    for _ in range(400):
        tt = synth.random_tiny(rng, max_v=12, max_c=200, max_t=100, max_lam=20)
        s = int(rng.integers(0, tt.n_vertices))
        ts = int(rng.integers(0, 60))
        csa, args = _run_all(tt, s, ts)
        assert np.array_equal(csa, oracle.brute_states(*args))
        assert np.array_equal(csa, oracle.te_dijkstra(*args))


def test_dijkstras_agree_with_csa_on_1k_city():
    tt, q = synth.workload("city-1k")
    c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    for s, ts in zip(q.s, q.ts):
        ref = c.query(s, ts)
        args = (tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts)
        assert np.array_equal(ref, oracle.td_dijkstra(*args))
        assert np.array_equal(ref, oracle.te_dijkstra(*args))
        assert oracle.certify(*args, ref) == 0


# ------------------------------------------------------------------ certificate

def test_certificate_rejects_mutated_answers():
    tt, q = synth.workload("city-1k")
    c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    rng = np.random.default_rng(5)
    n_mut = 0
    for s, ts in zip(q.s, q.ts):
        ref = c.query(s, ts)
        args = (tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts)
        assert oracle.certify(*args, ref) == 0
        finite = np.flatnonzero((ref < INF) & (np.arange(len(ref)) != s))
        unreached = np.flatnonzero(ref == INF)
        muts = []
        if len(finite):
            x = int(rng.choice(finite))
            for delta in (-1, +1):
                m = ref.copy(); m[x] += delta; muts.append(m)
            m = ref.copy(); m[x] = INF; muts.append(m)
        if len(unreached):
            m = ref.copy(); m[int(rng.choice(unreached))] = 86400 * 3; muts.append(m)
        m = ref.copy(); m[s] = ts + 1; muts.append(m)
        for m in muts:
            assert oracle.certify(*args, m) != 0
            n_mut += 1
    assert n_mut > 40


# ------------------------------------------------------------------ invariants

def test_invariants_on_1k_city():
    tt, q = synth.workload("city-1k")
    c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    u, v, t, lam = tt.u, tt.v, tt.t, tt.lam
    for s, ts in zip(q.s, q.ts):
        a = c.query(s, ts)
        assert a[s] == ts
        assert (a >= ts).all()
        board = a[u] <= t
        assert (a[v[board]] <= (t + lam)[board]).all()
        # FIFO: leaving later never arrives earlier
        later = c.query(s, min(ts + 1800, 2**31 - 2))
        assert (later >= a).all()
    # departing after the last departure reaches nothing but the source
    late = c.query(0, int(t.max()) + 1)
    assert late[0] == int(t.max()) + 1 and (late[1:] == INF).all()


def test_duplicates_and_self_loops_do_not_change_the_answer():
    tt, q = synth.workload("city-1k")
    rng = np.random.default_rng(9)
    pick = rng.choice(tt.n_conn, size=5000, replace=False)
    loops = rng.choice(tt.n_vertices, size=300)
    u = np.concatenate([tt.u, tt.u[pick], loops]).astype(np.int32)
    v = np.concatenate([tt.v, tt.v[pick], loops]).astype(np.int32)
    t = np.concatenate([tt.t, tt.t[pick], rng.integers(0, 86400, 300)]).astype(np.int32)
    lam = np.concatenate([tt.lam, tt.lam[pick], rng.integers(1, 100, 300)]).astype(np.int32)
    a = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    b = oracle.Csa(u, v, t, lam, tt.n_vertices)
    for s, ts in zip(q.s, q.ts):
        assert np.array_equal(a.query(s, ts), b.query(s, ts))


def test_invalid_inputs_are_rejected():
    ok = dict(u=[0], v=[1], t=[0], lam=[1])
    assert oracle.validate(**ok, nv=2)
    assert not oracle.validate(u=[0], v=[1], t=[0], lam=[0], nv=2)       # lam < 1
    assert not oracle.validate(u=[0], v=[1], t=[-1], lam=[1], nv=2)      # t < 0
    assert not oracle.validate(u=[0], v=[2], t=[0], lam=[1], nv=2)       # v out of range
    assert not oracle.validate(u=[0], v=[1], t=[2**31 - 2], lam=[1], nv=2)  # t+lam = INF
    with pytest.raises(oracle.OracleError):
        oracle.Csa([0], [1], [0], [0], 2)


def test_next_departure_is_the_minimum_at_or_after_x():
    d = [300, 10, 200, 10, 50]
    assert oracle.next_departure(d, 0) == 10
    assert oracle.next_departure(d, 10) == 10
    assert oracle.next_departure(d, 11) == 50
    assert oracle.next_departure(d, 201) == 300
    assert oracle.next_departure(d, 301) == INF
    assert oracle.next_departure([], 0) == INF


def test_next_departure_equals_a_sorted_search():
    """min{t >= x} (Section II-B) equals numpy's left-sided search in the
    sorted departures, on random departure sets in random order."""
    rng = np.random.default_rng(21)
    for _ in range(300):
        n = int(rng.integers(0, 40))
        d = rng.integers(0, 5000, size=n).astype(np.int32)
        srt = np.sort(d)
        for x in rng.integers(-5, 5100, size=25):
            x = max(int(x), 0)
            pos = int(np.searchsorted(srt, x, side="left"))
            want = int(srt[pos]) if pos < n else INF
            assert oracle.next_departure(d, x) == want, (d, x)


def test_csa_scan_order_over_the_whole_time_range():
    """Departure times spread over the full int32 range (both 16-bit digits of
    the scan's ordering vary): the scan still equals the time-dependent
    Dijkstra and the state closure."""
    rng = np.random.default_rng(31)
    for _ in range(200):
        nv = int(rng.integers(2, 12))
        n = int(rng.integers(1, 120))
        u = rng.integers(0, nv, size=n).astype(np.int32)
        v = rng.integers(0, nv, size=n).astype(np.int32)
        # a few anchor times spread over [0, 2^31 - 2^20) plus small offsets:
        # many equal high digits with different low digits, and the reverse
        anchors = rng.integers(0, 2**31 - 2**20, size=4)
        t = (anchors[rng.integers(0, 4, size=n)] + rng.integers(0, 3 * 65536, size=n)).astype(np.int32)
        lam = rng.integers(1, 70000, size=n).astype(np.int32)
        tt = synth.Timetable("wide", nv, u, v, t, lam, -1, -1, -1)
        s = int(rng.integers(0, nv))
        ts = int(rng.choice(t)) - int(rng.integers(0, 2))
        ts = max(ts, 0)
        csa, args = _run_all(tt, s, ts)
        assert np.array_equal(csa, oracle.td_dijkstra(*args)), (s, ts)
        assert np.array_equal(csa, oracle.brute_states(*args)), (s, ts)
