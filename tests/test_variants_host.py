"""Host parts of the paper's algorithm ladder, on the CPU (no GPU): the greedy
arithmetic-progression cover of Section I-A and the edge-scan-dependency
graph (ESDG) levels, against their definitions written out in Python on tiny
inputs, and the property the ESDG algorithm rests on: relaxing connections
level by level gives the EAT answer (checked against the oracle)."""
import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, synth

INF = oracle.INF


def _expand(cover):
    vals = []
    for first, last, diff in cover:
        if diff == 0:
            assert first == last
            vals.append(int(first))
        else:
            assert (last - first) % diff == 0
            vals.extend(range(int(first), int(last) + 1, int(diff)))
    return vals


def test_ap_cover_paper_example():
    # the progression 10, 15, .., 35 is the tuple (10, 35, 5) (Section I-A)
    assert eat.ap_cover([10, 15, 20, 25, 30, 35]).tolist() == [[10, 35, 5]]


def test_ap_cover_hand_case():
    # from 1 every difference covers two values: the smallest (1) wins; then
    # 4, 6, 8 with difference 2; 9 alone
    assert eat.ap_cover([1, 2, 4, 6, 8, 9]).tolist() == [[1, 2, 1], [4, 8, 2], [9, 9, 0]]
    # an hourly-like timetable with one extra departure: the progression first;
    # from 700 every choice covers one new value, and the longest (700, 900)
    # wins over 700 alone
    assert eat.ap_cover([300, 600, 700, 900, 1200]).tolist() == [[300, 1200, 300], [700, 900, 200]]


def test_ap_cover_properties_random():
    rng = np.random.default_rng(31)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        d = np.unique(rng.integers(0, 400, n)).astype(np.int32)
        cov = eat.ap_cover(d)
        vals = _expand(cov)
        # every value covered, nothing else: the expansion adds no departure
        assert set(vals) == set(d.tolist())
        # first terms increase, and each tuple starts at the smallest value not
        # covered by the tuples before it; from there no progression of values
        # of d covers more of the uncovered ones (the greedy rule)
        covered = set()
        for first, last, diff in cov:
            rest = sorted(set(d.tolist()) - covered)
            assert first == rest[0]
            mine = set(_expand([(first, last, diff)]))
            gain = len(mine - covered)
            s = set(d.tolist())
            for x in d[d > first]:
                dd = int(x - first)
                k, run = first, set()
                while k in s:
                    run.add(k)
                    k += dd
                assert len(run - covered) <= gain
            covered |= mine


def test_ap_cover_rejects_unsorted():
    with pytest.raises(eat.EatError):
        eat.ap_cover([5, 3])
    assert eat.ap_cover([]).shape == (0, 3)


def _brute_levels(u, v, t, lam):
    """ESDG of Section I-A from its definition: c -> c2 when c2 leaves c's head
    at or after c arrives and no connection of c2's edge leaving then arrives
    before c2; level = longest path from a connection without predecessors."""
    C = len(u)
    succ = [[] for _ in range(C)]
    for c in range(C):
        arr = int(t[c]) + int(lam[c])
        for c2 in range(C):
            if v[c] != u[c2] or t[c2] < arr:
                continue
            a2 = int(t[c2]) + int(lam[c2])
            if any(u[c3] == u[c2] and v[c3] == v[c2] and t[c3] >= arr and int(t[c3]) + int(lam[c3]) < a2
                   for c3 in range(C)):
                continue
            succ[c].append(c2)
    level = [0] * C
    for _ in range(C + 1):  # a DAG: C rounds settle every longest path
        for c in range(C):
            for c2 in succ[c]:
                level[c2] = max(level[c2], level[c] + 1)
    return level, sum(len(x) for x in succ)


def test_esdg_levels_equal_the_definition():
    rng = np.random.default_rng(32)
    for _ in range(300):
        tt = synth.random_tiny(rng, max_v=6, max_c=24)
        lv, nl, ne = eat.esdg_levels(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
        ref, ref_e = _brute_levels(tt.u, tt.v, tt.t, tt.lam)
        assert lv.tolist() == ref
        assert ne == ref_e
        assert nl == (max(ref) + 1 if len(ref) else 0)


def test_relaxing_level_by_level_gives_the_eat_answer():
    rng = np.random.default_rng(33)
    for _ in range(400):
        tt = synth.random_tiny(rng, max_v=7, max_c=30)
        lv, nl, _ = eat.esdg_levels(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
        s = int(rng.integers(0, tt.n_vertices))
        ts = int(rng.integers(0, 32))
        e = np.full(tt.n_vertices, INF, dtype=np.int64)
        e[s] = ts
        for level in range(nl):
            for c in np.flatnonzero(lv == level):  # one level: any order
                if e[tt.u[c]] <= tt.t[c] and tt.t[c] + tt.lam[c] < e[tt.v[c]]:
                    e[tt.v[c]] = tt.t[c] + tt.lam[c]
        exp = oracle.brute_states(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts)
        assert np.array_equal(e, exp)


def test_esdg_levels_on_a_city():
    tt, _ = synth.workload("city-1k")
    lv, nl, ne = eat.esdg_levels(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    assert nl > 1 and ne > 0
    # every dependency edge goes to a later departure, so the departure order
    # is a topological order: no connection has a level above its rank there
    assert lv.max() == nl - 1
