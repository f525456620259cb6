"""Sub-trip shortcuts (Section II-G) on the host: the library's shortcut
connections against the rule of Sections II-G and IV-B written out here from
the paper, the preprocessed layout holding exactly the input plus those
shortcuts, invalid trips rejected, and -- pinned by the oracle -- the
shortcuts never changing an earliest arrival time."""
import math

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, synth
from test_layout_host import _expand, _reference_types


def _round(x):
    return int(math.floor(x + 0.5))  # halves round up


def paper_shortcuts(tt, rule):
    """Shortcut connections of every trip: each trip, in departure order, is cut
    into consecutive sub-trips of r connections (the last one takes the rest);
    a sub-trip c_i..c_j with i < j adds (v_i, v_{j+1}, t_i, t_j + lam_j - t_i).
    rule: r >= 1 fixed, -1 = round(sqrt(k)) per trip of k connections,
    0 = round(sqrt(mean trip length))."""
    on = np.flatnonzero(tt.trip >= 0)
    order = on[np.lexsort((tt.t[on], tt.trip[on]))]
    trips = np.split(order, np.flatnonzero(np.diff(tt.trip[order])) + 1) if len(order) else []
    if rule == 0:
        rule = max(1, _round(math.sqrt(len(order) / len(trips))))
    out = []
    for tr in trips:
        k = len(tr)
        r = max(1, _round(math.sqrt(k))) if rule == -1 else rule
        for b in range(0, k, r):
            e = min(k, b + r) - 1
            if e > b:
                ci, cj = tr[b], tr[e]
                out.append((int(tt.u[ci]), int(tt.v[cj]), int(tt.t[ci]), int(tt.t[cj] + tt.lam[cj] - tt.t[ci])))
    return out


def _with(tt, extra):
    if not extra:
        return tt
    a = np.array(extra, dtype=np.int64)
    return synth.Timetable(tt.name, tt.n_vertices, np.r_[tt.u, a[:, 0]].astype(np.int32),
                           np.r_[tt.v, a[:, 1]].astype(np.int32), np.r_[tt.t, a[:, 2]].astype(np.int32),
                           np.r_[tt.lam, a[:, 3]].astype(np.int32), -1, -1, -1)


def _layout_types(lay, nv):
    view = lay.view()
    got = _expand(view)
    ty, vt = view["ty"], view["vt"]
    seen = {}
    for uu in range(nv):
        for j in range(vt[uu, 0], vt[uu, 0] + vt[uu, 1]):
            seen[(uu, int(ty[j, 0]), int(ty[j, 1]))] = got[j]
    return seen


def _hand_trip():
    # one vehicle: stops 0 -> 1 -> 2 -> 3 -> 4 -> 5, leaving every 100 s, 50 s per
    # segment, plus a connection on no trip
    u = np.array([0, 1, 2, 3, 4, 7], np.int32)
    v = np.array([1, 2, 3, 4, 5, 8], np.int32)
    t = np.array([100, 200, 300, 400, 500, 50], np.int32)
    lam = np.array([50, 50, 50, 50, 50, 9], np.int32)
    trip = np.array([3, 3, 3, 3, 3, -1], np.int32)
    perm = np.array([4, 0, 5, 2, 1, 3])  # input order carries no meaning
    return synth.Timetable("hand", 9, u[perm], v[perm], t[perm], lam[perm], -1, -1, -1, trip=trip[perm])


@pytest.mark.parametrize("rule,expected", [
    (2, [(0, 2, 100, 150), (2, 4, 300, 150)]),
    (3, [(0, 3, 100, 250), (3, 5, 400, 150)]),
    (5, [(0, 5, 100, 450)]),
    (10, [(0, 5, 100, 450)]),
    (1, []),
    (-1, [(0, 2, 100, 150), (2, 4, 300, 150)]),  # round(sqrt(5)) = 2
    (0, [(0, 2, 100, 150), (2, 4, 300, 150)]),   # one trip of 5: the same
])
def test_hand_trip_shortcuts(rule, expected):
    tt = _hand_trip()
    assert paper_shortcuts(tt, rule) == expected
    lay = eat.eat_layout_build_trips(tt.u, tt.v, tt.t, tt.lam, tt.trip, tt.n_vertices, subtrip_len=rule)
    info = lay.info()
    assert info.n_trips == 1 and info.n_shortcuts == len(expected)
    assert _layout_types(lay, tt.n_vertices) == _reference_types(_with(tt, expected))


def test_invalid_trips_are_rejected():
    tt = _hand_trip()
    base = dict(u=tt.u, v=tt.v, t=tt.t, lam=tt.lam, n_vertices=tt.n_vertices)
    # a trip whose next connection leaves from another stop
    bad = tt.u.copy()
    bad[np.flatnonzero((tt.u == 2) & (tt.trip == 3))[0]] = 6
    with pytest.raises(eat.EatError) as ei:
        eat.eat_layout_build_trips(**dict(base, u=bad), trip=tt.trip)
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    # a trip whose next connection leaves before the vehicle arrives
    lam = tt.lam.copy()
    lam[np.flatnonzero((tt.u == 1) & (tt.trip == 3))[0]] = 101
    with pytest.raises(eat.EatError) as ei:
        eat.eat_layout_build_trips(**dict(base, lam=lam), trip=tt.trip)
    assert ei.value.status == eat.EAT_ERR_INVALID_ARGUMENT
    with pytest.raises(eat.EatError):
        eat.eat_layout_build_trips(**base, trip=tt.trip, subtrip_len=-2)
    # the sub-trip length belongs to the trip-aware builds only
    o = eat.BuildOptions()
    o.subtrip_len = 2
    h = eat._vp()
    u, v, t, l = (np.ascontiguousarray(x, np.int32) for x in (tt.u, tt.v, tt.t, tt.lam))
    st = eat.lib().eat_layout_build(eat._ptr32(u), eat._ptr32(v), eat._ptr32(t), eat._ptr32(l), len(u),
                                    tt.n_vertices, eat.ctypes.byref(o), eat.ctypes.byref(h))
    assert st == eat.EAT_ERR_INVALID_ARGUMENT
    # no trip at all: nothing added
    lay = eat.eat_layout_build_trips(**base, trip=np.full(len(tt.u), -1, np.int32))
    assert lay.info().n_shortcuts == 0 and lay.info().n_trips == 0


@pytest.mark.parametrize("rule", [0, -1, 3])
def test_shortcuts_follow_the_rule_and_keep_every_answer(rule):
    """A 2,000-stop city served by bus lines: the layout holds exactly the
    input plus the shortcuts of the rule, and the oracle's answers with the
    shortcuts equal its answers without them."""
    tt = synth.lines_city(2_000, seed=611)
    sc = paper_shortcuts(tt, rule)
    lay = eat.eat_layout_build_trips(tt.u, tt.v, tt.t, tt.lam, tt.trip, tt.n_vertices, subtrip_len=rule)
    info = lay.info()
    assert info.n_trips == len(np.unique(tt.trip[tt.trip >= 0]))
    assert info.n_shortcuts == len(sc) > 0
    if rule == 0:
        k = np.bincount(tt.trip[tt.trip >= 0])
        assert info.subtrip_len == max(1, _round(math.sqrt(k[k > 0].mean())))
    aug = _with(tt, sc)
    assert _layout_types(lay, tt.n_vertices) == _reference_types(aug)
    plain = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    short = oracle.Csa(aug.u, aug.v, aug.t, aug.lam, aug.n_vertices)
    q = synth.queries(tt.n_vertices, 40, 612)
    for s, ts in zip(q.s, q.ts):
        assert np.array_equal(plain.query(s, ts), short.query(s, ts)), (s, ts)
