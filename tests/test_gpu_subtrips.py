"""Sub-trip shortcuts (Section II-G) on the GPU: a 10,000-stop city served by
bus lines, with and without shortcuts, against the oracle's connection scan
on the original connections (bit-exact), and the rounds the shortcuts save."""
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
def _city():
    tt = synth.lines_city(10_000)
    q = synth.queries(tt.n_vertices, 256, 10601)
    exp = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices).query_many(q.s, q.ts)
    return tt, q, exp


def _batch(g, q, V, **opt):
    slab = torch.full((len(q), V), -7, dtype=torch.int32, device="cuda")
    st = eat.eat_query_batch([g], np.zeros(len(q), np.int32), q.s, q.ts, [slab[i] for i in range(len(q))],
                             options=opt or None, stats=True)
    return slab.cpu().numpy(), st


@pytest.mark.parametrize("rule", [None, 0, -1, 2])
def test_shortcuts_keep_every_answer_and_save_rounds(rule):
    tt, q, exp = _city()
    g = eat.graph_from_timetable(tt, subtrip_len=rule)
    print(f"lines city, sub-trip rule {rule}: {g.info.n_shortcuts} shortcuts "
          f"(r = {g.info.subtrip_len}), {g.info.n_conn} connections kept", flush=True)
    got, st = _batch(g, q, tt.n_vertices)
    bad = [i for i in range(len(q)) if not np.array_equal(got[i], exp[i])]
    assert not bad, bad[:10]
    assert all(x["status"] == 0 for x in st)
    rounds = float(np.mean([x["rounds"] for x in st]))
    if rule is None:
        assert g.info.n_shortcuts == 0
        _city.rounds_plain = rounds
    else:
        assert g.info.n_shortcuts > 0
        print(f"  mean rounds {rounds:.2f} against {getattr(_city, 'rounds_plain', float('nan')):.2f} without",
              flush=True)
        if hasattr(_city, "rounds_plain"):
            assert rounds < _city.rounds_plain
    # the same with the window off (the schedule of Section III-B) and with
    # virtual warps
    got2, _ = _batch(g, q, tt.n_vertices, time_window=-1, threads_per_vertex=16)
    assert np.array_equal(got2, exp)
