"""GPU parity of the paper's algorithm ladder (Algorithms 4-6, Cluster-AP,
edge, (virtual) warps) and of the ESDG baseline, through the C ABI: every
variant's answer element by element against the connection scan."""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import eat, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eat.lib()


@functools.lru_cache(maxsize=None)
def _city(name):
    tt, q = synth.workload(name)
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    return tt, q, csa.query_many(q.s, q.ts)


@functools.lru_cache(maxsize=None)
def _vgraph(name, cw=0, esdg=True):
    tt, _, _ = _city(name)
    return eat.VariantGraph(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, cluster_seconds=cw, esdg=esdg)


CASES = [(eat.EAT_VARIANT_CONNECTION, 0), (eat.EAT_VARIANT_CONNECTION_TYPE, 0),
         (eat.EAT_VARIANT_CONNECTION_TYPE_AP, 0), (eat.EAT_VARIANT_CLUSTER_AP, 0), (eat.EAT_VARIANT_EDGE, 0),
         (eat.EAT_VARIANT_WARPS, 1), (eat.EAT_VARIANT_WARPS, 4), (eat.EAT_VARIANT_WARPS, 32),
         (eat.EAT_VARIANT_WARPS, 64), (eat.EAT_VARIANT_ESDG, 0)]


@pytest.mark.parametrize("variant,ws", CASES, ids=[f"{eat.VARIANT_NAMES[v]}-{w}" for v, w in CASES])
def test_variant_equals_oracle_city_1k(variant, ws):
    tt, q, exp = _city("city-1k")
    g = _vgraph("city-1k")
    its = []
    for i in range(len(q)):
        for every in (1, 5):
            out, st = g.query(int(q.s[i]), int(q.ts[i]), variant, warp_size=ws, check_every=every, count=True)
            assert np.array_equal(out.cpu().numpy(), exp[i]), (i, every)
            assert st["status"] == 0
            its.append(st["iterations"])
    _say(f"{eat.VARIANT_NAMES[variant]} ws={ws}: mean iterations {np.mean(its):.1f}")


@pytest.mark.parametrize("cw", [1800, 900, 300])
def test_cluster_widths(cw):
    tt, q, exp = _city("city-1k")
    g = _vgraph("city-1k", cw, False)
    assert g.info["n_clusters"] == int(tt.t.max()) // cw + 1
    for i in range(len(q)):
        for v in (eat.EAT_VARIANT_CLUSTER_AP, eat.EAT_VARIANT_WARPS):
            out, _ = g.query(int(q.s[i]), int(q.ts[i]), v, warp_size=8)
            assert np.array_equal(out.cpu().numpy(), exp[i]), (i, v)


def test_variants_city_50k_sampled():
    tt, q, exp = _city("city-50k")
    g = _vgraph("city-50k")
    _say(f"city-50k variant graph: {g.info}")
    for i in (0, 77, 191):
        for v in range(7):
            out, st = g.query(int(q.s[i]), int(q.ts[i]), v, warp_size=16, check_every=4)
            assert np.array_equal(out.cpu().numpy(), exp[i]), (i, v)


def test_variant_errors():
    tt, _, _ = _city("city-1k")
    g = eat.VariantGraph(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)  # no ESDG
    with pytest.raises(eat.EatError) as ei:
        g.query(0, 0, eat.EAT_VARIANT_ESDG)
    assert ei.value.status == eat.EAT_ERR_UNSUPPORTED
    for bad in ({"variant": 9}, {"warp_size": 3}):
        with pytest.raises(eat.EatError):
            g.query(0, 0, bad.get("variant", 0), warp_size=bad.get("warp_size", 0))
    with pytest.raises(eat.EatError):
        g.query(tt.n_vertices, 0, 0)
    with pytest.raises(eat.EatError) as ei:
        g.query(int(tt.u[0]), 0, eat.EAT_VARIANT_CONNECTION, max_iterations=1)
    assert ei.value.status == eat.EAT_ERR_NOT_CONVERGED
