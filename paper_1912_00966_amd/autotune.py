"""Autotuner for batched earliest-arrival-time launches.

Runs a prepared batch under each candidate set of run options, times the
launches with HIP events on the launch stream, checks that every candidate
gives the same arrival arrays (the answer is unique, so any difference is a
bug), and returns the fastest options.  Results are cached in a JSON file keyed
by the graphs' shape, the batch size and the device name, so a later call
with the same key returns at once.

Knobs (all exact; they change only speed):
  threads_per_vertex  0 = wave claims, or 16/32 lanes per active stop
                      (virtual warps)
  threads_per_query   1024, or 768 / 512 (two queries per CU)
  time_window         arrival window of a round (seconds; -1 = none)
  types_per_lane      load-balanced expansion: connection types each lane keeps
                      in flight
  table_cap           0 = arrivals in the on-chip table (auto size), -1 = in
                      the result slab (HBM)
  headers             header grid or compact headers (hybrid layout)
  mode                frontier-driven rounds, or a topology sweep every round
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Optional, Sequence

import numpy as np

from . import eat

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "eat_autotune.json")


def candidates():
    for tpv, window in itertools.product((0, 16, 32), (3600, 7200, -1)):
        yield {"threads_per_vertex": tpv, "time_window": window, "mode": eat.EAT_MODE_FRONTIER}
    for threads, window in itertools.product((768, 512), (3600, 7200)):
        yield {"threads_per_query": threads, "time_window": window}
    yield {"threads_per_vertex": 0, "types_per_lane": 2, "mode": eat.EAT_MODE_FRONTIER}
    yield {"table_cap": -1}
    yield {"headers": eat.EAT_HEADERS_COMPACT}
    yield {"mode": eat.EAT_MODE_TOPOLOGY}


def cache_key(graphs: Sequence[eat.Graph], n_queries: int, streams: int = 1) -> str:
    import torch
    shape = [(g.info.n_vertices, g.info.n_types, g.info.n_headers, g.info.n_conn, g.info.layout)
             for g in graphs]
    return json.dumps({"graphs": shape, "queries": int(n_queries), "streams": int(streams),
                       "device": torch.cuda.get_device_name()}, sort_keys=True)


def tune(graphs: Sequence[eat.Graph], q_graph, q_src, q_ts, reps: int = 5,
         cache_path: Optional[str] = DEFAULT_CACHE, cands=None, verbose: bool = False,
         streams: int = 1):
    """Returns (best options dict, [(options, mean ms per batch), ...]).  With
    streams > 1, consecutive runs alternate over that many streams (one
    prepared batch each), as a throughput-oriented caller would issue them."""
    import torch

    key = cache_key(graphs, len(q_src), streams)
    if cache_path and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
        except (OSError, ValueError):
            cached = None
        if cached:
            return cached["best"], [(r["options"], r["ms"]) for r in cached["results"]]

    import time

    S = max(1, int(streams))
    outsets = [[torch.empty(graphs[int(gi)].n_vertices, dtype=torch.int32, device="cuda") for gi in q_graph]
               for _ in range(S)]
    strs = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    results = []
    reference = None
    for opts in (cands or candidates()):
        bs = [eat.Batch(graphs, q_graph, q_src, q_ts, o, options=opts) for o in outsets]
        for b, st in zip(bs, strs):
            b.run(st)
        torch.cuda.synchronize()
        for b, o in zip(bs, outsets):
            b.wait()
            got = [x.cpu().numpy() for x in o] if reference is None else [x.cpu().numpy() for x in o[::7]]
            if reference is None:
                reference = got
            elif not all(np.array_equal(a, r) for a, r in zip(got, reference[::7])):
                raise RuntimeError(f"autotune: options {opts} changed the answers")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps * S):
            bs[i % S].run(strs[i % S])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / (reps * S)
        for b in bs:
            b.free()
        results.append((dict(opts), ms))
        if verbose:
            print(f"[autotune] {opts} {ms:.4f} ms", flush=True)
    best = min(results, key=lambda r: r[1])[0]
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        try:
            data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = {"best": best, "results": [{"options": o, "ms": m} for o, m in results]}
        tmp = cache_path + ".tmp"
        json.dump(data, open(tmp, "w"), indent=1)
        os.replace(tmp, cache_path)
    return best, results
