"""Autotuner of batched earliest-arrival-time launches.

The tuning itself is native (eat_batch_tune in the library): it runs a batch
under each candidate set of run options, checks on the device that every
candidate gives the same arrival arrays (the answer is unique, so any
difference is a bug), times the candidates with HIP events, and records the
fastest for the device, the graphs' shapes and the batch size.  Batches
created afterwards without run options (``eat.Batch(..., options=None)``,
``eat_batch_create`` with NULL) use that record.  Setting the environment
variable EAT_TUNE_FILE keeps the records across processes.

Knobs the candidates cover (all exact; they change only speed):
  threads_per_query   1024, or 768 / 512 (two queries per CU)
  types_per_lane      connection types each lane keeps in flight: a wave has
                      64 x that many (type, cluster) lookups in flight
  threads_per_vertex  0 = type windows, or 16 / 32 lanes per active stop
                      (virtual warps: threads per edge)
  time_window         arrival window of a round (seconds; -1 = none)
  mode                frontier-driven rounds, or a topology sweep every round
  headers             header grid or compact headers (hybrid layout)
"""
from __future__ import annotations

from typing import Sequence

from . import eat


def tune(graphs: Sequence[eat.Graph], q_graph, q_src, q_ts, outs, reps: int = 3, streams: int = 1,
         stream=None, verbose: bool = False):
    """Returns (best options dict, [(options dict, mean ms per run), ...]); `outs`
    are the batch's result slabs (they hold its answers on return)."""
    best, results = eat.eat_batch_tune(graphs, q_graph, q_src, q_ts, outs, stream=stream, reps=reps,
                                       n_streams=streams)
    if verbose:
        for o, ms in results:
            print(f"[autotune] {o} {ms:.4f} ms", flush=True)
    return best, results
