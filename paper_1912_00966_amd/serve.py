"""Request loop for serving earliest-arrival-time queries with continuous batching.

The loop drives a serving session (``eat.Session``): requests arrive over time,
are admitted as soon as a result slot of their graph's size is free in the
session's device pool, and are launched in steps -- one kernel launch over all
queries admitted since the previous step.  Steps go to the session's streams in
turn, so a step launched while earlier ones are still running shares the GPU with
them.  A finished query is reported at the next poll, its result handed to a
callback, and its slot released for the next request.

Batching policy: a step is launched when the GPU has no step in flight, when
``min_batch`` admitted queries are waiting, or when the oldest of them has waited
``max_delay_s``.

The session object only needs ``admit(graph, s, ts) -> slot | None``,
``step() -> int | None`` (None: every launch slot busy, nothing launched),
``poll() -> [slot]`` and ``release(slot)``; the tests drive the loop with a CPU
stand-in that computes nothing.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    id: int
    graph: int
    s: int
    ts: int
    arrival: float  # seconds after the start of the run


@dataclasses.dataclass
class ServeReport:
    n: int
    wall_s: float
    qps: float
    latency_s: np.ndarray  # per request, in request-id order
    steps: int
    mean_step_queries: float
    busy_waits: int  # admissions refused for lack of slot memory

    def percentile_ms(self, p: float) -> float:
        return float(np.percentile(self.latency_s, p) * 1e3) if self.n else float("nan")

    def as_dict(self) -> dict:
        return {"requests": self.n, "wall_s": round(self.wall_s, 4), "qps": round(self.qps, 1),
                "p50_ms": round(self.percentile_ms(50), 4), "p99_ms": round(self.percentile_ms(99), 4),
                "max_ms": round(float(self.latency_s.max() * 1e3), 4) if self.n else None,
                "steps": self.steps, "mean_step_queries": round(self.mean_step_queries, 2),
                "busy_waits": self.busy_waits}


def poisson_requests(rate_qps: float, n: int, graph_sizes: Sequence[int], seed: int) -> List[Request]:
    """n requests with exponential inter-arrival times at rate_qps; graph uniform
    among the graphs; source uniform over that graph's stops; ts uniform over the day."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_qps, size=n)
    t = np.cumsum(gaps) - gaps[0]
    g = rng.integers(0, len(graph_sizes), size=n)
    sizes = np.asarray(graph_sizes)
    s = (rng.random(n) * sizes[g]).astype(np.int64)
    ts = rng.integers(0, 86400, size=n)
    return [Request(i, int(g[i]), int(s[i]), int(ts[i]), float(t[i])) for i in range(n)]


def serve(session, requests: Sequence[Request],
          on_done: Optional[Callable[[Request, int], None]] = None,
          min_batch: int = 64, max_delay_s: float = 50e-6,
          clock: Callable[[], float] = time.perf_counter, stuck_s: float = 1.0) -> ServeReport:
    """Runs the open-loop request stream to completion; returns latencies.
    Raises RuntimeError when a request cannot be admitted for stuck_s seconds
    while nothing is in flight (its result slot can never fit the pool)."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    n = len(reqs)
    latency = np.zeros(n)
    waiting: deque = deque()        # arrived, not admitted
    pending: deque = deque()        # admitted, not launched: (slot, admit time)
    inflight = {}                   # slot -> request
    steps_open: deque = deque()     # slot sets of launched steps, oldest first
    n_steps = 0
    launched = 0
    busy = 0
    done = 0
    i = 0
    t0 = clock()
    blocked_since = None  # when admission began failing with nothing in flight
    while done < n:
        now = clock() - t0
        while i < n and reqs[i].arrival <= now:
            waiting.append(reqs[i])
            i += 1
        # admission: first come, first served, while slot memory lasts
        while waiting:
            r = waiting[0]
            slot = session.admit(r.graph, r.s, r.ts)
            if slot is None:
                busy += 1
                if inflight:
                    blocked_since = None
                elif blocked_since is None:
                    blocked_since = now
                elif now - blocked_since > stuck_s:
                    raise RuntimeError(f"request {r.id} cannot be admitted with nothing in flight: "
                                       "its result slot does not fit the session's pool")
                break
            blocked_since = None
            waiting.popleft()
            inflight[slot] = r
            pending.append((slot, now))
        # launch policy (a step refused because every launch slot is busy is
        # retried on a later pass, after completions)
        if pending and (not steps_open or len(pending) >= min_batch or now - pending[0][1] >= max_delay_s):
            k = session.step()
            if k:
                steps_open.append({s for s, _ in list(pending)[:k]})
                for _ in range(k):
                    pending.popleft()
                n_steps += 1
                launched += k
        # completions
        finished = session.poll()
        if finished:
            t_done = clock() - t0
            for slot in finished:
                r = inflight.pop(slot)
                latency[r.id] = t_done - r.arrival
                if on_done is not None:
                    on_done(r, slot)
                session.release(slot)
                done += 1
                for open_set in steps_open:
                    if slot in open_set:
                        open_set.discard(slot)
                        break
            while steps_open and not steps_open[0]:
                steps_open.popleft()
        elif not inflight and not waiting and i < n:
            # idle until the next arrival
            gap = reqs[i].arrival - (clock() - t0)
            if gap > 200e-6:
                time.sleep(gap - 100e-6)
    wall = clock() - t0
    span = wall - (reqs[0].arrival if n else 0.0)
    ordered = np.zeros(n)
    for k, r in enumerate(reqs):
        ordered[r.id] = latency[r.id]
    return ServeReport(n=n, wall_s=wall, qps=n / span if span > 0 else float("nan"),
                       latency_s=ordered, steps=n_steps,
                       mean_step_queries=launched / n_steps if n_steps else 0.0, busy_waits=busy)
