"""Request-loop policy of the serving driver, on the CPU, with a stand-in for
the GPU session that computes nothing (it only reports slots as finished a few
polls after their launch)."""
import numpy as np

from paper_1912_00966_amd import serve


class FakeSession:
    def __init__(self, capacity, polls_to_finish=3):
        self.capacity = capacity
        self.polls_to_finish = polls_to_finish
        self.used = set()
        self.free = []
        self.next = 0
        self.admitted = []
        self.running = []  # (finish at poll number, slot)
        self.polls = 0
        self.max_used = 0
        self.launches = []
        self.order = []

    def admit(self, g, s, ts):
        if len(self.used) >= self.capacity:
            return None
        slot = self.free.pop() if self.free else self.next
        if slot == self.next:
            self.next += 1
        self.used.add(slot)
        self.max_used = max(self.max_used, len(self.used))
        self.admitted.append(slot)
        self.order.append((g, s, ts))
        return slot

    def step(self):
        k = len(self.admitted)
        for slot in self.admitted:
            self.running.append((self.polls + self.polls_to_finish, slot))
        self.launches.append(k)
        self.admitted = []
        return k

    def poll(self):
        self.polls += 1
        done = [s for t, s in self.running if t <= self.polls]
        self.running = [(t, s) for t, s in self.running if t > self.polls]
        return done

    def release(self, slot):
        assert slot in self.used
        self.used.remove(slot)
        self.free.append(slot)


class TickClock:
    def __init__(self, dt):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


def test_every_request_completes_once_and_in_arrival_order_of_admission():
    reqs = serve.poisson_requests(10_000, 500, [100, 200], seed=1)
    fake = FakeSession(capacity=32)
    seen = []
    rep = serve.serve(fake, reqs, on_done=lambda r, slot: seen.append(r.id), clock=TickClock(20e-6))
    assert sorted(seen) == list(range(500))
    assert rep.n == 500 and (rep.latency_s > 0).all()
    assert fake.max_used <= 32
    assert not fake.used  # all slots released
    # admission is first come, first served
    by_arrival = sorted(reqs, key=lambda r: r.arrival)
    assert fake.order == [(r.graph, r.s, r.ts) for r in by_arrival]
    assert sum(fake.launches) == 500


def test_full_pool_makes_requests_wait_not_fail():
    reqs = serve.poisson_requests(1e6, 200, [10], seed=2)  # all arrive almost at once
    fake = FakeSession(capacity=4)
    rep = serve.serve(fake, reqs, clock=TickClock(5e-6))
    assert rep.n == 200 and rep.busy_waits > 0
    assert fake.max_used <= 4
    assert max(fake.launches) <= 4


def test_batching_policy_groups_waiting_queries():
    # a burst arrives while a step is in flight: the next step takes many at once
    reqs = serve.poisson_requests(5e6, 300, [10], seed=3)
    fake = FakeSession(capacity=1000, polls_to_finish=20)
    rep = serve.serve(fake, reqs, min_batch=64, max_delay_s=1.0, clock=TickClock(1e-6))
    assert rep.n == 300
    assert max(fake.launches) >= 64
    assert rep.steps < 300


def test_poisson_stream_is_seeded_and_well_formed():
    a = serve.poisson_requests(2000, 1000, [50, 80], seed=9)
    b = serve.poisson_requests(2000, 1000, [50, 80], seed=9)
    assert [(r.graph, r.s, r.ts, r.arrival) for r in a] == [(r.graph, r.s, r.ts, r.arrival) for r in b]
    arr = np.array([r.arrival for r in a])
    assert arr[0] == 0 and (np.diff(arr) >= 0).all()
    assert 0.35 < arr[-1] < 0.65  # ~1000 / 2000 s
    for r in a:
        assert 0 <= r.s < (50, 80)[r.graph] and 0 <= r.ts < 86400


class BusySession(FakeSession):
    """A session with two launch slots: a step while both are in flight is
    refused (None), as eat_session_step's EAT_ERR_BUSY."""

    def __init__(self, capacity, polls_to_finish=5, launch_slots=2):
        super().__init__(capacity, polls_to_finish)
        self.launch_slots = launch_slots
        self.refused = 0

    def step(self):
        in_flight = len({t for t, _ in self.running})
        if in_flight >= self.launch_slots:
            self.refused += 1
            return None
        return super().step()


def test_refused_steps_are_retried_and_every_request_completes():
    reqs = serve.poisson_requests(2e6, 400, [10, 20], seed=4)
    fake = BusySession(capacity=64)
    seen = []
    rep = serve.serve(fake, reqs, on_done=lambda r, slot: seen.append(r.id), min_batch=1, max_delay_s=0.0,
                      clock=TickClock(1e-6))
    assert sorted(seen) == list(range(400))
    assert fake.refused > 0
    assert sum(fake.launches) == 400 and rep.steps == len(fake.launches)
    assert not fake.used


def test_a_request_that_can_never_be_admitted_raises():
    class NeverFits(FakeSession):
        def admit(self, g, s, ts):
            return None if g == 1 else super().admit(g, s, ts)

    reqs = [serve.Request(id=0, graph=0, s=1, ts=0, arrival=0.0),
            serve.Request(id=1, graph=1, s=1, ts=0, arrival=0.0)]
    ticks = iter(range(10**6))
    try:
        serve.serve(NeverFits(capacity=4), reqs, clock=lambda: next(ticks) * 1e-3, stuck_s=0.05)
    except RuntimeError as e:
        assert "request 1" in str(e)
    else:
        raise AssertionError("serve() returned although request 1 can never be admitted")
