"""The serving loop's admission, batching and budget logic, driven by a fake
executor on the CPU (no GPU, deterministic simulated durations)."""
import math

import pytest

from paper_2604_26745_amd import serve


class FakeExecutor:
    """Each launch finishes after `cost[size] * batch` simulated seconds."""

    def __init__(self, cost, bytes_per_slice):
        self.cost, self.bps = cost, bytes_per_slice
        self.now = 0.0
        self.launches = []

    def workspace_bytes(self, size, b):
        return self.bps[size] * b

    def launch(self, size, reqs, slot):
        end = self.now + self.cost[size] * len(reqs)
        self.launches.append((self.now, size, [r.rid for r in reqs], slot))
        return end

    def done(self, handle):
        return self.now >= handle

    def warm(self, batch_sizes):
        pass


def drive(server, ex, reqs, dt=1e-3, horizon=100.0):
    i, done, n = 0, 0, len(reqs)
    t = 0.0
    while done < n:
        assert t < horizon
        ex.now = t
        while i < n and reqs[i].arrival <= t:
            server.queue.append(reqs[i])
            i += 1
        done += server.poll(t)
        server.admit(t)
        t += dt
    return t


def R(k, t, size):
    return serve.Request(k, t, size, 0)


def test_same_size_requests_are_batched_in_arrival_order():
    ex = FakeExecutor({64: 0.01, 128: 0.04}, {64: 1, 128: 4})
    srv = serve.Server(ex, hbm_budget=1e9, n_slots=1, max_batch=8)
    # a long request occupies the only slot while 6 more queue up
    reqs = [R(0, 0.0, 128)] + [R(k, 0.001 * k, 64 if k % 2 else 128) for k in range(1, 7)]
    drive(srv, ex, reqs)
    batches = [(l[1], l[2]) for l in ex.launches]
    # the oldest queued request decides the size of the next batch, which
    # takes the largest power-of-two count of queued requests of that size in
    # arrival order
    assert batches == [(128, [0]), (64, [1, 3]), (128, [2, 4]), (64, [5]), (128, [6])]
    assert all(not math.isnan(r.done) for r in reqs)


def test_budget_limits_in_flight_bytes():
    ex = FakeExecutor({64: 0.05}, {64: 10})
    srv = serve.Server(ex, hbm_budget=25, n_slots=8, max_batch=1)
    reqs = [R(k, 0.0, 64) for k in range(6)]
    drive(srv, ex, reqs)
    assert srv.max_in_flight_bytes <= 25
    # two at a time fit the budget: three waves
    starts = sorted(set(round(l[0], 3) for l in ex.launches))
    assert len(starts) == 3


def test_oversized_batch_admitted_when_idle():
    ex = FakeExecutor({256: 0.01}, {256: 100})
    srv = serve.Server(ex, hbm_budget=50, n_slots=2, max_batch=2)
    reqs = [R(0, 0.0, 256)]
    drive(srv, ex, reqs)
    assert len(ex.launches) == 1 and srv.max_in_flight_bytes == 100


def test_slots_refill_as_work_completes():
    ex = FakeExecutor({64: 0.02}, {64: 1})
    srv = serve.Server(ex, hbm_budget=1e9, n_slots=2, max_batch=1)
    reqs = [R(k, 0.0, 64) for k in range(5)]
    drive(srv, ex, reqs)
    slots_in_use = {}
    for t0, size, ids, slot in ex.launches:
        slots_in_use.setdefault(round(t0, 3), []).append(slot)
    # at most 2 concurrent, 3 waves for 5 requests
    assert all(len(v) <= 2 for v in slots_in_use.values())
    assert len(slots_in_use) == 3


def test_summary_percentiles():
    reqs = [serve.Request(k, 0.0, 64, 0, admit=0.0, done=0.001 * (k + 1)) for k in range(100)]
    st = serve.summarize(reqs, 0.1, [1] * 100, 0)
    assert abs(st["p50_ms"] - 50.5) < 1e-6
    assert abs(st["p99_ms"] - 99.01) < 1e-6
    assert abs(st["recon_per_s"] - 1000.0) < 1e-9


def test_trace_is_seeded():
    class P:  # minimal pool entries
        def __init__(self, n):
            self.cfg = type("C", (), {"n": n})()
    pool = [P(64), P(128), P(256)]
    a = serve.make_trace(50.0, 2.0, pool, seed=3)
    b = serve.make_trace(50.0, 2.0, pool, seed=3)
    assert [(r.arrival, r.size) for r in a] == [(r.arrival, r.size) for r in b]
    assert 60 <= len(a) <= 140


def test_cancelled_requests():
    """A queued request leaves at once and is never launched; an admitted one
    finishes with its batch (a solve cannot be interrupted) and is left out of
    the served statistics; unknown ids are ignored."""
    ex = FakeExecutor({64: 0.01}, {64: 1})
    srv = serve.Server(ex, hbm_budget=1e9, n_slots=1, max_batch=1)
    reqs = [R(k, 0.0, 64) for k in range(4)]
    for r in reqs:
        srv.queue.append(r)
    srv.admit(0.0)                       # request 0 is in flight, 1..3 queued
    assert srv.cancel(2, 0.0) == 1       # queued: gone now
    assert srv.cancel(0, 0.0) == 0       # in flight: completes through poll
    assert srv.cancel(99, 0.0) == 0
    done, t = 1, 0.0                     # request 2 counts as finished
    while done < len(reqs):
        t += 1e-3
        ex.now = t
        done += srv.poll(t)
        srv.admit(t)
        assert t < 10
    launched = [rid for l in ex.launches for rid in l[2]]
    assert launched == [0, 1, 3]
    assert reqs[0].cancelled and reqs[2].cancelled and not reqs[1].cancelled
    st = serve.summarize(reqs, t, srv.batches, 0)
    assert st["requests"] == 2 and st["cancelled"] == 2


class FakePool:
    """A slot pool whose slots finish after `iters[slot]` steps; a step takes
    `dt` simulated seconds."""

    def __init__(self, capacity, iters_of, dt, clock):
        self.capacity, self.iters_of, self.dt, self.clock = capacity, iters_of, dt, clock
        self.left = [None] * capacity
        self.loads, self.fetches, self.steps = [], [], []

    def load(self, slot, req):
        assert self.left[slot] is None
        self.left[slot] = self.iters_of(req)
        self.loads.append((self.clock[0], slot, req.rid))

    def step(self):
        busy = [s for s in range(self.capacity) if self.left[s] is not None]
        self.steps.append(busy)
        for s in busy:
            self.left[s] = max(0, self.left[s] - 1)
        return self.clock[0] + self.dt

    def done(self, h):
        return self.clock[0] >= h

    def finished(self):
        return [1 if (x is None or x == 0) else 0 for x in self.left]

    def fetch(self, slot, req):
        self.fetches.append((self.clock[0], slot, req.rid))
        self.left[slot] = None


def drive_iter(server, clock, reqs, dt=1e-3, horizon=100.0):
    i, done, n = 0, 0, len(reqs)
    t = 0.0
    while done < n:
        assert t < horizon
        clock[0] = t
        while i < n and reqs[i].arrival <= t:
            server.queue.append(reqs[i])
            i += 1
        done += server.poll(t)
        server.admit(t)
        t += dt
    return t


def test_iteration_level_admission_refills_slots_at_step_boundaries():
    """A request arriving while a long solve runs joins the same pool at the
    next step boundary and leaves as soon as its own iterations are done,
    before the long solve ends; freed slots take queued requests at once."""
    clock = [0.0]
    iters = {0: 15, 1: 3, 2: 3, 3: 2}
    pool = FakePool(2, lambda r: iters[r.rid], 0.01, clock)
    srv = serve.IterServer({64: pool}, hbm_budget=1e9)
    reqs = [R(0, 0.0, 64), R(1, 0.0305, 64), R(2, 0.0305, 64), R(3, 0.0306, 64)]
    drive_iter(srv, clock, reqs)
    # request 1 is loaded at the first boundary after its arrival, into the free slot
    t_load1 = next(t for t, s, rid in pool.loads if rid == 1)
    assert 0.0305 <= t_load1 <= 0.041
    # 1 finishes after its 3 steps, long before request 0 (15 steps)
    assert reqs[1].done < reqs[0].done
    assert reqs[0].done == pytest.approx(0.15, abs=0.011)
    # 2 takes the slot 1 left; 3 follows 2
    assert reqs[1].done <= next(t for t, s, rid in pool.loads if rid == 2) + 1e-9
    assert reqs[2].done < reqs[3].done < reqs[0].done
    # every step ran on at most 2 slots, never idle while work was loaded
    assert max(len(b) for b in pool.steps) == 2
    assert srv.batches and max(srv.batches) == 2


def test_iteration_level_pools_per_size_and_cancel():
    clock = [0.0]
    a = FakePool(1, lambda r: 4, 0.01, clock)
    b = FakePool(1, lambda r: 2, 0.02, clock)
    srv = serve.IterServer({64: a, 128: b}, hbm_budget=1e9)
    reqs = [R(0, 0.0, 64), R(1, 0.0, 128), R(2, 0.001, 64), R(3, 0.002, 64)]
    i = 0
    t = 0.0
    cancelled_queued = False
    done = 0
    while done < 4:
        clock[0] = t
        while i < 4 and reqs[i].arrival <= t:
            srv.queue.append(reqs[i])
            i += 1
        if t >= 0.003 and not cancelled_queued:
            done += srv.cancel(3, t)          # still queued: leaves at once
            srv.cancel(0, t)                  # running: fetched at the next boundary
            cancelled_queued = True
        done += srv.poll(t)
        srv.admit(t)
        t += 1e-3
        assert t < 10
    assert reqs[3].cancelled and reqs[0].cancelled and not reqs[2].cancelled
    assert reqs[0].done < 0.03              # cut short at the first boundary after the cancel
    assert [rid for _, _, rid in b.fetches] == [1]
    assert [rid for _, _, rid in a.fetches] == [0, 2]


def test_iteration_level_budget():
    class P:
        capacity, nbytes = 4, 5e9
    with pytest.raises(ValueError):
        serve.IterServer({64: P(), 128: P()}, hbm_budget=8e9)
