"""Continuous-batching request loop for LM reconstructions on one GPU.

Requests (one slice each, mixed grid sizes) arrive open-loop.  The server
keeps several solves in flight on separate HIP streams; a queued request is
admitted as soon as a stream is free and its workspace fits in the HBM budget
of in-flight work, together with up to ``max_batch`` other queued requests of
the same size (a batched solve of one plan).  Solver state stays on the
device for the whole solve (every LM decision is taken by the kernels), and
the early-exit tolerance lets converged slices skip their remaining work.
Completion is detected by polling an event recorded after each solve.

The comparison is the plain per-slice solver: the same trace, one request at
a time, in arrival order, on one stream.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import inputs, pget

BATCH_SIZES = (1, 2, 4, 8)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    size: int               # grid size N (selects the plan)
    slot: int               # index in the slice pool
    admit: float = math.nan
    done: float = math.nan
    batch: int = 0
    cancelled: bool = False


@dataclass
class Slice:
    cfg: inputs.SliceConfig
    y: object               # device tensors
    f0: object
    mu0: object


def make_pool(n_slices: int, max_outer: int = 15, n_cg: int = 30, seed0: int = 0):
    """Pre-generated request payloads: mixed-size rod-lattice slices (the
    library's forward map gives the clean data, counting noise on top)."""
    import torch
    plans: Dict[int, pget.Plan] = {}
    a1: Dict[int, np.ndarray] = {}
    pool: List[Slice] = []
    for k in range(n_slices):
        cfg, peak = inputs.mixed_config(seed0 + k)
        cfg = inputs.scaled(cfg, max_outer=max_outer, n_cg=n_cg)
        if cfg.n not in plans:
            plans[cfg.n] = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
            one = torch.ones((cfg.n, cfg.n), dtype=torch.float32, device="cuda")
            a1[cfg.n] = plans[cfg.n].forward(one, torch.zeros_like(one)).double().cpu().numpy()
        plan = plans[cfg.n]
        f, mu = inputs.rod_lattice(cfg, seed0 + k)
        T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
        y = inputs.poisson_counts(plan.forward(T(f), T(mu)).double().cpu().numpy(), peak, seed0 + k)
        c0 = float((a1[cfg.n] * y).sum() / (a1[cfg.n] * a1[cfg.n]).sum())
        pool.append(Slice(cfg, T(y), torch.full((cfg.n, cfg.n), c0, dtype=torch.float32,
                                                 device="cuda"),
                          torch.zeros((cfg.n, cfg.n), dtype=torch.float32, device="cuda")))
    return plans, pool


@dataclass
class _InFlight:
    reqs: List[Request]
    slot: int
    handle: object
    nbytes: int


class GpuExecutor:
    """Runs batched solves of one plan on one of several HIP streams; each
    stream slot owns reusable workspaces per (size, batch)."""

    def __init__(self, plans: Dict[int, pget.Plan], pool: List[Slice], params: pget.SolverParams,
                 n_slots: int = 4):
        import torch
        self.torch = torch
        self.plans, self.pool, self.params = plans, pool, params
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]   # default priority
        self.ws: Dict[tuple, object] = {}

    def workspace_bytes(self, size: int, b: int) -> int:
        return self.plans[size].workspace_bytes(pget.OP_LM, b)

    def _workspace(self, size: int, b: int, slot: int):
        key = (size, b, slot)
        if key not in self.ws:
            self.ws[key] = self.torch.empty(self.workspace_bytes(size, b), dtype=self.torch.uint8,
                                            device="cuda")
        return self.ws[key]

    def launch(self, size: int, reqs: List[Request], slot: int):
        b = len(reqs)
        s = self.streams[slot]
        with self.torch.cuda.stream(s):
            sl = [self.pool[r.slot] for r in reqs]
            out = self.plans[size].lm_solve_batched(
                [x.y for x in sl], [x.f0 for x in sl], [x.mu0 for x in sl], [self.params] * b,
                sync=False, ws=self._workspace(size, b, slot))
            ev = self.torch.cuda.Event()
            ev.record(s)
        return (ev, out)

    def done(self, handle) -> bool:
        return handle[0].query()

    def warm(self, batch_sizes):
        """Capture the solver graph of every (size, batch, slot) before the
        trace starts, so that no capture happens while requests wait."""
        for size in self.plans:
            sl = next(x for x in self.pool if x.cfg.n == size)
            for b in batch_sizes:
                for slot in range(len(self.streams)):
                    r = [Request(-1, 0.0, size, self.pool.index(sl))] * b
                    self.launch(size, r, slot)
        self.torch.cuda.synchronize()


class Server:
    """Admission (HBM budget of in-flight workspaces, free execution slots),
    same-size batching and completion tracking.  Executor-agnostic."""

    def __init__(self, executor, hbm_budget: float = 64e9, n_slots: int = 4, max_batch: int = 8):
        self.ex = executor
        self.budget = hbm_budget
        self.max_batch = max(b for b in BATCH_SIZES if b <= max_batch)
        self.batch_sizes = tuple(b for b in BATCH_SIZES if b <= self.max_batch)
        self.free_slots = list(range(n_slots))[::-1]
        self.queue: deque = deque()
        self.in_flight: List[_InFlight] = []
        self.in_flight_bytes = 0
        self.max_in_flight_bytes = 0
        self.batches: List[int] = []

    def warm(self):
        self.ex.warm(self.batch_sizes)

    def cancel(self, rid: int, now: float) -> int:
        """Cancel request `rid`.  A queued request leaves the queue at once
        (returns 1: it will not complete through poll); an admitted one runs
        to the end of its batch's solve, which cannot be interrupted, and its
        result is dropped (returns 0: poll still completes it).  Unknown or
        finished requests are left alone (returns 0)."""
        for r in self.queue:
            if r.rid == rid:
                self.queue.remove(r)
                r.cancelled, r.done = True, now
                return 1
        for job in self.in_flight:
            for r in job.reqs:
                if r.rid == rid:
                    r.cancelled = True
        return 0

    def poll(self, now: float) -> int:
        done = 0
        still = []
        for job in self.in_flight:
            if self.ex.done(job.handle):
                for r in job.reqs:
                    r.done = now
                self.in_flight_bytes -= job.nbytes
                self.free_slots.append(job.slot)
                done += len(job.reqs)
            else:
                still.append(job)
        self.in_flight = still
        return done

    def admit(self, now: float):
        """Admit the oldest queued request with up to max_batch queued requests
        of its size (largest supported batch size, arrival order), while an
        execution slot is free and the batch's workspace fits in the budget
        (a batch is always admitted when nothing is in flight)."""
        while self.queue and self.free_slots:
            head = self.queue[0]
            same = [r for r in self.queue if r.size == head.size][: self.max_batch]
            b = max(x for x in self.batch_sizes if x <= len(same))
            take = same[:b]
            nbytes = self.ex.workspace_bytes(head.size, b)
            if self.in_flight and self.in_flight_bytes + nbytes > self.budget:
                return
            for r in take:
                self.queue.remove(r)
                r.admit, r.batch = now, b
            slot = self.free_slots.pop()
            handle = self.ex.launch(head.size, take, slot)
            self.in_flight.append(_InFlight(take, slot, handle, nbytes))
            self.in_flight_bytes += nbytes
            self.max_in_flight_bytes = max(self.max_in_flight_bytes, self.in_flight_bytes)
            self.batches.append(b)


def run_trace(server: Server, reqs: List[Request], timeout: float = 600.0) -> dict:
    """Replay arrivals in real time through the server; returns statistics."""
    t0 = time.perf_counter()
    i, done, n = 0, 0, len(reqs)
    while done < n:
        now = time.perf_counter() - t0
        if now > timeout:
            raise RuntimeError("trace did not drain within %.0f s" % timeout)
        while i < n and reqs[i].arrival <= now:
            server.queue.append(reqs[i])
            i += 1
        done += server.poll(now)
        server.admit(now)
        queued = server.queued() if hasattr(server, "queued") else len(server.queue)
        if not server.in_flight and i < n and not queued:
            time.sleep(max(0.0, min(0.002, reqs[i].arrival - now)))
        else:
            time.sleep(0.0002)
    makespan = max(r.done for r in reqs)
    return summarize(reqs, makespan, server.batches, server.max_in_flight_bytes)


def run_plain(plans, pool, params, reqs: List[Request], timeout: float = 600.0) -> dict:
    """The plain per-slice solver: one request at a time, arrival order."""
    import torch
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for r in reqs:
            now = time.perf_counter() - t0
            if now > timeout:
                raise RuntimeError("plain solver did not drain within %.0f s" % timeout)
            if r.arrival > now:
                time.sleep(r.arrival - now)
            sl = pool[r.slot]
            r.admit = time.perf_counter() - t0
            plans[r.size].lm_solve(sl.y, sl.f0, sl.mu0, params, sync=False)
            stream.synchronize()
            r.done = time.perf_counter() - t0
            r.batch = 1
    return summarize(reqs, max(r.done for r in reqs), [1] * len(reqs), 0)


def summarize(reqs: List[Request], makespan: float, batches: List[int], peak_bytes: int) -> dict:
    served = [r for r in reqs if not r.cancelled]
    lat = np.array([r.done - r.arrival for r in served]) if served else np.zeros(1)
    return {
        "requests": len(served),
        "cancelled": len(reqs) - len(served),
        "recon_per_s": len(served) / makespan,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "makespan_s": makespan,
        "mean_batch": float(np.mean(batches)) if batches else 0.0,
        "peak_in_flight_gb": peak_bytes / 1e9,
    }


def make_trace(rate: float, duration: float, pool: List[Slice], seed: int = 0) -> List[Request]:
    arr = inputs.arrival_times(rate, duration, seed)
    rng = np.random.default_rng([seed, 4])
    picks = rng.integers(0, len(pool), size=len(arr))
    return [Request(k, float(t), pool[int(p)].cfg.n, int(p)) for k, (t, p) in enumerate(zip(arr, picks))]


# ---------------------------------------------------------------------------
# Continuous batching at outer-iteration boundaries.
#
# Each grid size has a slot pool (pget_lm_pool) on its own stream: one step
# is one outer LM iteration of every occupied slot.  Between steps, slots
# whose solve has stopped (max_outer, early-exit tolerance, damping
# overflow, non-finite) are retired and queued requests of that size take
# the free slots at once, so a request waits at most one outer iteration of
# its size for admission and never for a whole batch to finish.  Pools of
# different sizes step concurrently on their streams.


class GpuPool:
    """One size's slot pool on the GPU (pget.LMPool) behind the interface
    the iteration-level server drives: capacity, load, step, done,
    finished, fetch."""

    def __init__(self, plan: pget.Plan, pool: List[Slice], params: pget.SolverParams, capacity: int):
        import torch
        self.torch = torch
        self.pool, self.params = pool, params
        self.stream = torch.cuda.Stream()   # default priority
        with torch.cuda.stream(self.stream):
            self.p = pget.LMPool(plan, capacity, params.max_outer, params.n_cg, stream=self.stream, step=params.step)
        self.capacity = capacity
        self.nbytes = int(self.p.ws.numel())
        self.outputs: Dict[int, tuple] = {}   # rid -> (f, mu) of served requests (kept if keep_outputs)
        self.keep_outputs = False
        # per step: device time (events around it) and host time from launch
        # to the poll that saw it complete
        self.step_stats = {"steps": 0, "gpu_ms": 0.0, "wall_ms": 0.0}
        self._t = None

    def load(self, slot: int, req: Request):
        sl = self.pool[req.slot]
        self.p.load(slot, sl.y, sl.f0, sl.mu0, self.params)

    def step(self):
        start = self.torch.cuda.Event(enable_timing=True)
        start.record(self.stream)
        end = self.p.step(timing=True)
        self._t = (start, end, time.perf_counter())
        return end

    def done(self, handle) -> bool:
        if not handle.query():
            return False
        if self._t is not None and self._t[1] is handle:
            start, end, t0 = self._t
            self.step_stats["steps"] += 1
            self.step_stats["gpu_ms"] += start.elapsed_time(end)
            self.step_stats["wall_ms"] += 1e3 * (time.perf_counter() - t0)
            self._t = None
        return True

    def finished(self) -> List[int]:
        return self.p.finished.tolist()

    def fetch(self, slot: int, req: Request):
        f, mu, _ = self.p.fetch(slot, report=False)
        if self.keep_outputs:
            self.outputs[req.rid] = (f, mu)


class IterServer:
    """Admission at outer-iteration boundaries into per-size slot pools.
    Same driving interface as Server (queue, poll, admit, in_flight,
    batches, max_in_flight_bytes), executor-agnostic: `pools` maps a grid
    size to an object with capacity, load(slot, req), step() -> handle,
    done(handle), finished() -> per-slot flags, fetch(slot, req)."""

    def __init__(self, pools: Dict[int, object], hbm_budget: float = 64e9):
        self.pools = pools
        total = sum(getattr(p, "nbytes", 0) for p in pools.values())
        if total > hbm_budget:
            raise ValueError("slot pools need %.1f GB, over the %.1f GB budget" % (total / 1e9, hbm_budget / 1e9))
        self.max_in_flight_bytes = total
        self.queue: deque = deque()       # inbox (arrival order); sorted into per-size queues
        self.waiting: Dict[int, deque] = {s: deque() for s in pools}
        self.slots: Dict[int, List[Optional[Request]]] = {s: [None] * p.capacity for s, p in pools.items()}
        self.step_handle: Dict[int, object] = {s: None for s in pools}
        self.batches: List[int] = []      # occupied slots per step
        self.cancelled_rids: set = set()

    @property
    def in_flight(self):
        return [s for s, held in self.slots.items() if any(r is not None for r in held)]

    def queued(self) -> int:
        return len(self.queue) + sum(len(q) for q in self.waiting.values())

    def cancel(self, rid: int, now: float) -> int:
        """A queued request leaves at once (returns 1); an admitted one is
        fetched at its pool's next iteration boundary and dropped from the
        statistics (returns 0: poll completes it)."""
        self._sort_inbox()
        for q in self.waiting.values():
            for r in q:
                if r.rid == rid:
                    q.remove(r)
                    r.cancelled, r.done = True, now
                    return 1
        for held in self.slots.values():
            for r in held:
                if r is not None and r.rid == rid:
                    r.cancelled = True
        return 0

    def _sort_inbox(self):
        while self.queue:
            r = self.queue.popleft()
            self.waiting[r.size].append(r)

    def poll(self, now: float) -> int:
        """Retire finished (or cancelled) slots of every pool whose last step
        has completed; returns the number of requests completed."""
        done = 0
        for size, pool in self.pools.items():
            h = self.step_handle[size]
            if h is None or not pool.done(h):
                continue
            self.step_handle[size] = None
            flags = pool.finished()
            for slot, r in enumerate(self.slots[size]):
                if r is not None and (flags[slot] or r.cancelled):
                    pool.fetch(slot, r)
                    r.done = now
                    self.slots[size][slot] = None
                    done += 1
        return done

    def admit(self, now: float):
        """Load queued requests (arrival order) into the free slots of their
        size's pool, then start the next step of every idle pool that holds
        work."""
        self._sort_inbox()
        for size, pool in self.pools.items():
            if self.step_handle[size] is not None:
                continue
            held, q = self.slots[size], self.waiting[size]
            for slot in range(pool.capacity):
                if held[slot] is not None:
                    continue
                if not q:
                    break
                req = q.popleft()
                pool.load(slot, req)
                req.admit, req.batch = now, pool.capacity
                held[slot] = req
            busy = sum(r is not None for r in held)
            if busy:
                self.step_handle[size] = pool.step()
                self.batches.append(busy)


def make_pools(plans: Dict[int, pget.Plan], pool: List[Slice], params: pget.SolverParams,
               capacity: Dict[int, int]) -> Dict[int, GpuPool]:
    """A GPU slot pool per size, warmed (its step graph captured) before
    the trace starts."""
    import torch
    pools = {n: GpuPool(plans[n], pool, params, capacity[n]) for n in plans}
    for n, gp in pools.items():
        gp.step().synchronize()     # captures the step graph on empty slots
    torch.cuda.synchronize()
    return pools
