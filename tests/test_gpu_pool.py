"""Slot pools (continuous batching at outer-iteration boundaries) against
solves alone: slices loaded into a pool at different times, running at
different outer iterations in the same launches, retired as they finish and
replaced by queued ones, give the bits of their solves alone; a slot fetched
before it finishes (cancelled) holds the iterate of a solve stopped after
the same number of iterations."""
import sys

import pytest

from paper_2604_26745_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2604_26745_amd import pget, serve  # noqa: E402

SCALED = dict(w_mu=0.05 ** 2, d_mu=1.0 / 0.05 ** 2, active_set=1)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def same(ra, rb):
    a, b = ra.to_report(), rb.to_report()
    return (a.iters_run == b.iters_run and a.accepted == b.accepted and a.phi == b.phi and a.rho == b.rho
            and a.beta == b.beta and a.stop_reason == b.stop_reason and a.status == b.status)


@pytest.fixture(scope="module")
def slices():
    plans, pool = serve.make_pool(12, max_outer=6, n_cg=10)
    return plans, pool


def test_pool_results_equal_alone(slices):
    plans, pool = slices
    size = 64
    idx = [k for k, s in enumerate(pool) if s.cfg.n in (64, 96)]
    size = pool[idx[0]].cfg.n
    idx = [k for k in idx if pool[k].cfg.n == size]
    assert len(idx) >= 2
    plan = plans[size]
    # parameters per request: the scaled step; early exit on one, fewer
    # iterations on another, the plain step on a third
    prms = []
    for j in range(6):
        kw = dict(max_outer=6, n_cg=10, **SCALED)
        if j % 3 == 1:
            kw["tol"] = 1e-3
        if j % 3 == 2:
            kw["max_outer"] = 4
        if j == 5:
            kw = dict(max_outer=6, n_cg=10)
        prms.append(pget.SolverParams(**kw))
    reqs = [(pool[idx[j % len(idx)]], prms[j]) for j in range(6)]
    alone = [plan.lm_solve(sl.y, sl.f0, sl.mu0, p) for sl, p in reqs]
    P = pget.LMPool(plan, capacity=3, max_outer=6, n_cg=10)
    queue = list(range(6))
    where = {}          # slot -> request
    results = {}
    steps = 0
    while len(results) < 6:
        for slot in range(3):
            if slot not in where and queue:
                j = queue.pop(0)
                sl, p = reqs[j]
                P.load(slot, sl.y, sl.f0, sl.mu0, p)
                where[slot] = j
        ev = P.step()
        ev.synchronize()
        steps += 1
        fin = P.finished.tolist()
        for slot in list(where):
            if fin[slot]:
                results[where.pop(slot)] = P.fetch(slot)
        assert steps < 100
    torch.cuda.synchronize()
    log("pool of 3 slots served 6 requests in %d steps" % steps)
    for j in range(6):
        f, m, rb = results[j]
        fa, ma, ra = alone[j]
        assert torch.equal(f, fa) and torch.equal(m, ma), j
        assert same(rb, ra), j


def test_pool_cancel_mid_solve(slices):
    plans, pool = slices
    sl = next(s for s in pool if s.cfg.n == 128)
    plan = plans[128]
    P = pget.LMPool(plan, capacity=2, max_outer=6, n_cg=10)
    P.load(1, sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=6, n_cg=10, **SCALED))
    for _ in range(2):
        P.step().synchronize()
    assert P.finished.tolist() == [1, 0]   # slot 0 free, slot 1 running
    f, m, rb = P.fetch(1)
    fa, ma, ra = plan.lm_solve(sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=2, n_cg=10, **SCALED))
    assert torch.equal(f, fa) and torch.equal(m, ma)
    assert rb.to_report().accepted == ra.to_report().accepted
    # the freed slot takes a new slice, which runs to completion
    P.load(1, sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=3, n_cg=10, **SCALED))
    for _ in range(3):
        P.step().synchronize()
    assert P.finished.tolist() == [1, 1]
    f, m, _ = P.fetch(1)
    fa, ma, _ = plan.lm_solve(sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=3, n_cg=10, **SCALED))
    assert torch.equal(f, fa) and torch.equal(m, ma)


def test_pool_rejects_misuse(slices):
    plans, pool = slices
    sl = next(s for s in pool if s.cfg.n == 128)
    P = pget.LMPool(plans[128], capacity=2, max_outer=4, n_cg=10)
    with pytest.raises(pget.PgetError):
        P.load(0, sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=5, n_cg=10))   # longer than the pool
    with pytest.raises(pget.PgetError):
        P.load(0, sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=4, n_cg=8))    # other CG length
    with pytest.raises(pget.PgetError):
        P.fetch(1)                                                                 # free slot
    P.load(0, sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=4, n_cg=10))
    with pytest.raises(pget.PgetError):
        P.load(0, sl.y, sl.f0, sl.mu0, pget.SolverParams(max_outer=4, n_cg=10))   # busy slot
