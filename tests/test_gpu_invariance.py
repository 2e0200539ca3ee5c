"""Batch invariance: a slice's reconstruction is the same bits whether it is
solved alone, inside a same-size batch, inside a mixed-size call, or served
by the continuous-batching loop next to other requests.

Every order of additions in the solver depends on the slice's plan alone:
the ray march and the Jacobian product write one partial of each squared
norm per angle, consumers add partials with one wave in a fixed order, and
the adjoint gather sums fixed runs of angles (the plan's fine groups) into
partial images added in group order; the batch size only changes how many
blocks run them.  The tests use the benchmark's damped step (variables
scaled by their typical magnitudes, the active set) on the mixed grid sizes
{64, 96, 128, 192, 256}^2 (360 angles, 1.5 G bins), and compare with
torch.equal.
"""
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


def same_report(a, b):
    ra, rb = a.to_report(), b.to_report()
    return (ra.iters_run == rb.iters_run and ra.accepted == rb.accepted and ra.phi == rb.phi
            and ra.rho == rb.rho and ra.beta == rb.beta and ra.pred == rb.pred and ra.cg_rr == rb.cg_rr)


@pytest.fixture(scope="module")
def mixed_pool():
    # seeds 0..9 draw every size of the mix twice
    plans, pool = serve.make_pool(10, max_outer=5, n_cg=10)
    assert sorted({s.cfg.n for s in pool}) == list(inputs.MIX_SIZES)
    return plans, pool


def test_alone_equals_same_size_batch_and_mixed_call(mixed_pool):
    plans, pool = mixed_pool
    prm = pget.SolverParams(max_outer=5, n_cg=10, **SCALED)
    alone = []
    for k, sl in enumerate(pool):
        log("alone: slice %d (%d^2)" % (k, sl.cfg.n))
        alone.append(plans[sl.cfg.n].lm_solve(sl.y, sl.f0, sl.mu0, prm))
    for size, plan in plans.items():
        idx = [k for k, sl in enumerate(pool) if sl.cfg.n == size]
        # the slices of this size, twice over: a batch of four
        members = idx + idx
        log("batch of %d at %d^2" % (len(members), size))
        fs, ms, rbs = plan.lm_solve_batched([pool[k].y for k in members], [pool[k].f0 for k in members],
                                            [pool[k].mu0 for k in members], [prm] * len(members))
        for i, k in enumerate(members):
            assert torch.equal(fs[i], alone[k][0]) and torch.equal(ms[i], alone[k][1]), (size, k)
            assert same_report(rbs[i], alone[k][2]), (size, k)
    log("mixed call of %d slices" % len(pool))
    fs, ms, rbs = pget.lm_solve_multi([plans[sl.cfg.n] for sl in pool], [sl.y for sl in pool],
                                      [sl.f0 for sl in pool], [sl.mu0 for sl in pool], [prm] * len(pool))
    for k in range(len(pool)):
        assert torch.equal(fs[k], alone[k][0]) and torch.equal(ms[k], alone[k][1]), k
        assert same_report(rbs[k], alone[k][2]), k


def test_slice_of_a_batch_of_64_equals_alone():
    """The benchmark's launch configuration: a 128^2 slice (360 x 192) as
    slice 0 of 64 distinct slices gives the bits of its solve alone."""
    cfg = inputs.MAIN_128
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    one = torch.ones((cfg.n, cfg.n), dtype=torch.float32, device="cuda")
    a1 = plan.forward(one, torch.zeros_like(one)).double().cpu().numpy()
    ys, f0s, m0s = [], [], []
    for s in range(64):
        f, mu = inputs.rod_lattice(cfg, s)
        y = inputs.poisson_counts(plan.forward(T(f), T(mu)).double().cpu().numpy(), cfg.peak_counts, s)
        c0 = float((a1 * y).sum() / (a1 * a1).sum())
        ys.append(T(y))
        f0s.append(torch.full((cfg.n, cfg.n), c0, dtype=torch.float32, device="cuda"))
        m0s.append(torch.zeros_like(one))
    prm = pget.SolverParams(max_outer=4, n_cg=10, **SCALED)
    log("batch of 64 at 128^2")
    fs, ms, rbs = plan.lm_solve_batched(ys, f0s, m0s, [prm] * 64)
    for s in (0, 37):
        fa, ma, ra = plan.lm_solve(ys[s], f0s[s], m0s[s], prm)
        assert torch.equal(fs[s], fa) and torch.equal(ms[s], ma), s
        assert same_report(rbs[s], ra), s


def test_served_requests_equal_alone(mixed_pool):
    """Requests of mixed sizes served with early exit (tolerance 1e-4): each
    batched with others of its size, several solves in flight on different
    streams; every result has the bits of its slice solved alone."""
    plans, pool = mixed_pool
    prm = pget.SolverParams(max_outer=5, n_cg=10, tol=1e-4, **SCALED)
    ex = serve.GpuExecutor(plans, pool, prm, n_slots=3)
    srv = serve.Server(ex, hbm_budget=1e12, n_slots=3, max_batch=4)
    reqs = [serve.Request(k, 0.002 * k, pool[k % len(pool)].cfg.n, k % len(pool)) for k in range(20)]
    outputs = {}
    orig_launch = ex.launch

    def launch(size, rs, slot):
        h = orig_launch(size, rs, slot)
        for i, r in enumerate(rs):
            outputs[r.rid] = (h[1][0][i], h[1][1][i])
        return h

    ex.launch = launch
    st = serve.run_trace(srv, reqs, timeout=300)
    log("served %d requests, batches %s" % (st["requests"], sorted(set(srv.batches))))
    assert st["requests"] == 20 and max(srv.batches) > 1
    alone = {}
    for r in reqs:
        if r.slot not in alone:
            sl = pool[r.slot]
            alone[r.slot] = plans[r.size].lm_solve(sl.y, sl.f0, sl.mu0, prm)
        f, m = outputs[r.rid]
        assert torch.equal(f, alone[r.slot][0]) and torch.equal(m, alone[r.slot][1]), r.rid


def test_autotuned_shapes_keep_every_bit(mixed_pool):
    """The autotuner picks launch shapes only (angle slots per product block,
    fine groups per gather block): the solve after tuning has the same bits."""
    plans, pool = mixed_pool
    sl = next(s for s in pool if s.cfg.n == 96)
    plan = plans[96]
    prm = pget.SolverParams(max_outer=4, n_cg=8, **SCALED)
    f1, m1, r1 = plan.lm_solve(sl.y, sl.f0, sl.mu0, prm)
    shape = plan.autotune(1)
    log("tuned shape %s" % shape)
    f2, m2, r2 = plan.lm_solve(sl.y, sl.f0, sl.mu0, prm)
    assert torch.equal(f1, f2) and torch.equal(m1, m2) and same_report(r1, r2)


def test_iteration_level_served_requests_equal_alone(mixed_pool):
    """The same, served by per-size slot pools that admit requests at every
    outer-iteration boundary (slots at different iterations share launches)."""
    plans, pool = mixed_pool
    prm = pget.SolverParams(max_outer=5, n_cg=10, tol=1e-4, **SCALED)
    pools = serve.make_pools(plans, pool, prm, {n: 3 for n in plans})
    for gp in pools.values():
        gp.keep_outputs = True
    srv = serve.IterServer(pools, hbm_budget=1e12)
    reqs = [serve.Request(k, 0.003 * k, pool[k % len(pool)].cfg.n, k % len(pool)) for k in range(24)]
    st = serve.run_trace(srv, reqs, timeout=300)
    log("served %d requests through slot pools, mean occupancy %.2f" % (st["requests"], st["mean_batch"]))
    assert st["requests"] == 24
    outputs = {}
    for gp in pools.values():
        outputs.update(gp.outputs)
    torch.cuda.synchronize()
    alone = {}
    for r in reqs:
        if r.slot not in alone:
            sl = pool[r.slot]
            alone[r.slot] = plans[r.size].lm_solve(sl.y, sl.f0, sl.mu0, prm)
        f, m = outputs[r.rid]
        assert torch.equal(f, alone[r.slot][0]) and torch.equal(m, alone[r.slot][1]), r.rid


@pytest.mark.parametrize("storage,depth_response", [("fp32", False), ("fp32", True), ("bf16", False)],
                         ids=["plain", "depth_response", "bf16"])
def test_band_staging_keeps_every_bit(storage, depth_response):
    """With band staging on, a map whose bordered pair does not fit in LDS
    (FP32 150^2 at 60 x 220, BF16 210^2 at 60 x 300: two bands of rows) is
    walked band by band in every launch shape: product blocks of at least 6
    angle slots stage each band in LDS, smaller ones read the bordered copy
    in HBM over the same bands in the same order.  A Jacobian product and a
    solve give the same bits either way."""
    import numpy as np
    n, na, nb = (150, 60, 220) if storage == "fp32" else (210, 60, 300)
    plan = pget.Plan(n, na, nb, storage=storage)
    assert plan.set_band_staging(True) == 2
    if depth_response:
        n_t, K = plan.n_samples, plan.psf_half_width
        _, far = inputs.collimator_depth_response(n_t, K, 3.0)
        plan.set_depth_response(np.linspace(0.0, 1.0, n_t), far)
    k = n / 150.0
    cfg = inputs.SliceConfig("lattice5_n%d" % n, n, na, nb, n_rods=5, rod_radius=4.0 * k, pitch=24.0 * k,
                             can_half=66.0 * k, n_empty=2)
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = T(inputs.poisson_counts(plan.forward(T(f_true), T(mu_true)).double().cpu().numpy(), 1e4, 0))
    f0 = torch.full((n, n), float(f_true.mean()), device="cuda")
    m0 = torch.zeros((n, n), device="cuda")
    rng = np.random.default_rng(3)
    vf, vm = T(rng.standard_normal((n, n))), T(0.05 * rng.standard_normal((n, n)))
    prm = pget.SolverParams(max_outer=3, n_cg=8, **SCALED)
    runs = []
    for slots in (1, 8):
        shape = plan.set_shape(1, jvp_angle_slots=slots)
        log("%d^2 %s (%s): product %s" % (n, storage, "depth response" if depth_response else "plain", shape))
        assert shape["jvp_angle_slots"] == slots and shape["tuned"]
        jv = plan.jvp(f0, T(0.02 * f_true), vf, vm)
        runs.append((jv, plan.lm_solve(y, f0, m0, prm)))
    (jv1, (f1, m1, r1)), (jv2, (f2, m2, r2)) = runs
    assert torch.equal(jv1, jv2)
    assert torch.equal(f1, f2) and torch.equal(m1, m2) and same_report(r1, r2)
