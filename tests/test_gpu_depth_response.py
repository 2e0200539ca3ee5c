"""The depth-dependent collimator response (pget_plan_set_depth_response:
sample i seen through (1 - alpha_i) times the Gaussian taps plus alpha_i
times a far response) on the GPU against the FP64 oracle, which spreads
every sample with its own response:

* the operators with and without the quarter-turn fold of the gather, over
  a half turn (no mirror pairing), with maps too large for LDS (read from
  HBM) up to the largest map, and together with the depth factor of the
  attenuation path (relative L2 <= 1e-5, 2e-5 above 256 px as for the plain
  model; max-abs / max-ref <= 1e-4);
* an LM trajectory of the full discrete model (depth factor and response)
  with the oracle's decisions replayed (objective per iterate 1e-4, maps
  1e-3, as for the plain model);
* batched and mixed-size solves against single-slice solves of the same
  slices (each checked against the oracle above) with replayed decisions;
* that clearing the response gives back a fresh plan's results bitwise,
  that a solve after setting it does not reuse a captured sequence, the
  workspace growth, and argument errors.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import lm as OLM
from paper_2604_26745_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2604_26745_amd import pget  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def H(t):
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def depth_table(n_t):
    return tuple(1.0 + 0.6 * (1.0 - i / (n_t - 1)) for i in range(n_t))


def jittered_alpha(n_t, seed):
    a = 1.0 - np.arange(n_t) / (n_t - 1)
    a = np.clip(a + 0.15 * np.random.default_rng(seed).uniform(-1, 1, n_t), 0.0, 1.0)
    return tuple(float(v) for v in a)


def phantom(n, seed, mu_rod=0.08):
    cfg = inputs.SliceConfig("t", n, 8, n, n_rods=5, rod_radius=max(1.0, n / 24), pitch=n / 7,
                             can_half=0.42 * n, n_empty=2, rod_mu=mu_rod)
    return inputs.rod_lattice(cfg, seed)


@pytest.mark.parametrize("with_depth", [False, True], ids=["response", "response_and_depth"])
@pytest.mark.parametrize("n,na,nb,arc,bin_size,step", [
    (64, 120, 96, 2 * np.pi, 1.0, 1.0), (48, 90, 70, 2 * np.pi, 1.0, 1.0), (40, 45, 60, np.pi, 1.0, 1.0),
    (150, 24, 220, 2 * np.pi, 1.0, 1.0), (512, 8, 730, 2 * np.pi, 1.0, 1.0),
    (60, 36, 46, 2 * np.pi, 2.0, 1.0), (48, 40, 70, 2 * np.pi, 1.0, 1.5)],
    ids=["quad", "paired", "half_turn", "maps_in_hbm", "max_size", "bins_of_2px", "step_1p5"])
def test_operators_with_depth_response(n, na, nb, arc, bin_size, step, with_depth):
    plan = pget.Plan(n, na, nb, arc=arc, bin_size=bin_size, step=step)
    n_t, K = plan.n_samples, plan.psf_half_width
    _, far = inputs.collimator_depth_response(n_t, K, 3.0)
    al = jittered_alpha(n_t, 7)
    d = depth_table(n_t) if with_depth else None
    if d is not None:
        plan.set_depth_factor(d)
    plan.set_depth_response(al, far)
    og = O.Geometry(n, na, nb, arc=arc, bin_size=bin_size, step=step, depth=d, resp=al, far_taps=far)
    f, mu = phantom(n, 3)
    rng = np.random.default_rng(5)
    vf, vm = rng.standard_normal((2, n, n))
    vm *= 0.05
    w = rng.standard_normal((na, nb))
    log("case n=%d na=%d nb=%d arc=%.3f bin=%g step=%g depth=%s" % (n, na, nb, arc, bin_size, step, with_depth))
    y, y_ref = H(plan.forward(T(f), T(mu))), O.forward(og, f, mu)
    jv, jv_ref = H(plan.jvp(T(f), T(mu), T(vf), T(vm))), O.jvp(og, f, mu, vf, vm)
    gf, gm = plan.vjp(T(f), T(mu), T(w))
    gf_ref, gm_ref = O.vjp(og, f, mu, w)
    errs = (rel(y, y_ref), rel(jv, jv_ref), rel(H(gf), gf_ref), rel(H(gm), gm_ref))
    log("  forward %.2e jvp %.2e vjp f %.2e mu %.2e" % errs)
    # sample positions beyond ~256 px carry FP32 rounding of their coordinates
    assert max(errs) <= (1e-5 if n <= 256 else 2e-5)
    assert maxrel(y, y_ref) <= 1e-4 and maxrel(jv, jv_ref) <= 1e-4
    assert maxrel(H(gf), gf_ref) <= 1e-4 and maxrel(H(gm), gm_ref) <= 1e-4
    # the response is in effect
    assert rel(y, O.forward(O.Geometry(n, na, nb, arc=arc, bin_size=bin_size, step=step, depth=d), f, mu)) > 1e-3


def lattice_case():
    return inputs.SliceConfig("lattice3_n24", 24, 36, 36, n_rods=3, rod_radius=2.0, pitch=6.0,
                              can_half=10.0, n_empty=1, max_outer=6, n_cg=4)


def full_model(plan):
    n_t, K = plan.n_samples, plan.psf_half_width
    al, far = inputs.collimator_depth_response(n_t, K, 3.0)
    return depth_table(n_t), al, far


def test_lm_full_model_replayed():
    cfg = lattice_case()
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    d, al, far = full_model(plan)
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, depth=d, resp=al, far_taps=far)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(og, y)
    p = OLM.LMParams(max_outer=cfg.max_outer, n_cg=cfg.n_cg, w_mu=0.05 ** 2, active_set=True)
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p)
    plan.set_depth_factor(d)
    plan.set_depth_response(al, far)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(
        max_outer=cfg.max_outer, n_cg=cfg.n_cg, w_mu=0.05 ** 2, active_set=1, replay=orep.accepted))
    rep = rb.to_report()
    assert rep.accepted == orep.accepted
    for k in range(rep.iters_run + 1):
        e = abs(rep.phi[k] - orep.phi[k]) / orep.phi[k]
        log("k=%d phi %.8g / %.8g (%.1e)" % (k, rep.phi[k], orep.phi[k], e))
        assert e <= 1e-4
    log("maps rel L2: f %.2e mu %.2e" % (rel(H(f), of), rel(H(mu), om)))
    assert rel(H(f), of) <= 1e-3 and rel(H(mu), om) <= 1e-3


def test_batched_and_mixed_match_single_solves():
    """Slices of a batch and of a mixed-size call index the far planes of
    the per-ray sums by their own offsets: each equals its single-slice
    solve (same decisions replayed) to FP32 rounding of the launch shapes."""
    shapes = [(24, 36, 36), (32, 48, 44), (150, 16, 216)]   # the last: maps read from HBM
    plans, cases = {}, []
    for (n, na, nb) in shapes:
        plan = pget.Plan(n, na, nb)
        d, al, far = full_model(plan)
        plan.set_depth_factor(d)
        plan.set_depth_response(al, far)
        plans[n] = plan
        og = O.Geometry(n, na, nb, depth=d, resp=al, far_taps=far)
        for seed in range(2):
            f_true, mu_true = phantom(n, 10 + seed)
            y = inputs.poisson_counts(O.forward(og, f_true, mu_true), 1e4, seed)
            f0, mu0 = OLM.initial_guess(og, y)
            cases.append((n, y, f0, mu0))
    prm = dict(max_outer=4, n_cg=5, w_mu=0.05 ** 2, active_set=1)
    single = []
    for (n, y, f0, mu0) in cases:
        f, mu, rb = plans[n].lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(**prm))
        single.append((H(f), H(mu), rb.to_report()))

    def check(tag, k, f, mu, rep):
        sf, sm, srep = single[k]
        assert rep.accepted == srep.accepted
        e = max(abs(a - b) / b for a, b in zip(rep.phi[:rep.iters_run + 1], srep.phi[:rep.iters_run + 1]))
        log("%s slice %d: phi %.1e f %.1e mu %.1e" % (tag, k, e, rel(f, sf), rel(mu, sm)))
        assert e <= 1e-5 and rel(f, sf) <= 1e-4 and rel(mu, sm) <= 1e-4

    # batches of one shape
    for n in plans:
        idx = [k for k, c in enumerate(cases) if c[0] == n]
        fs, ms, rbs = plans[n].lm_solve_batched(
            [T(cases[k][1]) for k in idx], [T(cases[k][2]) for k in idx], [T(cases[k][3]) for k in idx],
            [pget.SolverParams(**prm, replay=single[k][2].accepted) for k in idx])
        for j, k in enumerate(idx):
            check("batch", k, H(fs[j]), H(ms[j]), rbs[j].to_report())
    # all four in one mixed-size call
    fs, ms, rbs = pget.lm_solve_multi(
        [plans[c[0]] for c in cases], [T(c[1]) for c in cases], [T(c[2]) for c in cases],
        [T(c[3]) for c in cases], [pget.SolverParams(**prm, replay=s[2].accepted) for s in single])
    for k in range(len(cases)):
        check("mixed", k, H(fs[k]), H(ms[k]), rbs[k].to_report())


def test_clearing_and_setting_the_response():
    n, na, nb = 32, 40, 48
    f, mu = phantom(n, 4)
    y = T(O.forward(O.Geometry(n, na, nb), f, mu))
    f0 = torch.full((n, n), 0.5, device="cuda")
    m0 = torch.zeros((n, n), device="cuda")
    prm = pget.SolverParams(max_outer=3, n_cg=6)
    fresh = pget.Plan(n, na, nb)
    y_plain = fresh.forward(T(f), T(mu))
    f_plain, _, _ = fresh.lm_solve(y, f0, m0, prm)
    plan = pget.Plan(n, na, nb)
    ws0 = plan.workspace_bytes(pget.OP_LM, 1)
    plan.lm_solve(y, f0, m0, prm)          # captures the solve without the response
    al, far = inputs.collimator_depth_response(plan.n_samples, plan.psf_half_width, 3.0)
    plan.set_depth_response(al, far)
    assert plan.workspace_bytes(pget.OP_LM, 1) > ws0
    f_r, _, _ = plan.lm_solve(y, f0, m0, prm)
    other = pget.Plan(n, na, nb)
    other.set_depth_response(al, far)
    f_ref, _, _ = other.lm_solve(y, f0, m0, prm)
    assert torch.equal(f_r, f_ref)          # not the earlier captured sequence
    assert not torch.equal(f_r, f_plain)
    plan.set_depth_response(None)
    assert plan.workspace_bytes(pget.OP_LM, 1) == ws0
    assert torch.equal(plan.forward(T(f), T(mu)), y_plain)
    f_back, _, _ = plan.lm_solve(y, f0, m0, prm)
    assert torch.equal(f_back, f_plain)


def test_bad_depth_response_rejected():
    plan = pget.Plan(16, 12, 24)
    n_t, K = plan.n_samples, plan.psf_half_width
    al, far = inputs.collimator_depth_response(n_t, K, 2.0)
    for a, t in [(al[:-1], far), (al, far[:-1]), (al[:-1] + (1.5,), far), (al[:-1] + (float("nan"),), far),
                 (al, far[:-1] + (far[-1] * 2,)), (al, far[:-1] + (float("inf"),))]:
        with pytest.raises(pget.PgetError) as e:
            plan.set_depth_response(a, t)
        assert e.value.status == -1
    bf = pget.Plan(16, 12, 24, storage="bf16")
    with pytest.raises(pget.PgetError) as e:
        bf.set_depth_response(al, far)
    assert e.value.status == -5
    # 8192 bins: three rows of sums per angle slot exceed a J v block's LDS;
    # the plan is refused the response and keeps working without it
    wide = pget.Plan(16, 8, 8192)
    aw, fw = inputs.collimator_depth_response(wide.n_samples, wide.psf_half_width, 2.0)
    with pytest.raises(pget.PgetError) as e:
        wide.set_depth_response(aw, fw)
    assert e.value.status == -5
    f = torch.ones((16, 16), device="cuda")
    y = wide.forward(f, torch.zeros_like(f))
    assert torch.isfinite(y).all() and float(y.sum()) > 0


def test_hook_with_full_model_matches_oracle():
    """The learned step's safeguard under the full discrete model: a hook
    that moves halfway from the LM trial point to the phantom, on the GPU and
    in the oracle (same decisions replayed): the same proposals kept, and
    m(0) - m(s~) and rho(s~) of every proposal within the tolerance of the
    maps (the proposals follow the FP32 iterates)."""
    cfg = lattice_case()
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    d, al, far = full_model(plan)
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, depth=d, resp=al, far_taps=far)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(og, y)
    p = OLM.LMParams(max_outer=6, n_cg=6)

    def blend_np(f, mu, sf, sm):
        return (f + sf + 0.5 * (f_true - (f + sf)), mu + sm + 0.5 * (mu_true - (mu + sm)))

    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p, hook=blend_np)
    ft, mt = T(f_true), T(mu_true)

    def blend(f, mu, sf, sm):
        return (f + sf + 0.5 * (ft - (f + sf)), mu + sm + 0.5 * (mt - (mu + sm)))

    plan.set_depth_factor(d)
    plan.set_depth_response(al, far)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(max_outer=6, n_cg=6, replay=orep.accepted),
                              hook=blend)
    rep = rb.to_report()
    log("hook kept %s (oracle %s); maps f %.1e mu %.1e" % (rep.hook_accepted, orep.hook_accepted,
                                                          rel(H(f), of), rel(H(mu), om)))
    assert rep.hook_accepted == orep.hook_accepted
    assert rel(H(f), of) <= 1e-3 and rel(H(mu), om) <= 1e-3
    assert np.array_equal(np.isnan(rep.hook_pred), np.isnan(orep.hook_pred))
    for a, b in zip(rep.hook_pred, orep.hook_pred):
        if not np.isnan(b):
            assert abs(a - b) <= 1e-3 * abs(b)
    for a, b in zip(rep.hook_rho, orep.hook_rho):
        if not np.isnan(b) and np.isfinite(b):
            assert abs(a - b) <= 1e-3 * max(1.0, abs(b))


def test_autotune_with_depth_response_keeps_results():
    """The autotuner times the depth-response kernels within their own LDS
    limit (three rows of sums per angle slot, alpha in LDS); the tuned shapes
    change no bit of the result."""
    n, na, nb = 64, 120, 96
    plan = pget.Plan(n, na, nb)
    d, al, far = full_model(plan)
    plan.set_depth_factor(d)
    plan.set_depth_response(al, far)
    og = O.Geometry(n, na, nb, depth=d, resp=al, far_taps=far)
    f_true, mu_true = phantom(n, 5)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), 1e4, 5)
    f0, mu0 = OLM.initial_guess(og, y)
    prm = pget.SolverParams(max_outer=3, n_cg=5)
    ys, f0s, m0s = [T(y)] * 4, [T(f0)] * 4, [T(mu0)] * 4
    fa, ma, _ = plan.lm_solve_batched(ys, f0s, m0s, [prm] * 4)
    shape = plan.autotune(4)
    log("tuned shape with the depth response: %s" % shape)
    assert shape["tuned"] and shape["jvp_angle_slots"] >= 1 and shape["vjp_angle_groups"] >= 1
    fb, mb, _ = plan.lm_solve_batched(ys, f0s, m0s, [prm] * 4)
    for k in range(4):
        assert torch.equal(fb[k], fa[k]) and torch.equal(mb[k], ma[k])


def test_graph_replay_with_full_model_matches_eager():
    """The captured solver sequence of the full discrete model (the far
    planes and the far prefix sums cleared by fill kernels, not memsets)
    replayed several times with eager work in between gives the eager result
    bit for bit, batched."""
    cfg = lattice_case()
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    d, al, far = full_model(plan)
    plan.set_depth_factor(d)
    plan.set_depth_response(al, far)
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, depth=d, resp=al, far_taps=far)
    ys, f0s, m0s = [], [], []
    for seed in range(3):
        f_true, mu_true = inputs.rod_lattice(cfg, seed)
        y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, seed)
        f0, mu0 = OLM.initial_guess(og, y)
        ys.append(T(y))
        f0s.append(T(f0))
        m0s.append(T(mu0))
    prm = [pget.SolverParams(max_outer=4, n_cg=5, w_mu=0.05 ** 2, active_set=1)] * 3
    pget.set_graphs(False)
    try:
        fe, me, _ = plan.lm_solve_batched(ys, f0s, m0s, prm)
    finally:
        pget.set_graphs(True)
    for rep_i in range(3):
        fg, mg, _ = plan.lm_solve_batched(ys, f0s, m0s, prm)
        for k in range(3):
            assert torch.equal(fg[k], fe[k]) and torch.equal(mg[k], me[k]), (rep_i, k)
        plan.forward(f0s[0], m0s[0])
        torch.cuda.synchronize()


def test_single_tap_response_is_a_depth_gain():
    """Without a blur (one tap) the response is a gain per sample,
    (1 - alpha_i) + alpha_i * far: here 1 at the detector side falling to 0.5
    at the far side.  Operators against the oracle."""
    n, na, nb = 32, 40, 48
    plan = pget.Plan(n, na, nb, psf_sigma=0.0)
    assert plan.psf_half_width == 0
    n_t = plan.n_samples
    al = tuple(1.0 - i / (n_t - 1) for i in range(n_t))
    plan.set_depth_response(al, (0.5,))
    og = O.Geometry(n, na, nb, psf_sigma=0.0, resp=al, far_taps=(0.5,))
    f, mu = phantom(n, 6)
    rng = np.random.default_rng(8)
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    y, y_ref = H(plan.forward(T(f), T(mu))), O.forward(og, f, mu)
    jv, jv_ref = H(plan.jvp(T(f), T(mu), T(vf), T(vm))), O.jvp(og, f, mu, vf, vm)
    gf, gm = plan.vjp(T(f), T(mu), T(w))
    gf_ref, gm_ref = O.vjp(og, f, mu, w)
    errs = (rel(y, y_ref), rel(jv, jv_ref), rel(H(gf), gf_ref), rel(H(gm), gm_ref))
    log("one tap: forward %.2e jvp %.2e vjp f %.2e mu %.2e" % errs)
    assert max(errs) <= 1e-5
    assert rel(y, O.forward(O.Geometry(n, na, nb, psf_sigma=0.0), f, mu)) > 1e-2
