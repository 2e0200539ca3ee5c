"""GPU parity of the block-scaled CG and the active set of the damped step
(solver options w_f, w_mu, active_set) and of the geometry prior (prior_w,
prior_ref, with and without continuation) against the FP64 oracle, with the
oracle's accept decisions replayed (as in test_gpu_lm).

With the scaled metric the LM steps are large and the trajectory becomes
sensitive to rounding as the CG count grows: the FP64 oracle itself, with
every operator product perturbed by 1e-6 relative noise (FP32 level), moves
Phi by up to 2e-2 and the maps by 3-7 % after a few iterations of a 64 x 64
solve with 20 CG steps, while with 4 CG steps on a 24 x 24 slice the spread
stays below 1e-5.  So:

* trajectory parity (24 x 24, 4 CG steps, 6 outer iterations): objective per
  iteration 1e-4 relative, predicted decrease and beta 1e-3, maps 1e-3
  relative L2, CG trace r^T W r 1e-3 of its start;
* at the 64 x 64 workload (20 CG steps, 3 outer iterations): the first
  linearisation tightly (objective 1e-6, gradient norm 1e-5, the first
  three CG residuals 1e-3 of the start), then the objective per iteration
  and the maps within five times the spread of two perturbed oracle solves,
  and at least as close as 1e-4 / 1e-3.

The free-variable mask is an FP32 decision on the sign of the gradient at
pixels on a bound; pixels outside every ray have an exact zero gradient on
both sides.
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


SMALL = inputs.SliceConfig("lattice3_n24", 24, 36, 36, n_rods=3, rod_radius=2.0, pitch=6.0,
                           can_half=10.0, n_empty=1, max_outer=6, n_cg=4)
W_MU = 0.05 ** 2       # attenuation scale 0.05 against emission scale 1


def problem(cfg, seed=0):
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(cfg, seed)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, seed)
    f0, mu0 = OLM.initial_guess(og, y)
    return og, y, f0, mu0


def compare(rep, orep, f, mu, of, om, tol_phi=1e-4, tol_map=1e-3):
    assert rep.iters_run == orep.iters_run
    assert rep.accepted == orep.accepted
    for k in range(rep.iters_run):
        e = abs(rep.phi[k] - orep.phi[k]) / orep.phi[k]
        log("k=%d phi %.8g / %.8g (%.1e) pred %.5g / %.5g beta %.4g / %.4g acc %d" % (
            k, rep.phi[k], orep.phi[k], e, rep.pred[k], orep.pred[k], rep.beta[k], orep.beta[k],
            rep.accepted[k]))
        assert e <= tol_phi
        assert abs(rep.beta[k] - orep.beta[k]) <= 1e-3 * orep.beta[k]
        assert abs(rep.gnorm[k] - orep.gnorm[k]) <= 1e-4 * orep.gnorm[k]
        if np.isfinite(orep.pred[k]) and orep.pred[k] > 0:
            assert abs(rep.pred[k] - orep.pred[k]) <= 1e-3 * abs(orep.pred[k])
    assert abs(rep.phi[-1] - orep.phi[-1]) <= tol_phi * orep.phi[-1]
    log("maps rel L2: f %.2e mu %.2e" % (rel(H(f), of), rel(H(mu), om)))
    assert rel(H(f), of) <= tol_map
    assert rel(H(mu), om) <= tol_map


@pytest.mark.parametrize("active", [0, 1], ids=["scaled", "scaled_active"])
def test_small_trajectory_with_replay(active):
    og, y, f0, mu0 = problem(SMALL)
    p = OLM.LMParams(max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=bool(active))
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p)
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(
        max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=active, replay=orep.accepted))
    rep = rb.to_report()
    assert rep.status == 0
    compare(rep, orep, f, mu, of, om)
    for m in range(SMALL.n_cg):
        assert abs(rep.cg_rr[0][m] - orep.cg_rr[0][m]) <= 1e-3 * orep.cg_rr[0][0]
    if active:
        # the active set keeps every step of this solve (Phi falls ~100x)
        assert all(orep.accepted) and orep.phi[-1] < 0.02 * orep.phi[0]


def _perturbed_solve(monkeypatch, og, y, f0, mu0, p, replay, seed):
    """The oracle's solve with every normal-operator product multiplied by
    (1 + 1e-6 N(0, 1)) elementwise: the spread of FP32-level rounding."""
    rng = np.random.default_rng(seed)
    plain = OLM.cg

    def cg_noisy(matvec, bf, bm, n, wf=1.0, wm=1.0):
        def mv(a, b):
            qa, qb = matvec(a, b)
            return qa * (1 + 1e-6 * rng.standard_normal(qa.shape)), qb * (1 + 1e-6 * rng.standard_normal(qb.shape))
        return plain(mv, bf, bm, n, wf, wm)
    monkeypatch.setattr(OLM, "cg", cg_noisy)
    try:
        return OLM.lm_solve(og, y, f0, mu0, p, replay=replay)
    finally:
        monkeypatch.setattr(OLM, "cg", plain)


def test_64_workload_within_rounding_spread(monkeypatch):
    cfg = inputs.SMALL_64
    og, y, f0, mu0 = problem(cfg)
    p = OLM.LMParams(max_outer=3, n_cg=cfg.n_cg, w_mu=W_MU, active_set=True)
    log("oracle LM 64x64, 3 outer x %d CG, scaled, active set (+2 perturbed solves)" % cfg.n_cg)
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p)
    spread_phi = np.zeros(len(orep.phi))
    spread_f = spread_m = 0.0
    for seed in (1, 2):
        pf, pm, prep = _perturbed_solve(monkeypatch, og, y, f0, mu0, p, orep.accepted, seed)
        spread_phi = np.maximum(spread_phi, np.abs(np.array(prep.phi) / np.array(orep.phi) - 1))
        spread_f, spread_m = max(spread_f, rel(pf, of)), max(spread_m, rel(pm, om))
    log("oracle spread: phi %s maps %.1e %.1e" % (" ".join("%.1e" % v for v in spread_phi), spread_f, spread_m))
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(
        max_outer=3, n_cg=cfg.n_cg, w_mu=W_MU, active_set=1, replay=orep.accepted))
    rep = rb.to_report()
    assert rep.accepted == orep.accepted
    # the first linearisation is common to both and well conditioned
    assert abs(rep.phi[0] - orep.phi[0]) <= 1e-6 * orep.phi[0]
    assert abs(rep.gnorm[0] - orep.gnorm[0]) <= 1e-5 * orep.gnorm[0]
    for m in range(3):
        assert abs(rep.cg_rr[0][m] - orep.cg_rr[0][m]) <= 1e-3 * orep.cg_rr[0][0]
    for k in range(1, len(orep.phi)):
        e = abs(rep.phi[k] - orep.phi[k]) / orep.phi[k]
        log("k=%d phi %.8g / %.8g (%.1e, bound %.1e)" % (k, rep.phi[k], orep.phi[k], e, max(1e-4, 5 * spread_phi[k])))
        assert e <= max(1e-4, 5 * spread_phi[k])
    ef, em = rel(H(f), of), rel(H(mu), om)
    log("maps rel L2: f %.2e (bound %.1e) mu %.2e (bound %.1e)" % (ef, max(1e-3, 5 * spread_f), em, max(1e-3, 5 * spread_m)))
    assert ef <= max(1e-3, 5 * spread_f) and em <= max(1e-3, 5 * spread_m)


def test_mixed_options_in_one_batch_equal_alone():
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    prms = [pget.SolverParams(max_outer=4, n_cg=6),
            pget.SolverParams(max_outer=4, n_cg=6, w_mu=W_MU, active_set=1),
            pget.SolverParams(max_outer=4, n_cg=6, w_f=2.0, w_mu=W_MU)]
    ys, f0s, m0s = [], [], []
    for i in range(3):
        og, y, f0, mu0 = problem(SMALL, seed=i)
        ys.append(T(y)); f0s.append(T(f0)); m0s.append(T(mu0))
    fs, ms, rbs = plan.lm_solve_batched(ys, f0s, m0s, prms)
    for i in range(3):
        fa, ma, ra = plan.lm_solve(ys[i], f0s[i], m0s[i], prms[i])
        assert torch.equal(fa, fs[i]) and torch.equal(ma, ms[i])
        assert ra.to_report().phi == rbs[i].to_report().phi


def test_invalid_options_rejected():
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    og, y, f0, mu0 = problem(SMALL)
    for bad in (dict(w_f=-1.0), dict(w_mu=float("nan")), dict(active_set=2)):
        with pytest.raises(pget.PgetError):
            plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(max_outer=2, n_cg=2, **bad))


def test_unit_scaling_is_plain_cg():
    """w = 1 (or 0, read as 1) with the active set off runs plain CG: the
    result is bitwise that of the default parameters."""
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    og, y, f0, mu0 = problem(SMALL, seed=2)
    f1, m1, _ = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(max_outer=3, n_cg=6))
    f2, m2, _ = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(max_outer=3, n_cg=6, w_f=0.0, w_mu=0.0))
    assert torch.equal(f1, f2) and torch.equal(m1, m2)


def _prior(n, seed):
    rng = np.random.default_rng(seed)
    wf = rng.uniform(0.0, 5.0, (n, n)) * (rng.uniform(size=(n, n)) < 0.5)
    wm = rng.uniform(0.0, 500.0, (n, n)) * (rng.uniform(size=(n, n)) < 0.5)
    return wf, wm, rng.uniform(0.0, 0.5, (n, n)), rng.uniform(0.0, 0.02, (n, n))


def _prior_dev(pr):
    wf, wm, rf, rm = pr
    return T(np.stack([wf, wm])), T(np.stack([rf, rm]))


@pytest.mark.parametrize("decay", [1.0, 5.0], ids=["fixed", "continuation"])
def test_prior_trajectory_with_replay(decay):
    """The geometry prior (per-pixel weights and references) with the scaled
    active-set step, 4 CG steps, and the alphas and prior weights divided by
    5 per iteration for 3 iterations in the continuation case."""
    og, y, f0, mu0 = problem(SMALL)
    pr = _prior(SMALL.n, 21)
    p = OLM.LMParams(max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=True,
                     alpha_decay=decay, alpha_decay_until=3,
                     prior_w_f=pr[0], prior_w_mu=pr[1], prior_ref_f=pr[2], prior_ref_mu=pr[3])
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p)
    pw, pref = _prior_dev(pr)
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(
        max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=1, alpha_decay=decay,
        alpha_decay_until=3, prior_w=pw, prior_ref=pref, replay=orep.accepted))
    rep = rb.to_report()
    assert rep.status == 0
    compare(rep, orep, f, mu, of, om)
    # the prior moved the solution: without it the oracle ends elsewhere
    of2, om2, _ = OLM.lm_solve(og, y, f0, mu0, OLM.LMParams(
        max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=True, alpha_decay=decay,
        alpha_decay_until=3))
    assert rel(of2, of) > 1e-2


def test_prior_in_batch_equal_alone_and_checked():
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    pa, pb = _prior_dev(_prior(SMALL.n, 22)), _prior_dev(_prior(SMALL.n, 23))
    base = dict(max_outer=4, n_cg=4, w_mu=W_MU, active_set=1)
    prms = [pget.SolverParams(**base), pget.SolverParams(prior_w=pa[0], prior_ref=pa[1], **base),
            pget.SolverParams(prior_w=pb[0], **base)]
    ys, f0s, m0s = [], [], []
    for i in range(3):
        og, y, f0, mu0 = problem(SMALL, seed=i)
        ys.append(T(y)); f0s.append(T(f0)); m0s.append(T(mu0))
    fs, ms, rbs = plan.lm_solve_batched(ys, f0s, m0s, prms)
    for i in range(3):
        fa, ma, ra = plan.lm_solve(ys[i], f0s[i], m0s[i], prms[i])
        assert torch.equal(fa, fs[i]) and torch.equal(ma, ms[i])
    with pytest.raises(ValueError):
        plan.lm_solve(ys[0], f0s[0], m0s[0], pget.SolverParams(prior_w=pa[0][:1], **base))
    with pytest.raises(ValueError):
        plan.lm_solve(ys[0], f0s[0], m0s[0], pget.SolverParams(prior_w=pa[0].double(), **base))


def test_upper_bounds_with_replay():
    """Box constraints with finite upper bounds that bind within the six
    iterations (emission at 0.7 of the phantom's peak, attenuation at 0.004,
    below what the unbounded solve reaches): the clamp and the active set act
    at the upper bound too (8 and 25 pixels end on it in the oracle's run).
    Decisions replayed from the oracle; tolerances as for the other
    trajectories."""
    og, y, f0, mu0 = problem(SMALL)
    f_true, _ = inputs.rod_lattice(SMALL, 0)
    f_hi, mu_hi = 0.7 * float(f_true.max()), 0.004
    p = OLM.LMParams(max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=True,
                     f_hi=f_hi, mu_hi=mu_hi)
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p)
    assert (of == f_hi).sum() >= 4 and (om == mu_hi).sum() >= 4     # both upper bounds bind
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), pget.SolverParams(
        max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=W_MU, active_set=1, f_hi=f_hi, mu_hi=mu_hi,
        replay=orep.accepted))
    rep = rb.to_report()
    assert rep.status == 0
    compare(rep, orep, f, mu, of, om)
    assert float(f.max()) <= np.float32(f_hi) and float(mu.max()) <= np.float32(mu_hi)
