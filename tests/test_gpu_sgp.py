"""The damped step by scaled gradient projection (PGET_STEP_SGP; Sec. 2.2)
on the GPU against the FP64 oracle's SGP.

* A small slice with binding box bounds, the oracle's accept decisions
  replayed: objective per iterate within 1e-4 relative, the step's model
  value q(s) after each SGP iteration of the first outer iteration within
  1e-4 of its start, maps within 1e-3 (the same bounds as the CG step's
  trajectory tests; SGP's line search and steplength choices are discrete
  decisions taken in FP64 on FP32 sums, as the CG's are not).
* Step-by-step at the GPU's own iterates on the 128^2 benchmark slice
  (slice 0 of a batch of 64): Phi, ||g||, pred, ared, rho as for the CG
  step (tests/test_gpu_stepwise.py), and the SGP solve from the GPU's first
  iterate against the oracle's within its own spread.
* Alone == in a batch, bitwise.
* The comparison with the active-set CG at equal operator products on the
  benchmark slice (15 outer x 30): both decrease the objective; the printed
  values are the design notes' comparison.
"""
import os
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

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_stepwise import run_stepwise  # noqa: E402

SMALL = inputs.SliceConfig("lattice3_n24", 24, 36, 36, n_rods=3, rod_radius=2.0, pitch=6.0,
                           can_half=10.0, n_empty=1, max_outer=6, n_cg=8)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_sgp_trajectory_matches_oracle_with_binding_bounds():
    cfg = SMALL
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(og, y)
    box = dict(f_hi=0.7 * float(f_true.max()), mu_hi=0.04)
    op = OLM.LMParams(max_outer=6, n_cg=8, w_mu=0.05 ** 2, d_mu=400.0, step="sgp", **box)
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, op)
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    prm = pget.SolverParams(max_outer=6, n_cg=8, w_mu=0.05 ** 2, d_mu=400.0, step=pget.STEP_SGP,
                            replay=orep.accepted, **box)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), prm)
    rep = rb.to_report()
    errs = [abs(a / b - 1) for a, b in zip(rep.phi, orep.phi)]
    q_err = [abs(a - b) / abs(orep.cg_rr[0][-1]) for a, b in zip(rep.cg_rr[0], orep.cg_rr[0])]
    log("SGP: phi rel err per iterate %s; q(s) per SGP step (iteration 0) %s; maps f %.1e mu %.1e; "
        "decisions %s" % (" ".join("%.1e" % e for e in errs), " ".join("%.0e" % e for e in q_err),
                          rel(f.cpu().numpy(), of), rel(mu.cpu().numpy(), om), orep.accepted))
    assert max(errs) <= 1e-4 and max(q_err) <= 1e-4
    assert rel(f.cpu().numpy(), of) <= 1e-3 and rel(mu.cpu().numpy(), om) <= 1e-3
    # the box binds, and every returned value lies in it (the kernels take
    # the bounds rounded to FP32)
    f_hi, mu_hi = float(np.float32(box["f_hi"])), float(np.float32(box["mu_hi"]))
    assert float(mu.max()) <= mu_hi and float(f.max()) <= f_hi and float(mu.min()) >= 0.0
    assert float(mu.max()) == mu_hi or float(f.max()) == f_hi


def _main_batch(plan, cfg):
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(og, y)
    ones = torch.ones((cfg.n, cfg.n), device="cuda")
    a1 = plan.forward(ones, torch.zeros_like(ones)).double()
    ys, f0s, m0s = [T(y)], [T(f0)], [T(mu0)]
    for s_ in range(1, 64):
        f, mu = inputs.rod_lattice(cfg, s_)
        yc = plan.forward(T(f), T(mu)).double().cpu().numpy()
        ys_ = T(inputs.poisson_counts(yc, cfg.peak_counts, s_))
        c0 = float((a1 * ys_.double()).sum() / (a1 * a1).sum())
        ys.append(ys_)
        f0s.append(torch.full_like(ones, c0))
        m0s.append(torch.zeros_like(ones))
    return og, y, ys, f0s, m0s


def test_sgp_stepwise_and_batch_invariance_on_the_benchmark_slice():
    cfg = inputs.MAIN_128
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    og, y, ys, f0s, m0s = _main_batch(plan, cfg)
    w_mu = 0.05 ** 2
    base = dict(max_outer=6, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, w_mu=w_mu, d_mu=1 / w_mu,
                step=pget.STEP_SGP)
    op = OLM.LMParams(max_outer=6, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, w_mu=w_mu,
                      d_mu=1 / w_mu, step="sgp")
    rep, cg_errs = run_stepwise(og, y, plan, ys, f0s, m0s, base, op, cg_iters=(0,))
    for e, spread in cg_errs:
        assert e <= max(1e-4, 5 * spread)
    fa, ma, _ = plan.lm_solve(ys[0], f0s[0], m0s[0], pget.SolverParams(**base))
    fb, mb, _ = plan.lm_solve_batched(ys[:4], f0s[:4], m0s[:4], [pget.SolverParams(**base)] * 4)
    assert torch.equal(fa, fb[0]) and torch.equal(ma, mb[0])


def test_sgp_against_active_set_cg_at_equal_operator_products():
    cfg = inputs.MAIN_128
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    og, y, ys, f0s, m0s = _main_batch(plan, cfg)
    w_mu = 0.05 ** 2
    base = dict(max_outer=15, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, w_mu=w_mu, d_mu=1 / w_mu)
    res = {}
    for name, extra in (("active-set CG", dict(active_set=1)), ("SGP", dict(step=pget.STEP_SGP))):
        fs, ms, rbs = plan.lm_solve_batched(ys[:16], f0s[:16], m0s[:16], [pget.SolverParams(**base, **extra)] * 16)
        reps = [r.to_report() for r in rbs]
        res[name] = (np.median([r.phi[-1] / r.phi[0] for r in reps]), np.mean([sum(r.accepted) for r in reps]))
        assert all(r.status == 0 and r.phi[-1] < r.phi[0] for r in reps)
    log("128^2, 15 outer x 30 operator products, 16 slices: final / initial Phi (median) and accepted steps "
        "(mean): %s" % {k: ("%.3e" % v[0], "%.1f" % v[1]) for k, v in res.items()})
