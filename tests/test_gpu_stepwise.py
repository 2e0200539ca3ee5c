"""Step-by-step parity of the LM solver at the GPU's own iterates.

The benchmark's configuration (scaled damping and CG with the active set,
15 outer x 30 CG steps) on slice 0 of a batch of 64, free running (no
replayed decisions).  The solver records every outer iteration's iterate
u_k and trial point u'_k (the parameters' iterate trace); the FP64 oracle
then evaluates, at those same FP32 points, the quantities the gain-ratio
test uses (Sec. 2.2 eq. m-function, Sec. 3.1 eq. rho_agreement): Phi(u_k),
||g(u_k)||, pred(s_k) with s_k = u'_k - u_k, ared = Phi(u_k) - Phi(u'_k)
and rho, and whether the test accepts.  Errors of the trajectory do not
compound here: each iteration is checked from where the GPU stands.

Bounds, from the arithmetic:
* Phi and ||g||: 1e-5 relative (the FP32 operators' bound; the sums are
  FP64).
* pred: 1e-4 relative (||J s||^2 from an FP32 product, g.s and s.R s from
  FP32 vectors, all summed in FP64).
* ared: Phi(u) and Phi(u') each carry the FP32 residual's rounding, about
  1e-7 of Phi, so |ared_gpu - ared| <= 1e-4 |ared| + 1e-6 Phi; rho then
  within the same bound divided by pred.
* the decision: equal to the oracle's rho > eta wherever rho - eta exceeds
  that bound.
At two iterations the oracle also runs the whole CG solve from the GPU's
u_k and damping beta_k; the trial points agree to the stated relative L2
bound (CG in FP32 over 30 steps amplifies rounding by the system's
condition; the oracle's own spread under 1e-6 perturbations is of the same
order).
"""
import dataclasses
import multiprocessing as mp
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

GOLDEN_SCANNER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                              "scanner9x9_n165_scaled_oracle.npz")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def run_stepwise(og, y, plan, ys, f0s, m0s, base, op, cg_iters):
    """Solve the batch with slice 0 traced, then check every iteration of
    slice 0 against the oracle evaluated at the GPU's iterates."""
    n, K = og.n, base["max_outer"]
    tu = torch.zeros((K, 2, n, n), dtype=torch.float32, device="cuda")
    tt = torch.zeros_like(tu)
    prm = [pget.SolverParams(trace_u=tu, trace_t=tt, **base)] + [pget.SolverParams(**base)] * (len(ys) - 1)
    log("GPU solve: batch of %d, %d x %d" % (len(ys), K, base["n_cg"]))
    fs, ms, rbs = plan.lm_solve_batched(ys, f0s, m0s, prm)
    rep = rbs[0].to_report()
    U, Ut = tu.double().cpu().numpy(), tt.double().cpu().numpy()
    kw = dataclasses.asdict(og)
    jobs = [(kw, y, U[k, 0], U[k, 1], Ut[k, 0], Ut[k, 1], op, k, None, None) for k in range(rep.iters_run)]
    # the CG solve from the GPU's iterate and damping: exact, and twice with
    # its operator products perturbed at FP32 size (its own spread)
    jobs += [(kw, y, U[k, 0], U[k, 1], None, None, op, k, rep.beta[k], seed) for k in cg_iters
             for seed in (None, 1, 2)]
    log("oracle: %d step evaluations and %d CG solves" % (rep.iters_run, 3 * len(cg_iters)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(len(jobs), 12)) as pool:
        res = pool.map(OLM.step_quantities_job, jobs)
    q, cg = res[:rep.iters_run], res[rep.iters_run:]
    rows, worst = [], {"phi": 0.0, "gnorm": 0.0, "pred": 0.0, "ared": 0.0, "rho": 0.0}
    for k in range(rep.iters_run):
        o = q[k]
        e_phi = abs(rep.phi[k] / o["phi"] - 1)
        e_g = abs(rep.gnorm[k] / o["gnorm"] - 1)
        e_pred = abs(rep.pred[k] / o["pred"] - 1)
        ared_bound = 1e-4 * abs(o["ared"]) + 1e-6 * o["phi"]
        e_ared = abs(rep.ared[k] - o["ared"]) / ared_bound
        rho_bound = ared_bound / o["pred"] + 1e-4 * abs(o["rho"]) if o["pred"] > 0 else np.inf
        e_rho = abs(rep.rho[k] - o["rho"]) / rho_bound if np.isfinite(o["rho"]) else 0.0
        rows.append("k=%2d phi %.1e  |g| %.1e  pred %.1e  ared %.2e (%.2f of bound)  rho %.4f vs %.4f  acc %d"
                    % (k, e_phi, e_g, e_pred, abs(rep.ared[k] - o["ared"]) / max(abs(o["ared"]), 1e-300),
                       e_ared, rep.rho[k], o["rho"], rep.accepted[k]))
        assert e_phi <= 1e-5, rows[-1]
        assert e_g <= 1e-5, rows[-1]
        assert e_pred <= 1e-4, rows[-1]
        assert e_ared <= 1.0, rows[-1]
        assert e_rho <= 1.0, rows[-1]
        if abs(o["rho"] - op.eta) > rho_bound:
            assert bool(rep.accepted[k]) == bool(o["rho"] > op.eta), rows[-1]
        for key, v in (("phi", e_phi), ("gnorm", e_g), ("pred", e_pred), ("ared", e_ared), ("rho", e_rho)):
            worst[key] = max(worst[key], v)
    log("\n".join(rows))
    log("worst: phi %.1e, |g| %.1e, pred %.1e, ared %.2f and rho %.2f of their bounds" % (
        worst["phi"], worst["gnorm"], worst["pred"], worst["ared"], worst["rho"]))
    cg_errs = []
    step = lambda ft, mt, k: np.concatenate([(ft - U[k, 0]).ravel(), (mt - U[k, 1]).ravel()])
    for i, k in enumerate(cg_iters):
        exact, p1, p2 = cg[3 * i: 3 * i + 3]
        s_ora = step(exact["f_trial"], exact["mu_trial"], k)
        e_gpu = rel(step(Ut[k, 0], Ut[k, 1], k), s_ora)
        spread = max(rel(step(c["f_trial"], c["mu_trial"], k), s_ora) for c in (p1, p2))
        rr_g, rr_o = rep.cg_rr[k], exact["cg_rr"]
        rr_e = [abs(a / b - 1) for a, b in zip(rr_g, rr_o)]
        cg_errs.append((e_gpu, spread))
        log("k=%d: step of the CG solve from the GPU's iterate and beta: rel L2 %.2e (oracle's own spread "
            "under 1e-6 perturbations %.2e); r.W r per CG step rel err %s" % (
                k, e_gpu, spread, " ".join("%.0e" % e for e in rr_e[:8])))
    return rep, cg_errs


def test_stepwise_lattice9_n128_scaled_slice_of_batch64():
    cfg = inputs.MAIN_128
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(og, y)
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
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
    w_mu = 0.05 ** 2
    base = dict(max_outer=15, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, w_mu=w_mu, d_mu=1 / w_mu,
                active_set=1)
    op = OLM.LMParams(max_outer=15, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, w_mu=w_mu,
                      d_mu=1 / w_mu, active_set=True)
    rep, cg_errs = run_stepwise(og, y, plan, ys, f0s, m0s, base, op, cg_iters=(0, 7))
    assert rep.iters_run == 15
    for e, spread in cg_errs:
        assert e <= max(1e-4, 5 * spread)


def test_stepwise_scanner_scaled_slice_of_batch64():
    if not os.path.exists(GOLDEN_SCANNER):
        pytest.skip("stored scanner slice not present")
    ref = np.load(GOLDEN_SCANNER)
    CFG = inputs.SCANNER_165

    def geoms(oversample):
        d = inputs.scanner_geometry(CFG, oversample)
        og = O.Geometry(d["n"], d["n_angles"], d["n_bins"], bin_size=d["bin_size"], step=d["step"],
                        psf_sigma=d["psf_sigma"], atten_scale=d["atten_scale"])
        pl = pget.Plan(d["n"], d["n_angles"], d["n_bins"], bin_size=d["bin_size"], step=d["step"],
                       psf_sigma=d["psf_sigma"], atten_scale=d["atten_scale"])
        return og, pl

    og, pl = geoms(1)
    fine = geoms(2)[1]
    fscale = inputs.scanner_geometry(CFG, 2)["y_scale"] / inputs.scanner_geometry(CFG, 1)["y_scale"]
    kinds = ("full", "missing", "replaced", "medium")
    y = ref["y"]
    ys, f0s, m0s = [T(y)], [T(ref["f0"])], [T(ref["mu0"])]
    one = torch.ones((CFG.n, CFG.n), device="cuda")
    a1 = pl.forward(one, torch.zeros_like(one)).double()
    for s_ in range(1, 64):
        ff, mf = inputs.scanner_phantom(CFG, s_, kinds[s_ % 4], 2)
        yy = inputs.gaussian_noise(fscale * fine.forward(T(ff), T(mf)).double().cpu().numpy(), CFG.noise, s_)
        c0 = float((a1.cpu().numpy() * yy).sum() / (a1 * a1).sum().item())
        ys.append(T(yy))
        f0s.append(torch.full_like(one, c0))
        m0s.append(T(ref["mu0"]))
    w_mu, d_mu = float(ref["w_mu"]), float(ref["d_mu"])
    base = dict(max_outer=15, n_cg=CFG.n_cg, alpha_f=CFG.alpha, alpha_mu=CFG.alpha, w_mu=w_mu, d_mu=d_mu,
                active_set=1)
    op = OLM.LMParams(max_outer=15, n_cg=CFG.n_cg, alpha_f=CFG.alpha, alpha_mu=CFG.alpha, w_mu=w_mu, d_mu=d_mu,
                      active_set=True)
    rep, cg_errs = run_stepwise(og, y, pl, ys, f0s, m0s, base, op, cg_iters=(0, 7))
    assert rep.iters_run == 15
    for e, spread in cg_errs:
        assert e <= max(1e-4, 5 * spread)
