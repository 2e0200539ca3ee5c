"""FP64 Levenberg-Marquardt solver of the oracle (test infrastructure only).

Follows Sec. 2.2 of the paper (eqs. linearized_prob, m-function, LMA-step) and
the safeguard of Sec. 3.1 (eq. rho_agreement, Prop. 3.2, Alg. 2), with the
readings where the paper is silent:

* objective  Phi(u) = 0.5*||A(u) - y||^2 + 0.5*alpha_f*||grad f||^2
                      + 0.5*alpha_mu*||grad mu||^2,  u = (f, mu);
  its gradient g = J^T (A(u) - y) + R u with R = diag(alpha_f L, alpha_mu L),
  L = grad^T grad.
* step       CG with x0 = 0 and a fixed number of steps on
             (J^T J + beta D + R) x = -g, D = diag(d_f I, d_mu I)
             (eq. LMA-step solved through its normal equations),
             preconditioned by W = diag(w_f I, w_mu I): the metric of the
             variables scaled by their typical magnitudes (the paper solves
             the constrained step by a scaled gradient projection, Sec. 2.2);
             W = I is plain CG.
* active set (option) a variable sitting on a bound whose gradient points
             out of the box is held at zero step: CG runs on the free
             variables, F (J^T J + beta D + R) F x = -F g, F the 0/1 mask of
             free variables.  Off: every variable is free.
* trial      u' = clamp(u + x) to the box constraints, s = u' - u.
* model      pred = m(0) - m(s) = -(g.s + 0.5*(||J s||^2 + s.R s))  (eq. m-function)
* gain ratio rho = (Phi(u) - Phi(u')) / pred  (eq. rho_agreement), -inf if pred <= 0;
             accept iff rho > eta.
* damping    Nielsen's rule: accept -> beta *= max(1/3, 1 - (2 rho - 1)^3), nu = 2;
             reject -> beta *= nu, nu *= 2.  beta0 = tau * ||J 1||^2 / ||1||^2
             unless given.
* hook       after an accepted step, u~ = G(u, s) replaces u' iff
             rho(u~ - u) > eta and m(u~ - u) <= m(s)  (Prop. 3.2, Alg. 2).
* continuation  alpha_k = alpha / decay**min(k, decay_until)  (Sec. 3.1).
* geometry prior (option; the paper's P1, P2 of Sec. 2.2, which penalise
             emission and attenuation outside the possible rod locations):
             + 0.5 * sum_m w_f[m] (f[m] - r_f[m])^2 + the same for mu, with
             per-pixel weights w >= 0 and references r given by the caller
             (e.g. w = gamma outside the rod disks, r_mu = water there);
             its Hessian diag(w) joins R, and it decays with the alphas.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import Geometry, forward, jvp, reg_energy, reg_gradient, vjp


@dataclass
class LMParams:
    max_outer: int = 15
    n_cg: int = 20
    alpha_f: float = 1e-2
    alpha_mu: float = 1e-2
    alpha_decay: float = 1.0
    alpha_decay_until: int = 0
    beta0: float = 0.0
    tau: float = 1e-3
    eta: float = 1e-3
    d_f: float = 1.0
    d_mu: float = 1.0
    f_lo: float = 0.0
    f_hi: float = np.inf
    mu_lo: float = 0.0
    mu_hi: float = np.inf
    tol: float = 0.0
    w_f: float = 1.0
    w_mu: float = 1.0
    active_set: bool = False
    # the damped step's solver: "cg" (CG on the normal equations, clamped
    # into the box) or "sgp" (the scaled gradient projection of the
    # box-constrained step, Sec. 2.2); n_cg is its number of iterations
    # (one normal-operator product each)
    step: str = "cg"
    prior_w_f: Optional[np.ndarray] = None
    prior_w_mu: Optional[np.ndarray] = None
    prior_ref_f: Optional[np.ndarray] = None
    prior_ref_mu: Optional[np.ndarray] = None


@dataclass
class LMReport:
    phi: List[float] = field(default_factory=list)
    rho: List[float] = field(default_factory=list)
    beta: List[float] = field(default_factory=list)
    pred: List[float] = field(default_factory=list)
    ared: List[float] = field(default_factory=list)
    gnorm: List[float] = field(default_factory=list)
    accepted: List[int] = field(default_factory=list)
    hook_accepted: List[int] = field(default_factory=list)
    hook_rho: List[float] = field(default_factory=list)    # rho(s~) of the proposal, NaN if none
    hook_pred: List[float] = field(default_factory=list)   # m(0) - m(s~), NaN if none
    cg_rr: List[List[float]] = field(default_factory=list)
    iters_run: int = 0
    beta_final: float = 0.0
    stop_reason: str = "max_outer"


def alphas_at(p: LMParams, k: int):
    decay = p.alpha_decay ** min(k, p.alpha_decay_until)
    return p.alpha_f / decay, p.alpha_mu / decay


def prior_at(p: LMParams, k: int):
    """(w_f, w_mu, r_f, r_mu) of the geometry prior at outer iteration k
    (weights divided by the same continuation factor as the alphas), or
    None when the solve has no prior.  A missing weight or reference map
    is zero."""
    if p.prior_w_f is None and p.prior_w_mu is None:
        return None
    shape = np.shape(p.prior_w_f if p.prior_w_f is not None else p.prior_w_mu)
    decay = p.alpha_decay ** min(k, p.alpha_decay_until)

    def as_map(a):
        return np.zeros(shape) if a is None else np.asarray(a, dtype=np.float64)
    return (as_map(p.prior_w_f) / decay, as_map(p.prior_w_mu) / decay,
            as_map(p.prior_ref_f), as_map(p.prior_ref_mu))


def objective(g: Geometry, y, f, mu, af, am, prior=None):
    """Phi(u) and the data residual A(u) - y."""
    r = forward(g, f, mu) - y
    phi = 0.5 * float(np.dot(r.ravel(), r.ravel())) + reg_energy(af, f) + reg_energy(am, mu)
    if prior is not None:
        wf, wm, rf, rm = prior
        phi += 0.5 * float(np.sum(wf * (f - rf) ** 2) + np.sum(wm * (mu - rm) ** 2))
    return phi, r


def gradient(g: Geometry, f, mu, r, af, am, prior=None):
    gf, gm = vjp(g, f, mu, r)
    gf, gm = gf + reg_gradient(af, f), gm + reg_gradient(am, mu)
    if prior is not None:
        wf, wm, rf, rm = prior
        gf, gm = gf + wf * (f - rf), gm + wm * (mu - rm)
    return gf, gm


def normal_matvec(g: Geometry, f, mu, pf, pm, beta, p: LMParams, af, am, prior=None):
    """(J^T J + beta D + R) [pf, pm]  (R includes the prior's diag(w))."""
    jp = jvp(g, f, mu, pf, pm)
    qf, qm = vjp(g, f, mu, jp)
    qf = qf + beta * p.d_f * pf + reg_gradient(af, pf)
    qm = qm + beta * p.d_mu * pm + reg_gradient(am, pm)
    if prior is not None:
        qf, qm = qf + prior[0] * pf, qm + prior[1] * pm
    return qf, qm


def cg(matvec: Callable, bf, bm, n_steps: int, wf: float = 1.0, wm: float = 1.0):
    """Conjugate gradients from x0 = 0 for a fixed number of steps,
    preconditioned by W = diag(wf I, wm I) (z = W r; W = I is plain CG).

    Returns (xf, xm, rr) where rr[m] is r^T W r after step m (the recurrence
    residual).  Stops early if p^T M p <= 0 or r^T W r == 0; the remaining
    rr entries then repeat the last value.
    """
    xf = np.zeros_like(bf)
    xm = np.zeros_like(bm)
    rf, rm = bf.copy(), bm.copy()
    pf, pm = wf * rf, wm * rm
    rr = float(np.sum(rf * pf) + np.sum(rm * pm))
    trace = []
    for _ in range(n_steps):
        if rr == 0.0:
            trace.append(rr)
            continue
        qf, qm = matvec(pf, pm)
        gamma = float(np.sum(pf * qf) + np.sum(pm * qm))
        if not gamma > 0.0:
            trace.append(rr)
            continue
        a = rr / gamma
        xf += a * pf
        xm += a * pm
        rf -= a * qf
        rm -= a * qm
        zf, zm = wf * rf, wm * rm
        rr_new = float(np.sum(rf * zf) + np.sum(rm * zm))
        pf = zf + (rr_new / rr) * pf
        pm = zm + (rr_new / rr) * pm
        rr = rr_new
        trace.append(rr)
    return xf, xm, trace


# Parameters of the scaled gradient projection (Bonettini, Zanella, Zanni,
# Inverse Problems 25 (2009) 015002, cited for the constrained step in
# Sec. 2.2): Armijo sufficient-decrease factor and backtracking ratio,
# steplength bounds, the alternation threshold of the two Barzilai-Borwein
# rules and its memory, and the first steplength.
SGP_ARMIJO = 1e-4
SGP_BACKTRACK = 0.4
SGP_ALPHA_MIN = 1e-10
SGP_ALPHA_MAX = 1e5
SGP_TAU0 = 0.5
SGP_MEMORY = 3
SGP_ALPHA0 = 1.0


def sgp(matvec: Callable, gf, gm, lo_f, hi_f, lo_m, hi_m, n_steps: int, wf: float = 1.0, wm: float = 1.0):
    """Scaled gradient projection for the box-constrained quadratic
    min q(s) = g.s + 0.5 s.M s over lo <= s <= hi (lo <= 0 <= hi), from
    s = 0, with the diagonal scaling D = diag(wf I, wm I) (the metric of the
    variables scaled by their typical magnitudes).  Each iteration:
      y = P_box(s - alpha D grad q(s)),  d = y - s;
      lambda = 1, times 0.4 until q(s + lambda d) <= q(s) + 1e-4 lambda grad q.d
        (q is quadratic: q(s + l d) - q(s) = l grad.d + l^2/2 d.M d);
      s += lambda d,  grad += lambda M d;
      the next alpha from the scaled Barzilai-Borwein rules with
        BB1 = d.D^-2 d / d.D^-1 M d,  BB2 = d.D M d / (M d).D^2 (M d)
        (s and grad changes are lambda d and lambda M d; lambda cancels):
      BB2 / BB1 <= tau: alpha = min of the last 3 BB2, tau *= 0.9;
      else alpha = BB1, tau *= 1.1; alpha clamped to [1e-10, 1e5].
    One product M d per iteration.  Returns (sf, sm, qvals): qvals[m] is
    q(s) after iteration m.  A zero direction (the projected gradient
    vanishes) leaves s unchanged."""
    sf = np.zeros_like(gf)
    sm = np.zeros_like(gm)
    rf, rm = np.array(gf, dtype=np.float64), np.array(gm, dtype=np.float64)   # grad q(s)
    alpha, tau = SGP_ALPHA0, SGP_TAU0
    bb2_hist: List[float] = []
    qv = 0.0
    trace = []
    for _ in range(n_steps):
        yf = np.clip(sf - alpha * wf * rf, lo_f, hi_f)
        ym = np.clip(sm - alpha * wm * rm, lo_m, hi_m)
        df, dm = yf - sf, ym - sm
        gd = float(np.sum(rf * df) + np.sum(rm * dm))
        if not gd < 0.0:
            trace.append(qv)
            continue
        qf, qm = matvec(df, dm)
        dMd = float(np.sum(df * qf) + np.sum(dm * qm))
        lam = 1.0
        while lam * gd + 0.5 * lam * lam * dMd > SGP_ARMIJO * lam * gd and lam > 1e-30:
            lam *= SGP_BACKTRACK
        sf, sm = sf + lam * df, sm + lam * dm
        rf, rm = rf + lam * qf, rm + lam * qm
        qv += lam * gd + 0.5 * lam * lam * dMd
        trace.append(qv)
        # the next steplength (scaled Barzilai-Borwein with alternation)
        den1 = float(np.sum(df * qf) / wf + np.sum(dm * qm) / wm)
        num1 = float(np.sum(df * df) / wf ** 2 + np.sum(dm * dm) / wm ** 2)
        num2 = float(wf * np.sum(df * qf) + wm * np.sum(dm * qm))
        den2 = float(wf ** 2 * np.sum(qf * qf) + wm ** 2 * np.sum(qm * qm))
        bb1 = num1 / den1 if den1 > 0.0 else SGP_ALPHA_MAX
        bb2 = num2 / den2 if num2 > 0.0 else SGP_ALPHA_MAX
        bb2_hist = (bb2_hist + [bb2])[-SGP_MEMORY:]
        if bb2 / bb1 <= tau:
            alpha = min(bb2_hist)
            tau *= 0.9
        else:
            alpha = bb1
            tau *= 1.1
        alpha = min(max(alpha, SGP_ALPHA_MIN), SGP_ALPHA_MAX)
    return sf, sm, trace


def free_set(f, mu, gf, gm, p: LMParams):
    """0/1 masks of the free variables: a variable is held when it lies on
    its lower bound with a positive gradient, or on its upper bound with a
    negative one (the descent direction -g would leave the box there)."""
    hold_f = ((f <= p.f_lo) & (gf > 0.0)) | ((f >= p.f_hi) & (gf < 0.0))
    hold_m = ((mu <= p.mu_lo) & (gm > 0.0)) | ((mu >= p.mu_hi) & (gm < 0.0))
    return (~hold_f).astype(np.float64), (~hold_m).astype(np.float64)


def model_decrease(g: Geometry, f, mu, gf, gm, sf, sm, af, am, prior=None) -> float:
    """pred = m(0) - m(s) = -(g.s + 0.5*(||J s||^2 + s.R s))  (eq. m-function)."""
    js = jvp(g, f, mu, sf, sm)
    sRs = 2.0 * (reg_energy(af, sf) + reg_energy(am, sm))
    if prior is not None:
        sRs += float(np.sum(prior[0] * sf * sf) + np.sum(prior[1] * sm * sm))
    gs = float(np.sum(gf * sf) + np.sum(gm * sm))
    return -(gs + 0.5 * (float(np.sum(js * js)) + sRs))


def nielsen_update(beta: float, nu: float, accepted: bool, rho: float):
    """Nielsen's damping update (H.B. Nielsen, IMM-REP-1999-05)."""
    if accepted:
        return beta * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3), 2.0
    return beta * nu, 2.0 * nu


def initial_damping(g: Geometry, f, mu, p: LMParams) -> float:
    if p.beta0 > 0.0:
        return float(p.beta0)
    one = np.ones(g.image_shape)
    j1 = jvp(g, f, mu, one, one)
    return p.tau * float(np.sum(j1 * j1)) / (2.0 * g.n * g.n)


def initial_guess(g: Geometry, y):
    """mu0 = 0, f0 = c0 * 1 with c0 the least-squares fit of A(1, 0) to y."""
    one = np.ones(g.image_shape)
    a1 = forward(g, one, np.zeros(g.image_shape))
    c0 = float(np.sum(a1 * y) / np.sum(a1 * a1))
    return c0 * one, np.zeros(g.image_shape)


@dataclass
class Iterate:
    """Everything one outer iteration produces (for step-by-step comparison)."""

    phi: float
    gf: np.ndarray
    gm: np.ndarray
    xf: np.ndarray
    xm: np.ndarray
    cg_rr: list
    sf: np.ndarray
    sm: np.ndarray
    pred: float
    ared: float
    rho: float
    phi_trial: float
    f_trial: np.ndarray
    mu_trial: np.ndarray


def lm_iteration(g: Geometry, y, f, mu, beta, p: LMParams, k: int) -> Iterate:
    """One outer iteration up to (not including) the accept decision."""
    af, am = alphas_at(p, k)
    pr = prior_at(p, k)
    phi, r = objective(g, y, f, mu, af, am, pr)
    gf, gm = gradient(g, f, mu, r, af, am, pr)
    if p.step == "sgp":
        xf, xm, rr = sgp(lambda a, b: normal_matvec(g, f, mu, a, b, beta, p, af, am, pr), gf, gm,
                         p.f_lo - f, p.f_hi - f, p.mu_lo - mu, p.mu_hi - mu, p.n_cg, p.w_f, p.w_mu)
    elif p.active_set:
        ff, fm = free_set(f, mu, gf, gm, p)

        def mv(a, b):
            qf, qm = normal_matvec(g, f, mu, ff * a, fm * b, beta, p, af, am, pr)
            return ff * qf, fm * qm
        xf, xm, rr = cg(mv, -ff * gf, -fm * gm, p.n_cg, p.w_f, p.w_mu)
    else:
        xf, xm, rr = cg(
            lambda a, b: normal_matvec(g, f, mu, a, b, beta, p, af, am, pr), -gf, -gm, p.n_cg, p.w_f, p.w_mu
        )
    ft = np.clip(f + xf, p.f_lo, p.f_hi)
    mt = np.clip(mu + xm, p.mu_lo, p.mu_hi)
    sf, sm = ft - f, mt - mu
    pred = model_decrease(g, f, mu, gf, gm, sf, sm, af, am, pr)
    phi_t, _ = objective(g, y, ft, mt, af, am, pr)
    ared = phi - phi_t
    rho = ared / pred if pred > 0.0 else -np.inf
    return Iterate(phi, gf, gm, xf, xm, rr, sf, sm, pred, ared, rho, phi_t, ft, mt)


HookFn = Callable[[np.ndarray, np.ndarray, np.ndarray, np.ndarray], tuple]


def lm_solve(
    g: Geometry,
    y,
    f0,
    mu0,
    p: LMParams,
    hook: Optional[HookFn] = None,
    replay: Optional[List[int]] = None,
    on_iterate: Optional[Callable] = None,
):
    """Run the LM iteration; returns (f, mu, LMReport).

    ``replay`` forces the accept decision of each outer iteration (1 accept,
    0 reject) instead of the test rho > eta; everything else is unchanged.
    ``hook(f, mu, s_f, s_mu) -> (f~, mu~)`` is the learned refinement.
    ``on_iterate(k, f, mu)`` (reporting only) sees the iterate after outer
    iteration k.
    """
    f = np.array(f0, dtype=np.float64)
    mu = np.array(mu0, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    rep = LMReport()
    beta = initial_damping(g, f, mu, p)
    beta_init = beta
    nu = 2.0
    for k in range(p.max_outer):
        it = lm_iteration(g, y, f, mu, beta, p, k)
        af, am = alphas_at(p, k)
        rep.phi.append(it.phi)
        rep.beta.append(beta)
        rep.pred.append(it.pred)
        rep.ared.append(it.ared)
        rep.rho.append(it.rho)
        rep.gnorm.append(float(np.sqrt(np.sum(it.gf ** 2) + np.sum(it.gm ** 2))))
        rep.cg_rr.append(list(it.cg_rr))
        acc = (it.rho > p.eta) if replay is None else bool(replay[k])
        rep.accepted.append(int(acc))
        hook_ok = 0
        hook_vals = (np.nan, np.nan)
        rep.iters_run = k + 1
        if acc:
            unorm = float(np.sqrt(np.sum(f ** 2) + np.sum(mu ** 2)))
            snorm = float(np.sqrt(np.sum(it.sf ** 2) + np.sum(it.sm ** 2)))
            f_old, mu_old = f, mu
            f, mu = it.f_trial, it.mu_trial
            beta, nu = nielsen_update(beta, nu, True, it.rho)
            if hook is not None:
                ft, mt = hook(f_old, mu_old, it.sf, it.sm)
                ft = np.asarray(ft, dtype=np.float64)
                mt = np.asarray(mt, dtype=np.float64)
                stf, stm = ft - f_old, mt - mu_old
                pr = prior_at(p, k)
                pred_t = model_decrease(g, f_old, mu_old, it.gf, it.gm, stf, stm, af, am, pr)
                phi_t, _ = objective(g, y, ft, mt, af, am, pr)
                rho_t = (it.phi - phi_t) / pred_t if pred_t > 0.0 else -np.inf
                hook_vals = (rho_t, pred_t)
                if rho_t > p.eta and pred_t >= it.pred:
                    f, mu = ft, mt
                    hook_ok = 1
            rep.hook_accepted.append(hook_ok)
            rep.hook_rho.append(hook_vals[0])
            rep.hook_pred.append(hook_vals[1])
            if p.tol > 0.0 and (it.ared <= p.tol * it.phi or snorm <= p.tol * unorm):
                rep.stop_reason = "tol"
                if on_iterate is not None:
                    on_iterate(k, f, mu)
                break
        else:
            beta, nu = nielsen_update(beta, nu, False, it.rho)
            rep.hook_accepted.append(0)
            rep.hook_rho.append(np.nan)
            rep.hook_pred.append(np.nan)
        if on_iterate is not None:
            on_iterate(k, f, mu)
        if beta > 1e16 * beta_init:
            rep.stop_reason = "beta_overflow"
            break
    af, am = alphas_at(p, rep.iters_run)
    rep.phi.append(objective(g, y, f, mu, af, am, prior_at(p, rep.iters_run))[0])
    rep.beta_final = beta
    return f, mu, rep


def step_quantities(g: Geometry, y, f, mu, f_trial, mu_trial, p: LMParams, k: int) -> dict:
    """The gain-ratio quantities of outer iteration k evaluated at a given
    iterate u = (f, mu) and trial point u' (eqs. m-function and
    rho_agreement): Phi(u), ||g(u)||, pred = m(0) - m(s) with s = u' - u,
    ared = Phi(u) - Phi(u'), and rho = ared / pred (-inf if pred <= 0).
    For checking another implementation step by step at its own iterates."""
    f, mu = np.asarray(f, np.float64), np.asarray(mu, np.float64)
    ft, mt = np.asarray(f_trial, np.float64), np.asarray(mu_trial, np.float64)
    y = np.asarray(y, np.float64)
    af, am = alphas_at(p, k)
    pr = prior_at(p, k)
    phi, r = objective(g, y, f, mu, af, am, pr)
    gf, gm = gradient(g, f, mu, r, af, am, pr)
    pred = model_decrease(g, f, mu, gf, gm, ft - f, mt - mu, af, am, pr)
    phi_t = objective(g, y, ft, mt, af, am, pr)[0]
    ared = phi - phi_t
    return {"phi": phi, "gnorm": float(np.sqrt(np.sum(gf ** 2) + np.sum(gm ** 2))), "pred": pred,
            "ared": ared, "phi_trial": phi_t, "rho": ared / pred if pred > 0.0 else -np.inf}


def step_quantities_job(args):
    """step_quantities from plain arguments (geometry keywords, arrays, the
    parameters, k), or with beta given the whole iteration from u (its CG
    solve included) as lm_iteration computes it: for process pools.  With a
    noise seed, every normal-operator product of that CG solve is multiplied
    elementwise by (1 + 1e-6 N(0, 1)): the solve's sensitivity to rounding
    of FP32 size."""
    geom_kw, y, f, mu, ft, mt, p, k, beta, noise_seed = args
    g = Geometry(**geom_kw)
    if beta is None:
        return step_quantities(g, y, f, mu, ft, mt, p, k)
    global normal_matvec
    exact = normal_matvec
    if noise_seed is not None:
        rng = np.random.default_rng(noise_seed)

        def normal_matvec(*a, **kw):
            qf, qm = exact(*a, **kw)
            return (qf * (1.0 + 1e-6 * rng.standard_normal(qf.shape)),
                    qm * (1.0 + 1e-6 * rng.standard_normal(qm.shape)))
    try:
        it = lm_iteration(g, np.asarray(y, np.float64), np.asarray(f, np.float64), np.asarray(mu, np.float64),
                          beta, p, k)
    finally:
        normal_matvec = exact
    return {"f_trial": it.f_trial, "mu_trial": it.mu_trial, "pred": it.pred, "ared": it.ared, "rho": it.rho,
            "cg_rr": list(it.cg_rr)}
