"""Planted mistakes: each plausible slip in the oracle must fail at least one
of its pins.  Mutated copies of the oracle's sources (C operators, numpy LM)
are built in a temporary directory; the original sources must pass every
pin, each mutant must fail one.

Operator pins (8 x 8 maps, a plain geometry and one with a depth factor and
a depth-dependent response): the forward map against the dense brute-force
formulation, J v and J^T w against torch autograd of it, the regulariser's
gradient against central differences of its energy.  Solver pins: the gain
ratio of an emission-only step is exactly 1 (the data term is linear in f,
the penalty and the prior quadratic), preconditioned CG reaches the direct
solve in as many steps as unknowns, Nielsen's damping factor at
rho = 0.75 is 1 - 0.5^3, the initial damping equals tau times the Rayleigh
quotient of J^T J at the all-ones vector with J from torch autograd of the
dense formulation, the continuation's alphas after its halt are alpha /
decay^until, and ten rejections in a row (beta0 * 2^55 > 1e16 beta0) stop
the solve, and the scaled gradient projection reaches the bounded least
squares solution of a box-constrained quadratic, decreasing monotonically."""
import ctypes
import os
import subprocess
import sys
import types

import numpy as np
import pytest

import oracle as O
from oracle.dense import DenseModel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_SRC = os.path.join(ROOT, "oracle", "pget_oracle.c")
LM_SRC = os.path.join(ROOT, "oracle", "lm.py")

C_MUTANTS = {
    "self-attenuation without the half": ("double B = g->step * (0.5 * mu_s[i] + beyond);",
                                          "double B = g->step * (mu_s[i] + beyond);"),
    "sign of omega_perp": ("*qx = -r->s * r->sn + t * r->cs;", "*qx = r->s * r->sn + t * r->cs;"),
    "J v: beam transform without the half": ("double V = g->step * (0.5 * vmu_s[i] + beyond);",
                                             "double V = g->step * (vmu_s[i] + beyond);"),
    "J v: sign of the attenuation term": ("c = E[i] * (vf_s[i] - path_factor(g, i) * lam_s[i] * V);",
                                          "c = E[i] * (vf_s[i] + path_factor(g, i) * lam_s[i] * V);"),
    "J^T w: self term without the half": ("d_mu = -g->step * g->step * wr * (0.5 * cle + before);",
                                          "d_mu = -g->step * g->step * wr * (cle + before);"),
    "J^T w: farther samples dropped": ("                    before += cle;\n",
                                       "                    before += 0.0 * cle;\n"),
    "depth factor ignored": ("return g->depth ? g->atten_scale * g->depth[i] : g->atten_scale;",
                             "return g->atten_scale;"),
    "response blend swapped": ("return (1.0 - g->resp[i]) * taps[k + K] + g->resp[i] * g->far_taps[k + K];",
                               "return g->resp[i] * taps[k + K] + (1.0 - g->resp[i]) * g->far_taps[k + K];"),
    "response depth reversed": (
        "return (1.0 - g->resp[i]) * taps[k + K] + g->resp[i] * g->far_taps[k + K];",
        "int ii = og_n_samples(g) - 1 - i;\n"
        "    return (1.0 - g->resp[ii]) * taps[k + K] + g->resp[ii] * g->far_taps[k + K];"),
    "bilinear axes transposed": ("double wt = tent(qx - ((double)c - half)) * tent(qy - ((double)r - half));",
                                 "double wt = tent(qx - ((double)r - half)) * tent(qy - ((double)c - half));"),
    "regulariser gradient sign": ("                out[r * n + c] -= alpha * d;\n",
                                  "                out[r * n + c] += alpha * d;\n"),
}

LM_MUTANTS = {
    "pred without the half": ("return -(gs + 0.5 * (float(np.sum(js * js)) + sRs))",
                              "return -(gs + 1.0 * (float(np.sum(js * js)) + sRs))"),
    "CG beta inverted": ("pf = zf + (rr_new / rr) * pf\n        pm = zm + (rr_new / rr) * pm",
                         "pf = zf + (rr / rr_new) * pf\n        pm = zm + (rr / rr_new) * pm"),
    "Nielsen exponent": ("1.0 - (2.0 * rho - 1.0) ** 3", "1.0 - (2.0 * rho - 1.0) ** 2"),
    "r instead of W r in CG": ("zf, zm = wf * rf, wm * rm", "zf, zm = rf, rm"),
    "objective without the half": ("phi = 0.5 * float(np.dot(r.ravel(), r.ravel()))",
                                   "phi = float(np.dot(r.ravel(), r.ravel()))"),
    "prior gradient sign": ("gf, gm = gf + wf * (f - rf), gm + wm * (mu - rm)",
                            "gf, gm = gf - wf * (f - rf), gm - wm * (mu - rm)"),
    "beta0 over N^2 instead of the 2 N^2 unknowns": ("/ (2.0 * g.n * g.n)", "/ (g.n * g.n)"),
    "beta0 from the emission block only": ("j1 = jvp(g, f, mu, one, one)", "j1 = jvp(g, f, mu, one, 0.0 * one)"),
    "continuation without its halt": ("decay = p.alpha_decay ** min(k, p.alpha_decay_until)\n    return",
                                      "decay = p.alpha_decay ** k\n    return"),
    "damping overflow never stops": ("if beta > 1e16 * beta_init:", "if beta > 1e16 * beta:"),
    "SGP without the projection": ("yf = np.clip(sf - alpha * wf * rf, lo_f, hi_f)", "yf = sf - alpha * wf * rf"),
    "SGP gradient not updated": ("rf, rm = rf + lam * qf, rm + lam * qm", "rf, rm = rf, rm + lam * qm"),
    "SGP without its line search": ("        while lam * gd + 0.5 * lam * lam * dMd > SGP_ARMIJO * lam * gd and lam > 1e-30:",
                                    "        while False:"),
}


def mutate(src, old, new):
    assert src.count(old) >= 1, old
    # the first site only (a slip is made in one place)
    return src.replace(old, new, 1)


# ---------------------------------------------------------------- C operators
def build_c(tmp_path, name, src):
    c = tmp_path / (name + ".c")
    c.write_text(src)
    so = tmp_path / (name + ".so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"], check=True,
                   capture_output=True)
    lib = ctypes.CDLL(str(so))
    P = ctypes.POINTER(O._CGeometry)
    D = ctypes.POINTER(ctypes.c_double)
    lib.og_forward.argtypes = [P, D, D, D]
    lib.og_jvp.argtypes = [P, D, D, D, D, D]
    lib.og_vjp.argtypes = [P, D, D, D, D, D]
    lib.og_reg_energy.argtypes = [ctypes.c_int, ctypes.c_double, D]
    lib.og_reg_energy.restype = ctypes.c_double
    lib.og_reg_gradient.argtypes = [ctypes.c_int, ctypes.c_double, D, D]
    return lib


def ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def operator_pins(lib):
    """Each operator pin's error and the tolerance the oracle meets it to."""
    torch = pytest.importorskip("torch")
    n, na, nb = 8, 8, 14
    g0 = O.Geometry(n, na, nb, psf_sigma=1.5, atten_scale=0.7)
    n_t, K = g0.n_samples, g0.psf_half_width
    depth = tuple(1.0 + 0.6 * (1.0 - i / (n_t - 1)) for i in range(n_t))
    rng = np.random.default_rng(41)
    alpha = tuple(np.clip(1.0 - np.arange(n_t) / (n_t - 1) + 0.1 * rng.uniform(-1, 1, n_t), 0, 1))
    k = np.arange(-K, K + 1)
    far = np.exp(-(k ** 2) / (2 * 2.5 ** 2))
    far = tuple(far / far.sum())
    f = rng.uniform(0.1, 1.0, (n, n))
    mu = rng.uniform(0.0, 0.3, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    T = lambda a: torch.tensor(a, dtype=torch.float64)
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    pins = {}
    for tag, extra in (("plain", {}), ("full model", {"depth": depth, "resp": alpha, "far_taps": far})):
        g = O.Geometry(n, na, nb, psf_sigma=1.5, atten_scale=0.7, **extra)
        D = DenseModel(n, na, nb, psf_sigma=1.5, atten_scale=0.7, **extra)
        gc = g._c()
        y = np.empty((na, nb))
        lib.og_forward(ctypes.byref(gc), ptr(f), ptr(mu), ptr(y))
        pins["forward vs dense, " + tag] = (rel(y, D.forward(f, mu)), 1e-12)
        fn = lambda a, b: D.forward(a, b, xp=torch)
        _, jt = torch.func.jvp(fn, (T(f), T(mu)), (T(vf), T(vm)))
        jv = np.empty((na, nb))
        lib.og_jvp(ctypes.byref(gc), ptr(f), ptr(mu), ptr(vf), ptr(vm), ptr(jv))
        pins["J v vs autograd, " + tag] = (rel(jv, jt.numpy()), 1e-12)
        _, back = torch.func.vjp(fn, T(f), T(mu))
        tf, tm = back(T(w))
        gf, gm = np.empty((n, n)), np.empty((n, n))
        lib.og_vjp(ctypes.byref(gc), ptr(f), ptr(mu), ptr(w), ptr(gf), ptr(gm))
        pins["J^T w vs autograd, " + tag] = (max(rel(gf, tf.numpy()), rel(gm, tm.numpy())), 1e-12)
    # regulariser gradient against central differences of its energy (the
    # differences carry about 1e-9 of truncation and rounding)
    x = np.ascontiguousarray(rng.standard_normal((n, n)))
    grad = np.empty((n, n))
    lib.og_reg_gradient(n, 0.7, ptr(x), ptr(grad))
    fd = np.empty((n, n))
    h = 1e-6
    for idx in np.ndindex(n, n):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd[idx] = (lib.og_reg_energy(n, 0.7, ptr(xp)) - lib.og_reg_energy(n, 0.7, ptr(xm))) / (2 * h)
    pins["regulariser gradient vs differences"] = (rel(grad, fd), 1e-7)
    return pins


def check(pins, name):
    """The original passes every pin; a mutant misses one by 100x its tolerance."""
    missed = {k: e for k, (e, tol) in pins.items() if e > 100 * tol}
    if name is None:
        assert all(e <= tol for e, tol in pins.values()), pins
    else:
        print("%-40s fails %d pin(s), e.g. %s" % (name, len(missed), next(iter(missed.items()), None)))
        assert missed, name


def test_c_oracle_mutants_fail_a_pin(tmp_path):
    src = open(C_SRC).read()
    check(operator_pins(build_c(tmp_path, "original", src)), None)
    for k, (name, (old, new)) in enumerate(C_MUTANTS.items()):
        check(operator_pins(build_c(tmp_path, "m%d" % k, mutate(src, old, new))), name)


# ------------------------------------------------------------------ numpy LM
def load_lm(name, src):
    """The LM module built from `src` (registered while it executes, as its
    dataclasses need)."""
    full = "oracle._mutant_" + name
    mod = types.ModuleType(full)
    mod.__package__ = "oracle"
    sys.modules[full] = mod
    try:
        exec(compile(src, LM_SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules[full]
    return mod


def lm_pins(L):
    """Each solver pin's error and the tolerance the oracle meets it to."""
    rng = np.random.default_rng(42)
    n, na, nb = 8, 10, 14
    g = O.Geometry(n, na, nb, psf_sigma=1.5)
    f = rng.uniform(0.2, 1.0, (n, n))
    mu = rng.uniform(0.0, 0.1, (n, n))
    y = O.forward(g, f, mu) * (1 + 0.05 * rng.standard_normal((na, nb)))
    af, am = 0.03, 0.02
    prior = (rng.uniform(0, 2, (n, n)), rng.uniform(0, 1, (n, n)), rng.uniform(0, 1, (n, n)),
             rng.uniform(0, 0.1, (n, n)))
    phi, r = L.objective(g, y, f, mu, af, am, prior=prior)
    gf, gm = L.gradient(g, f, mu, r, af, am, prior=prior)
    sf = 0.1 * rng.standard_normal((n, n))
    sm = np.zeros((n, n))
    pred = L.model_decrease(g, f, mu, gf, gm, sf, sm, af, am, prior=prior)
    ared = phi - L.objective(g, y, f + sf, mu, af, am, prior=prior)[0]
    pins = {"rho of an emission step": (abs(ared / pred - 1.0), 1e-9)}
    # preconditioned CG on a small SPD system reaches the direct solve
    m = 6
    A = rng.standard_normal((2 * m, 2 * m))
    A = A @ A.T + 2 * m * np.eye(2 * m)
    b = rng.standard_normal(2 * m)

    def mv(a, c):
        out = A @ np.concatenate([a.ravel(), c.ravel()])
        return out[:m].reshape(a.shape), out[m:].reshape(c.shape)
    xf, xm = L.cg(mv, b[:m].copy(), b[m:].copy(), 2 * m, 0.3, 2.0)[:2]    # M x = b from x = 0
    x = np.linalg.solve(A, b)
    got = np.concatenate([np.ravel(xf), np.ravel(xm)])
    pins["CG vs direct solve"] = (float(np.abs(got - x).max() / np.abs(x).max()), 1e-8)
    beta, _ = L.nielsen_update(1.0, 2.0, True, 0.75)
    pins["Nielsen factor at rho = 0.75"] = (abs(beta - (1.0 - 0.5 ** 3)), 1e-15)
    # initial damping against the dense Jacobian (torch autograd of the
    # dense formulation, both blocks, all-ones direction)
    torch = pytest.importorskip("torch")
    D = DenseModel(n, na, nb, psf_sigma=1.5)
    T = lambda a: torch.tensor(a, dtype=torch.float64)
    Jf, Jm = torch.autograd.functional.jacobian(lambda a, b: D.forward(a, b, xp=torch), (T(f), T(mu)))
    J = np.concatenate([Jf.numpy().reshape(na * nb, n * n), Jm.numpy().reshape(na * nb, n * n)], axis=1)
    p0 = L.LMParams(tau=1e-3)
    want = 1e-3 * float(np.sum((J @ np.ones(2 * n * n)) ** 2)) / (2 * n * n)
    pins["beta0 vs dense Rayleigh quotient"] = (abs(L.initial_damping(g, f, mu, p0) / want - 1.0), 1e-12)
    pc = L.LMParams(alpha_f=1e-2, alpha_mu=1e-2, alpha_decay=5.0, alpha_decay_until=3)
    pins["alpha after the continuation's halt"] = (abs(L.alphas_at(pc, 5)[0] / 8e-5 - 1.0), 1e-15)
    # ten rejections in a row end the solve (beta0 * 2^55 > 1e16 beta0)
    po = L.LMParams(max_outer=12, n_cg=2, beta0=1.0)
    rep = L.lm_solve(g, y, f, mu, po, replay=[0] * 12)[2]
    pins["damping overflow after ten rejections"] = (float(abs(rep.iters_run - 10)), 0.0)
    # scaled gradient projection of a box-constrained quadratic against
    # scipy's bounded-variable least squares (through the Cholesky factor)
    from scipy.optimize import lsq_linear
    k = 12
    B = rng.standard_normal((k, k))
    Mq = B @ B.T + 0.5 * np.eye(k)
    gq = rng.standard_normal(k)
    lo, hi = -0.05 * rng.uniform(0.2, 1, k), 0.05 * rng.uniform(0.2, 1, k)
    Lc = np.linalg.cholesky(Mq)
    ref = lsq_linear(Lc.T, -np.linalg.solve(Lc, gq), bounds=(lo, hi), method="bvls", tol=1e-14).x
    h = k // 2

    def mvq(a, c):
        out = Mq @ np.concatenate([a, c])
        return out[:h], out[h:]
    sf, sm, qv = L.sgp(mvq, gq[:h], gq[h:], lo[:h], hi[:h], lo[h:], hi[h:], 500, 0.5, 2.0)
    got = np.concatenate([sf, sm])
    pins["SGP vs bounded least squares"] = (float(np.abs(got - ref).max() / np.abs(ref).max()), 1e-8)
    pins["SGP monotone"] = (max([0.0] + [b - a for a, b in zip(qv, qv[1:])]), 1e-12)
    return pins


def test_lm_oracle_mutants_fail_a_pin():
    src = open(LM_SRC).read()
    check(lm_pins(load_lm("original", src)), None)
    for k, (name, (old, new)) in enumerate(LM_MUTANTS.items()):
        check(lm_pins(load_lm("m%d" % k, mutate(src, old, new))), name)
