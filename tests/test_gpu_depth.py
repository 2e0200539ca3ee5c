"""The depth factor of the attenuation path (the vertical correction of the
discrete model, pget_plan_set_depth_factor) on the GPU against the FP64
oracle: the operators with and without the quarter-turn fold of the gather
(relative L2 <= 1e-5, max-abs / max-ref <= 1e-4; BF16 storage: products
<= 4e-3 as in test_gpu_bf16), an LM trajectory with the oracle's decisions
replayed (objective per iterate 1e-4, maps 1e-3, as in test_gpu_lm), that
clearing the factor gives back a fresh plan's results bitwise, that a solve
after changing it does not reuse the captured sequence, and argument errors.
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
    """Larger far from the detector (sample 0), 1 at the detector side."""
    return tuple(1.0 + 0.6 * (1.0 - i / (n_t - 1)) for i in range(n_t))


def phantom(n, seed, mu_rod=0.08):
    cfg = inputs.SliceConfig("t", n, 8, n, n_rods=5, rod_radius=max(1.0, n / 24), pitch=n / 7,
                             can_half=0.42 * n, n_empty=2, rod_mu=mu_rod)
    return inputs.rod_lattice(cfg, seed)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("n,na,nb", [(64, 120, 96), (48, 90, 70)], ids=["quad", "no_quad"])
def test_operators_with_depth(n, na, nb, storage):
    plan = pget.Plan(n, na, nb, storage=storage)
    d = depth_table(plan.n_samples)
    plan.set_depth_factor(d)
    og = O.Geometry(n, na, nb, depth=d)
    f, mu = phantom(n, 3)
    rng = np.random.default_rng(5)
    vf, vm = rng.standard_normal((2, n, n))
    vm *= 0.05
    w = rng.standard_normal((na, nb))
    y, y_ref = H(plan.forward(T(f), T(mu))), O.forward(og, f, mu)
    jv, jv_ref = H(plan.jvp(T(f), T(mu), T(vf), T(vm))), O.jvp(og, f, mu, vf, vm)
    gf, gm = plan.vjp(T(f), T(mu), T(w))
    gf_ref, gm_ref = O.vjp(og, f, mu, w)
    errs = (rel(y, y_ref), rel(jv, jv_ref), rel(H(gf), gf_ref), rel(H(gm), gm_ref))
    log("depth %s %dx%d: forward %.2e jvp %.2e vjp f %.2e mu %.2e" % ((storage, na, nb) + errs))
    assert errs[0] <= 1e-5 and maxrel(y, y_ref) <= 1e-4
    bound = 1e-5 if storage == "fp32" else 4e-3
    assert max(errs[1:]) <= bound
    if storage == "fp32":
        assert maxrel(jv, jv_ref) <= 1e-4
        assert maxrel(H(gf), gf_ref) <= 1e-4 and maxrel(H(gm), gm_ref) <= 1e-4
    # the factor is in effect: without it the forward map differs
    assert rel(y, O.forward(O.Geometry(n, na, nb), f, mu)) > 1e-3


def test_lm_with_depth_replayed():
    cfg = inputs.SliceConfig("lattice3_n24", 24, 36, 36, n_rods=3, rod_radius=2.0, pitch=6.0,
                             can_half=10.0, n_empty=1, max_outer=6, n_cg=4)
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins)
    d = depth_table(plan.n_samples)
    og = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, depth=d)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(og, y)
    p = OLM.LMParams(max_outer=cfg.max_outer, n_cg=cfg.n_cg, w_mu=0.05 ** 2, active_set=True)
    of, om, orep = OLM.lm_solve(og, y, f0, mu0, p)
    plan.set_depth_factor(d)
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


def test_clearing_and_changing_the_factor():
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
    d = depth_table(plan.n_samples)
    plan.lm_solve(y, f0, m0, prm)          # captures the solve without the factor
    plan.set_depth_factor(d)
    f_d, _, _ = plan.lm_solve(y, f0, m0, prm)
    other = pget.Plan(n, na, nb)
    other.set_depth_factor(d)
    f_ref, _, _ = other.lm_solve(y, f0, m0, prm)
    assert torch.equal(f_d, f_ref)          # not the earlier captured sequence
    assert not torch.equal(f_d, f_plain)
    plan.set_depth_factor(None)
    assert torch.equal(plan.forward(T(f), T(mu)), y_plain)
    f_back, _, _ = plan.lm_solve(y, f0, m0, prm)
    assert torch.equal(f_back, f_plain)


def test_bad_depth_factor_rejected():
    plan = pget.Plan(16, 12, 24)
    n_t = plan.n_samples
    with pytest.raises(pget.PgetError):
        plan.set_depth_factor((1.0,) * (n_t - 1))
    with pytest.raises(pget.PgetError):
        plan.set_depth_factor((1.0,) * (n_t - 1) + (-1.0,))
    with pytest.raises(pget.PgetError):
        plan.set_depth_factor((1.0,) * (n_t - 1) + (float("nan"),))
