"""The Deep Gauss-Newton path on the GPU with a real (untrained, seeded) CNN
as the learned step: for every hook call the device's decision is the
safeguard of Prop. 3.2 / Alg. 2 applied to the values it reports
(rho(s~) > eta and m(0) - m(s~) >= m(0) - m(s)), those values match the
FP64 oracle's evaluation of the same proposal at the same iterate (relative
1e-3: the proposal differs from the oracle's by FP32 rounding of the
network and the iterate), and a proposal that is kept becomes the next
iterate.  Also the staged training of Alg. 1 on a tiny set: the networks
are built and trained and the step collection sees accepted LM steps.
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

from paper_2604_26745_amd import pget, refine  # noqa: E402

SMALL = inputs.SliceConfig("lattice3_n24", 24, 36, 36, n_rods=3, rod_radius=2.0, pitch=6.0,
                           can_half=10.0, n_empty=1, max_outer=6, n_cg=4)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def setup(seed=0):
    torch.backends.cudnn.enabled = False
    og = O.Geometry(SMALL.n, SMALL.n_angles, SMALL.n_bins, psf_sigma=SMALL.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(SMALL, seed)
    y = inputs.poisson_counts(O.forward(og, f_true, mu_true), SMALL.peak_counts, seed)
    f0, mu0 = OLM.initial_guess(og, y)
    return og, y, f0, mu0, f_true, mu_true


@pytest.mark.parametrize("gain", [0.0, 1.05], ids=["near_u", "extends_step"])
def test_cnn_hook_decisions_follow_reported_safeguard(gain):
    """gain 0: the decoder's output is scaled to ~0, so the proposal is ~u
    (no decrease: rejected); gain 1.05: L is the identity and the decoder
    outputs ~1.05, so the proposal extends the LM step by ~5 % (kept where
    the longer step still decreases the model as much)."""
    og, y, f0, mu0, ft, mt = setup()
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    torch.manual_seed(5)
    model = refine.build_cnn(f_max=2.0, mu_max=0.05).cuda().eval()
    with torch.no_grad():
        model.dec[-1].weight.mul_(0.01)
        model.dec[-1].bias.fill_(gain)
        if gain:
            model.L.weight.zero_()
            model.L.weight[0, 0, 2, 2] = 1.0
            model.L.weight[1, 1, 2, 2] = 1.0
    calls = []

    def hook(f, mu, sf, sm):
        with torch.no_grad():
            out = model(torch.stack([f, mu])[None], torch.stack([sf, sm])[None])[0]
        calls.append((f.double().cpu().numpy(), mu.double().cpu().numpy(), sf.double().cpu().numpy(),
                      sm.double().cpu().numpy(), out[0].double().cpu().numpy(), out[1].double().cpu().numpy()))
        return out[0].contiguous(), out[1].contiguous()

    prm = pget.SolverParams(max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=0.05 ** 2, d_mu=1 / 0.05 ** 2,
                            active_set=1)
    f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), prm, hook=hook)
    rep = rb.to_report()
    acc = [k for k in range(rep.iters_run) if rep.accepted[k]]
    assert len(calls) == len(acc) >= 2
    p = OLM.LMParams(max_outer=SMALL.max_outer, n_cg=SMALL.n_cg, w_mu=0.05 ** 2, d_mu=1 / 0.05 ** 2, active_set=True)
    for (fo, mo, sf, sm, ftl, mtl), k in zip(calls, acc):
        kept = rep.hook_rho[k] > prm.eta and rep.hook_pred[k] >= rep.pred[k]
        assert rep.hook_accepted[k] == int(kept)
        # the oracle's values for the same proposal at the same iterate
        af, am = OLM.alphas_at(p, k)
        phi, r = OLM.objective(og, y, fo, mo, af, am)
        gf, gm = OLM.gradient(og, fo, mo, r, af, am)
        pred_t = OLM.model_decrease(og, fo, mo, gf, gm, ftl - fo, mtl - mo, af, am)
        phi_t = OLM.objective(og, y, ftl, mtl, af, am)[0]
        rho_t = (phi - phi_t) / pred_t if pred_t > 0 else -np.inf
        log("k=%d hook pred %.6g / %.6g rho %.5g / %.5g lm pred %.6g kept %d" % (
            k, rep.hook_pred[k], pred_t, rep.hook_rho[k], rho_t, rep.pred[k], rep.hook_accepted[k]))
        assert abs(rep.hook_pred[k] - pred_t) <= 1e-3 * max(abs(pred_t), 1e-3 * phi)
        if np.isfinite(rho_t):
            assert abs(rep.hook_rho[k] - rho_t) <= 1e-3 * max(1.0, abs(rho_t))
    if gain:
        assert sum(rep.hook_accepted) >= 1
    else:
        assert sum(rep.hook_accepted) == 0
    # a kept proposal is the next iterate: the following call starts there
    for c in range(len(acc) - 1):
        if rep.hook_accepted[acc[c]]:
            assert np.allclose(calls[c + 1][0], calls[c][4], rtol=0, atol=1e-6)
            assert np.allclose(calls[c + 1][1], calls[c][5], rtol=0, atol=1e-7)


def test_staged_training_runs():
    torch.backends.cudnn.enabled = False
    plan = pget.Plan(SMALL.n, SMALL.n_angles, SMALL.n_bins)
    ys, u0s, truths = [], [], []
    for s in range(4):
        og, y, f0, mu0, ft, mt = setup(s)
        ys.append(T(y)); u0s.append((T(f0), T(mu0))); truths.append((T(ft), T(mt)))
    prm = pget.SolverParams(max_outer=3, n_cg=SMALL.n_cg, w_mu=0.05 ** 2, d_mu=1 / 0.05 ** 2, active_set=1)
    steps = refine.collect_steps(plan, ys, u0s, prm)
    assert all(float(torch.abs(sf).max()) > 0 for sf, sm in steps)      # an LM step was accepted
    models, rep = refine.train_networks(plan, ys, u0s, truths, prm, K=2, epochs=3, f_max=2.0, mu_max=0.05)
    assert len(models) == 2 and rep.n_params == 27198
    assert all(np.isfinite(v) for v in rep.loss_before + rep.loss_after)
    st = {}
    f, mu, rb = refine.deep_gn_solve(plan, ys[0], *u0s[0], prm, models, st)
    assert st["hook_calls"] == sum(rb.to_report().accepted) >= 1
