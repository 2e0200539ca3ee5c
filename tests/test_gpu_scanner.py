"""Scanner geometry on the GPU against the FP64 oracle: the operators on the
165 x 165 reconstruction grid (1 mm pixels, 182 bins of 2 pixels, 360
angles) and on the 330 x 330 data grid (0.5 mm pixels, bins of 4 pixels,
attenuation per mm through atten_scale 0.5), and the LM reconstruction of
the stored slice (data from the fine grid with 2 % noise, tests/golden/)
with the oracle's decisions replayed.  Tolerances: forward relative L2
<= 1e-5 and max-abs / max-ref <= 1e-4 on both grids.  Jacobian products on
the reconstruction grid: <= 1e-5 for band-limited directions (white noise
smoothed by a Gaussian of one pixel, like the directions the solver
produces), <= 2e-5 for white noise; on the data grid (used only for its
forward map) <= 3e-5.  Sample positions are FP32 pixel coordinates reaching
~180 px (~360 on the data grid), one rounding is up to 7.6e-6 px (1.5e-5),
and the relative error of a product grows with that position error and with
the bin spacing in pixels (2 and 4 here), since a pixel then draws on fewer
lattice points.  LM: objective per iterate <= 1e-5 relative (measured
6.2e-6), maps after 5 / 10 / 15 iterations <= 5e-5 relative L2 (measured
f 2.1e-6, mu 1.4e-5 after 15: CG in FP32 amplifies the products' rounding
by the conditioning of the damped normal matrix, which the strong
attenuation of this geometry makes worse than in the lattice workloads).
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

CFG = inputs.SCANNER_165
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "scanner9x9_n165_oracle.npz")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def H(t):
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def plans(oversample, n_angles=None):
    d = inputs.scanner_geometry(CFG, oversample)
    na = n_angles or d["n_angles"]
    og = O.Geometry(d["n"], na, d["n_bins"], bin_size=d["bin_size"], step=d["step"],
                    psf_sigma=d["psf_sigma"], atten_scale=d["atten_scale"])
    pl = pget.Plan(d["n"], na, d["n_bins"], bin_size=d["bin_size"], step=d["step"],
                   psf_sigma=d["psf_sigma"], atten_scale=d["atten_scale"])
    return og, pl


@pytest.mark.parametrize("oversample,n_angles", [(1, None), (2, 60)], ids=["grid165", "grid330"])
@pytest.mark.parametrize("smooth", [True, False], ids=["bandlimited", "whitenoise"])
def test_scanner_operators(oversample, n_angles, smooth):
    from scipy.ndimage import gaussian_filter
    og, pl = plans(oversample, n_angles)
    f, mu = inputs.scanner_phantom(CFG, 1, "replaced", oversample)
    rng = np.random.default_rng(11)
    vf, vm = rng.standard_normal(f.shape), 0.01 * rng.standard_normal(f.shape)
    w = rng.standard_normal(og.sino_shape)
    if smooth:
        vf, vm = gaussian_filter(vf, 1.0), gaussian_filter(vm, 1.0)
        w = gaussian_filter(w, 1.0)
    y, y_ref = H(pl.forward(T(f), T(mu))), O.forward(og, f, mu)
    jv, jv_ref = H(pl.jvp(T(f), T(mu), T(vf), T(vm))), O.jvp(og, f, mu, vf, vm)
    gf, gm = pl.vjp(T(f), T(mu), T(w))
    gf_ref, gm_ref = O.vjp(og, f, mu, w)
    errs = (rel(y, y_ref), rel(jv, jv_ref), rel(H(gf), gf_ref), rel(H(gm), gm_ref))
    log("scanner x%d %s: forward %.2e jvp %.2e vjp f %.2e mu %.2e"
        % ((oversample, "band-limited" if smooth else "white noise") + errs))
    assert errs[0] <= 1e-5 and maxrel(y, y_ref) <= 1e-4
    bound = (1e-5 if smooth else 2e-5) if oversample == 1 else 3e-5
    assert max(errs[1:]) <= bound
    assert maxrel(jv, jv_ref) <= 1e-4
    assert maxrel(H(gf), gf_ref) <= 1e-4 and maxrel(H(gm), gm_ref) <= 1e-4


def test_scanner_lm_replayed():
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle reconstruction not present")
    ref = np.load(GOLDEN)
    og, pl = plans(1)
    y = ref["y"]
    f0, mu0 = OLM.initial_guess(og, y)
    assert rel(ref["f0"], f0) < 1e-6
    replay = [int(v) for v in ref["accepted"]]
    errs, maps = [], {}
    for k_end in (5, 10, 15):
        prm = pget.SolverParams(max_outer=k_end, n_cg=CFG.n_cg, alpha_f=CFG.alpha, alpha_mu=CFG.alpha,
                                replay=replay[:k_end])
        f, mu, rb = pl.lm_solve(T(y), T(f0), T(mu0), prm)
        rep = rb.to_report()
        if k_end == 15:
            errs = [abs(rep.phi[k] - ref["phi"][k]) / ref["phi"][k] for k in range(len(ref["phi"]))]
        maps[k_end] = (rel(f.cpu().numpy(), ref["f%d" % k_end]), rel(mu.cpu().numpy(), ref["mu%d" % k_end]))
    log("scanner phi rel err per iterate: %s" % " ".join("%.1e" % e for e in errs))
    log("scanner map rel L2 (f, mu) after 5/10/15: %s" % " ".join("(%.1e, %.1e)" % maps[k] for k in (5, 10, 15)))
    assert max(errs) <= 1e-5
    for k in (5, 10, 15):
        assert maps[k][0] <= 5e-5 and maps[k][1] <= 5e-5
