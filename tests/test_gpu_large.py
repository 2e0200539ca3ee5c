"""The 256x256 slice (17x17 rod lattice, 360 angles x 256 bins, 15 outer x 30
CG) against the FP64 oracle's stored reconstruction (tests/golden/, written by
make_lattice17_n256_reference.py from the oracle alone).

With the oracle's accept decisions replayed, per-iterate objective and the
maps after iterations 5, 10 and 15 are compared.  Stated tolerances:
FP32  objective per iterate <= 1e-5 relative, maps <= 1e-5 relative L2
      (measured 4e-7 and 2e-6);
BF16  objective per iterate <= 1e-4 relative, maps <= 2e-3 relative L2
      (measured 1.1e-5 and 3.2e-4: BF16 weights perturb every Jacobian
      product by about 2e-3, which the damped steps mostly absorb).
"""
import os

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

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lattice17_n256_oracle.npz")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def case():
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle reconstruction not present")
    ref = np.load(GOLDEN)
    cfg = inputs.LARGE_256
    g = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(g, f_true, mu_true), cfg.peak_counts, 0)
    f0, mu0 = OLM.initial_guess(g, y)
    assert rel(ref["f0"], f0) < 1e-6
    return cfg, ref, y, f0, mu0


@pytest.mark.parametrize("storage,tphi,tmap", [("fp32", 1e-5, 1e-5), ("bf16", 1e-4, 2e-3)])
def test_lattice17_n256_replayed(case, storage, tphi, tmap):
    cfg, ref, y, f0, mu0 = case
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, storage=storage)
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")
    replay = [int(v) for v in ref["accepted"]]
    errs, maps = [], {}
    for k_end in (5, 10, 15):
        prm = pget.SolverParams(max_outer=k_end, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha,
                                replay=replay[:k_end])
        f, mu, rb = plan.lm_solve(T(y), T(f0), T(mu0), prm)
        rep = rb.to_report()
        if k_end == 15:
            errs = [abs(rep.phi[k] - ref["phi"][k]) / ref["phi"][k] for k in range(len(ref["phi"]))]
        maps[k_end] = (rel(f.cpu().numpy(), ref["f%d" % k_end]), rel(mu.cpu().numpy(), ref["mu%d" % k_end]))
    print("%s phi rel err per iterate: %s" % (storage, " ".join("%.1e" % e for e in errs)), flush=True)
    print("%s map rel L2 (f, mu) after 5/10/15: %s" % (
        storage, " ".join("(%.1e, %.1e)" % maps[k] for k in (5, 10, 15))), flush=True)
    assert max(errs) <= tphi
    for k in (5, 10, 15):
        assert maps[k][0] <= tmap and maps[k][1] <= tmap
