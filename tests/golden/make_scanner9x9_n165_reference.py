"""Writes the FP64 oracle's reconstruction of one slice in the scanner
geometry (9 x 9 assembly with missing rods, seed 0): data from the oracle's
projection of the phantom on the 330 x 330 grid (0.5 mm pixels) plus 2 %
Gaussian noise, reconstructed on the 165 x 165 grid (15 outer LM iterations
x 30 CG steps).  Stores the sinogram, per-iterate objective, gain ratio,
damping and decisions, and the maps after iterations 5, 10 and 15, to
scanner9x9_n165_oracle.npz.  Calls only the oracle and the input generator;
takes about a quarter of an hour on one core.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import lm as L  # noqa: E402
from paper_2604_26745_amd import inputs  # noqa: E402


def oracle_geometry(cfg, oversample):
    d = inputs.scanner_geometry(cfg, oversample)
    g = O.Geometry(d["n"], d["n_angles"], d["n_bins"], bin_size=d["bin_size"], step=d["step"],
                   psf_sigma=d["psf_sigma"], atten_scale=d["atten_scale"])
    return g, d["y_scale"]


def main(out_path):
    cfg = inputs.SCANNER_165
    gf, sf = oracle_geometry(cfg, cfg.oversample)
    f_fine, mu_fine = inputs.scanner_phantom(cfg, 0, "missing", cfg.oversample)
    y = inputs.gaussian_noise(sf * O.forward(gf, f_fine, mu_fine), cfg.noise, 0)
    g, s = oracle_geometry(cfg, 1)
    assert s == 1.0
    f0, mu0 = L.initial_guess(g, y)
    p = L.LMParams(max_outer=cfg.max_outer, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha)
    snaps = {}
    t0 = time.time()

    def keep(k, f, mu):
        print("iteration %d done after %.0f s" % (k + 1, time.time() - t0), flush=True)
        if k + 1 in (5, 10, 15):
            snaps[k + 1] = (f.astype(np.float32), mu.astype(np.float32))

    f, mu, rep = L.lm_solve(g, y, f0, mu0, p, on_iterate=keep)
    np.savez_compressed(
        out_path, y=y,
        phi=np.array(rep.phi), rho=np.array(rep.rho), beta=np.array(rep.beta),
        accepted=np.array(rep.accepted, dtype=np.int8),
        f5=snaps[5][0], mu5=snaps[5][1], f10=snaps[10][0], mu10=snaps[10][1],
        f15=snaps[15][0], mu15=snaps[15][1], f0=f0.astype(np.float32),
    )


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "scanner9x9_n165_oracle.npz"))
