"""Writes the FP64 oracle's reconstruction of one 128x128 9x9-lattice slice
(360 angles x 192 bins, seed 0; 15 outer LM iterations x 30 CG steps) to
lattice9_n128_oracle.npz: per-iterate objective, gain ratio, damping and
decisions, and the maps after iterations 5, 10 and 15 (float32).  Calls only
the oracle and the input generator.  Takes about eight minutes on one core.
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


def main(out_path):
    cfg = inputs.MAIN_128
    g = O.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f_true, mu_true = inputs.rod_lattice(cfg, 0)
    y = inputs.poisson_counts(O.forward(g, f_true, mu_true), cfg.peak_counts, 0)
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
        out_path,
        phi=np.array(rep.phi), rho=np.array(rep.rho), beta=np.array(rep.beta),
        accepted=np.array(rep.accepted, dtype=np.int8),
        f5=snaps[5][0], mu5=snaps[5][1], f10=snaps[10][0], mu10=snaps[10][1],
        f15=snaps[15][0], mu15=snaps[15][1], f0=f0.astype(np.float32),
    )


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice9_n128_oracle.npz"))
