"""Writes the FP64 oracle's reconstruction of one slice in the scanner
geometry (9 x 9 assembly with missing rods, seed 0): data from the oracle's
projection of the phantom on the 330 x 330 grid (0.5 mm pixels) plus 2 %
Gaussian noise, reconstructed on the 165 x 165 grid (15 outer LM iterations
x 30 CG steps).  Stores the sinogram, per-iterate objective, gain ratio,
damping and decisions, the maps after iterations 5, 10 and 15, and the
spread of the same solve under FP32-level rounding (two solves with the
decisions replayed in which every normal-operator product is multiplied
elementwise by 1 + 1e-6 N(0, 1), seeds 1 and 2, run in parallel) to
scanner9x9_n165_oracle.npz.  Calls only the oracle and the input generator;
takes about three quarters of an hour on three cores.
"""
import multiprocessing as mp
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


def problem():
    cfg = inputs.SCANNER_165
    gf, sf = oracle_geometry(cfg, cfg.oversample)
    f_fine, mu_fine = inputs.scanner_phantom(cfg, 0, "missing", cfg.oversample)
    g, s = oracle_geometry(cfg, 1)
    # data in the reconstruction grid's units (its ray sums count its own
    # pixel steps): millimetres from the fine grid divided by its pixel size
    y = inputs.gaussian_noise((sf / s) * O.forward(gf, f_fine, mu_fine), cfg.noise, 0)
    f0, mu0 = L.initial_guess(g, y)
    p = L.LMParams(max_outer=cfg.max_outer, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha)
    return g, y, f0, mu0, p


def solve(seed, replay=None):
    """The reference solve (seed None) or a perturbed one replaying its
    decisions; returns the objective per iterate and the maps after 5, 10
    and 15 iterations."""
    g, y, f0, mu0, p = problem()
    if seed is not None:
        rng = np.random.default_rng(seed)
        plain = L.cg

        def noisy(matvec, bf, bm, n, wf=1.0, wm=1.0):
            def mv(a, b):
                qa, qb = matvec(a, b)
                return (qa * (1 + 1e-6 * rng.standard_normal(qa.shape)),
                        qb * (1 + 1e-6 * rng.standard_normal(qb.shape)))
            return plain(mv, bf, bm, n, wf, wm)
        L.cg = noisy
    snaps = {}
    t0 = time.time()

    def keep(k, f, mu):
        print("seed %s: iteration %d done after %.0f s" % (seed, k + 1, time.time() - t0), flush=True)
        if k + 1 in (5, 10, 15):
            snaps[k + 1] = (f.copy(), mu.copy())
    f, mu, rep = L.lm_solve(g, y, f0, mu0, p, replay=replay, on_iterate=keep)
    return rep, snaps, y, f0


def main(out_path):
    rep, snaps, y, f0 = solve(None)
    with mp.get_context("spawn").Pool(2) as pool:
        runs = pool.starmap(solve, [(1, rep.accepted), (2, rep.accepted)])
    spread_phi = np.zeros(len(rep.phi))
    spread = {k: [0.0, 0.0] for k in (5, 10, 15)}
    for prep, psnaps, _, _ in runs:
        spread_phi = np.maximum(spread_phi, np.abs(np.array(prep.phi) / np.array(rep.phi) - 1))
        for k in (5, 10, 15):
            for c in range(2):
                e = float(np.linalg.norm(psnaps[k][c] - snaps[k][c]) / np.linalg.norm(snaps[k][c]))
                spread[k][c] = max(spread[k][c], e)
    np.savez_compressed(
        out_path, y=y,
        phi=np.array(rep.phi), rho=np.array(rep.rho), beta=np.array(rep.beta),
        accepted=np.array(rep.accepted, dtype=np.int8),
        f5=snaps[5][0].astype(np.float32), mu5=snaps[5][1].astype(np.float32),
        f10=snaps[10][0].astype(np.float32), mu10=snaps[10][1].astype(np.float32),
        f15=snaps[15][0].astype(np.float32), mu15=snaps[15][1].astype(np.float32), f0=f0.astype(np.float32),
        spread_phi=spread_phi, spread_maps=np.array([spread[k] for k in (5, 10, 15)]),
    )


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "scanner9x9_n165_oracle.npz"))
