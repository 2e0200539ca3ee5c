"""Scanner geometry (182 bins at 2 mm, 165 x 165 grid of 2 mm pixels, data on
a grid twice as fine): the unit bookkeeping of ``inputs.scanner_geometry`` and
the phantom generator, pinned through the oracle to things other than itself.

* A uniform disk without attenuation projects to its chord lengths
  2 sqrt(R^2 - s^2) (mm) at bin offsets s = (j - 90.5) * 2 mm.
* A smooth object projected on the fine grid (1 mm pixels, attenuation per
  mm through atten_scale = 1, ray sums scaled by 1 mm) agrees with its
  projection on the reconstruction grid to the discretisation error
  (second order in the pixel size).
* The phantom's total emission and attenuation agree across resolutions.
"""
import math

import numpy as np

import oracle as O
from paper_2604_26745_amd import inputs

CFG = inputs.SCANNER_165


def geometry(oversample, **kw):
    d = inputs.scanner_geometry(CFG, oversample)
    d.update(kw)
    y_scale = d.pop("y_scale")
    return O.Geometry(d["n"], d["n_angles"], d["n_bins"], bin_size=d["bin_size"], step=d["step"],
                      psf_sigma=d["psf_sigma"], atten_scale=d["atten_scale"]), y_scale


def grid_mm(oversample):
    n = CFG.n * oversample
    px = CFG.pixel_mm / oversample
    c = (np.arange(n) - 0.5 * (n - 1)) * px
    return np.meshgrid(c, c)


def test_uniform_disk_projects_to_chord_lengths():
    g, ys = geometry(1, n_angles=8, psf_sigma=0.0)
    X, Y = grid_mm(1)
    R = 40.0
    # 8 x 8 supersampled disk (area-weighted pixels; offsets in mm)
    sub = 8
    off = ((np.arange(sub) + 0.5) / sub - 0.5) * CFG.pixel_mm
    f = np.zeros_like(X)
    for a in off:
        for b in off:
            f += ((X + a) ** 2 + (Y + b) ** 2 <= R * R)
    f /= sub * sub
    y = ys * O.forward(g, f, np.zeros_like(f))
    s = (np.arange(CFG.n_bins) - 0.5 * (CFG.n_bins - 1)) * CFG.bin_mm
    chord = 2.0 * np.sqrt(np.maximum(R * R - s * s, 0.0))
    inner = np.abs(s) < R - 3.0
    for a in range(8):
        # mm: sampling an area-weighted edge every pixel (2 mm) along the ray
        # moves the chord by a fraction of a sample; a wrong bin spacing would
        # shift it by tens of mm
        err = np.abs(y[a, inner] - chord[inner]).max()
        assert err < 0.5 * CFG.pixel_mm, (a, err)
        assert np.linalg.norm(y[a, inner] - chord[inner]) / np.linalg.norm(chord[inner]) < 1e-2
    # total: every angle integrates the disk area (pi R^2 in mm^2) over bins of 2 mm
    assert abs(y.sum(axis=1).mean() * CFG.bin_mm - math.pi * R * R) / (math.pi * R * R) < 2e-3


def test_fine_grid_projection_matches_reconstruction_grid():
    def smooth(oversample):
        X, Y = grid_mm(oversample)
        f = np.exp(-((X - 10.0) ** 2 + (Y + 5.0) ** 2) / (2 * 18.0 ** 2))
        mu = 0.06 * np.exp(-((X + 8.0) ** 2 + (Y - 12.0) ** 2) / (2 * 25.0 ** 2))
        return f, mu
    g1, s1 = geometry(1, n_angles=24)
    g2, s2 = geometry(2, n_angles=24)
    y1 = s1 * O.forward(g1, *smooth(1))
    y2 = s2 * O.forward(g2, *smooth(2))
    rel = np.linalg.norm(y2 - y1) / np.linalg.norm(y1)
    assert rel < 2e-3, rel
    # attenuation per pixel of the coarse grid on the fine grid (a factor-2
    # slip in the pixel size) would be a gross mismatch
    g2_wrong = O.Geometry(g2.n, g2.n_angles, g2.n_bins, bin_size=g2.bin_size, step=g2.step,
                          psf_sigma=g2.psf_sigma, atten_scale=2.0 * g2.atten_scale)
    y2_wrong = s2 * O.forward(g2_wrong, *smooth(2))
    assert np.linalg.norm(y2_wrong - y1) / np.linalg.norm(y1) > 20 * rel


def test_phantom_totals_agree_across_resolutions():
    for kind in ("full", "missing", "replaced", "medium"):
        f1, mu1 = inputs.scanner_phantom(CFG, 3, kind, 1)
        f2, mu2 = inputs.scanner_phantom(CFG, 3, kind, 2)
        assert abs(f2.sum() / 4.0 - f1.sum()) <= 1e-3 * f1.sum()
        assert abs(mu2.sum() / 4.0 - mu1.sum()) <= 1e-3 * mu1.sum()
        assert f1.max() <= 1.0 and mu1.max() <= 0.14 + 1e-12


def test_noise_level():
    y = np.linspace(1.0, 2.0, 5000)
    yn = inputs.gaussian_noise(y, 0.02, 0)
    assert abs(np.linalg.norm(yn - y) / np.linalg.norm(y) - 0.02) < 2e-3


def test_rod_prior_holds_for_every_phantom_kind():
    """The geometry prior's region and references agree with the phantoms it
    is meant for: no emission there, attenuation equal to the reference
    (water in the field of view) except on pixels the field-of-view circle
    cuts, for every kind and several seeds (rod jitter included)."""
    out, ref_f, ref_mu = inputs.scanner_rod_prior(CFG)
    # the region is the image minus 81 disks of radius rod + jitter + a pixel
    # (to the pixel-centre discretisation of disks about 4 pixels across:
    # a few percent of their area)
    reach = CFG.rod_radius_mm + CFG.jitter_mm + CFG.pixel_mm
    expect = 1.0 - CFG.n_rods ** 2 * math.pi * reach ** 2 / (CFG.n * CFG.pixel_mm) ** 2
    assert abs(out.mean() - expect) < 0.02 and np.all(ref_f == 0.0)
    cc = np.arange(CFG.n) - 0.5 * (CFG.n - 1)
    X, Y = np.meshgrid(cc, cc)
    edge = np.abs(np.sqrt(X ** 2 + Y ** 2) - 0.5 * CFG.n) < 1.0
    on = (out > 0) & ~edge
    for seed in range(3):
        for kind in ("full", "missing", "replaced", "medium"):
            f, mu = inputs.scanner_phantom(CFG, seed, kind, 1)
            assert f[out > 0].max() == 0.0
            assert np.abs(mu - ref_mu)[on].max() <= 1e-12
    # a rod that the prior region covered would show up as emission there
    wider = inputs.scanner_rod_prior(CFG, margin_mm=-CFG.rod_radius_mm)[0]
    f, _ = inputs.scanner_phantom(CFG, 0, "full", 1)
    assert f[wider > 0].max() > 0.5


def test_lattice_rod_prior_holds():
    cfg = inputs.MAIN_128
    out, ref_f, ref_mu = inputs.lattice_rod_prior(cfg)
    for seed in range(4):
        f, mu = inputs.rod_lattice(cfg, seed)
        assert f[out > 0].max() == 0.0
        assert np.abs(mu - ref_mu)[out > 0].max() <= 1e-12


def test_full_model_tables():
    """The full discrete model's per-sample tables for the scanner plans:
    alpha linear from 1 (sample 0, farthest from the detector) to 0, the
    vertical correction 1 + 0.05 alpha, the far taps a normalised symmetric
    Gaussian of 2 bins over the taps the full-model plan uses."""
    import math
    import numpy as np
    from paper_2604_26745_amd import inputs
    cfg = inputs.SCANNER_165
    for o in (1, cfg.oversample):
        d = inputs.scanner_geometry(cfg, o, full_model=True)
        K = d["psf_radius"]
        assert K == math.ceil(3 * cfg.psf_sigma_far_bins)
        n_t = 2 * math.ceil(d["n"] / math.sqrt(2.0) + 1.0)
        depth, alpha, far = inputs.scanner_full_model(cfg, n_t)
        a = np.array(alpha)
        assert len(alpha) == len(depth) == n_t and len(far) == 2 * K + 1
        assert a[0] == 1.0 and a[-1] == 0.0 and np.allclose(np.diff(a), -1.0 / (n_t - 1))
        assert np.allclose(depth, 1.0 + (cfg.depth_factor_far - 1.0) * a)
        t = np.array(far)
        assert abs(t.sum() - 1.0) < 1e-12 and np.array_equal(t, t[::-1])
        k = np.arange(-K, K + 1)
        var = float((k ** 2 * t).sum())
        assert 0.8 * cfg.psf_sigma_far_bins ** 2 < var < cfg.psf_sigma_far_bins ** 2
