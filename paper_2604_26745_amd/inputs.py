"""Seeded synthetic inputs: rod-lattice phantoms, count noise, request traces.

This module holds no arithmetic of the reconstruction method.  It only draws
the test objects (emission and attenuation maps of a fuel-assembly-like rod
lattice, Sec. 3.3 of the paper describes the family it imitates), the
counting noise applied to a clean sinogram someone else computed, and the
arrival times of a request stream.  Both the CPU oracle's tests and the GPU
path use it, so that both see the same inputs.

Phantom recipe: a square can of coolant (background attenuation, no
emission) holding an n_rods x n_rods square lattice of disk rods.  Rods are
centred at ((k - (n_rods-1)/2) * pitch, (l - (n_rods-1)/2) * pitch); a few
randomly chosen rods are empty (replaced by coolant: no emission, background
attenuation).  Each pixel value is the mean over a 4 x 4 sub-pixel grid, so
rod edges are area-weighted.  Random draws, in this order, from
``numpy.random.default_rng([seed, 0])``: the empty rod indices (without
replacement), the emission of each rod (row-major), the attenuation of each
rod (row-major, when it is drawn).  Noise draws from ``default_rng([seed, 1])``;
mixed-size configurations draw their size/lattice from ``default_rng([seed, 2])``
and request arrivals from ``default_rng([seed, 3])``; the scanner-geometry
phantoms (``scanner_phantom``) draw from ``default_rng([seed, 6])`` and their
Gaussian noise from ``default_rng([seed, 5])``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class SliceConfig:
    """One slice: geometry, phantom family and solver sizes."""

    name: str
    n: int
    n_angles: int
    n_bins: int
    psf_sigma: float = 1.5
    n_rods: int = 9
    rod_radius: float = 2.0
    pitch: float = 6.0
    can_half: float = 27.0
    rod_mu: Optional[float] = 0.05           # fixed rod attenuation, or None -> uniform draw
    rod_mu_range: Tuple[float, float] = (0.03, 0.08)
    bg_mu: float = 0.01
    f_sigma: float = 0.3                     # rod emission ~ lognormal(0, f_sigma)
    n_empty: int = 5
    peak_counts: float = 1e4
    max_outer: int = 15
    n_cg: int = 20
    alpha: float = 1e-2


# The five workloads.  Sizes in pixels, angles over a full turn.
SMALL_64 = SliceConfig("lattice9_n64_a120_b96", 64, 120, 96)
MAIN_128 = SliceConfig(
    "lattice9_n128_a360_b192", 128, 360, 192, rod_radius=4.0, pitch=12.0,
    can_half=54.0, n_cg=30,
)
LARGE_256 = SliceConfig(
    "lattice17_n256_a360_b256", 256, 360, 256, n_rods=17, rod_radius=3.0,
    pitch=10.0, can_half=85.0, rod_mu=None, f_sigma=0.5, n_empty=29, n_cg=30,
)
MIX_SIZES = (64, 96, 128, 192, 256)


def mixed_config(seed: int) -> Tuple[SliceConfig, float]:
    """One slice of the mixed-size batch: size G in MIX_SIZES, 360 angles,
    1.5 G bins, 9x9 or 17x17 lattice (even odds), can half-side 0.42 G,
    pitch 2h/n_rods, rod radius pitch/3, 0..ceil(0.1 n^2) empty rods, peak
    counts 10**U(3, 5).  Returns (config, peak)."""
    rng = np.random.default_rng([seed, 2])
    G = int(MIX_SIZES[rng.integers(0, len(MIX_SIZES))])
    big = bool(rng.integers(0, 2))
    n_rods = 17 if big else 9
    h = 0.42 * G
    pitch = 2.0 * h / n_rods
    n_empty = int(rng.integers(0, math.ceil(0.1 * n_rods * n_rods) + 1))
    peak = float(10.0 ** rng.uniform(3.0, 5.0))
    cfg = SliceConfig(
        "mix_n%d_r%d" % (G, n_rods), G, 360, int(round(1.5 * G)), n_rods=n_rods,
        rod_radius=pitch / 3.0, pitch=pitch, can_half=h,
        rod_mu=None if big else 0.05, f_sigma=0.5 if big else 0.3,
        n_empty=n_empty, peak_counts=peak, n_cg=30,
    )
    return cfg, peak


def rod_lattice(cfg: SliceConfig, seed: int = 0):
    """Ground-truth emission f and attenuation mu (N x N, float64)."""
    rng = np.random.default_rng([seed, 0])
    nr = cfg.n_rods
    n_rod_total = nr * nr
    empty = set(int(i) for i in rng.choice(n_rod_total, size=cfg.n_empty, replace=False)) \
        if cfg.n_empty > 0 else set()
    rod_f = rng.lognormal(0.0, cfg.f_sigma, size=n_rod_total)
    if cfg.rod_mu is None:
        rod_mu = rng.uniform(cfg.rod_mu_range[0], cfg.rod_mu_range[1], size=n_rod_total)
    else:
        rod_mu = np.full(n_rod_total, cfg.rod_mu)

    n = cfg.n
    sub = 4
    off = (np.arange(sub) + 0.5) / sub - 0.5
    cc = np.arange(n) - 0.5 * (n - 1)
    # sub-pixel sample coordinates, shape (n*sub,)
    xs = (cc[:, None] + off[None, :]).reshape(-1)
    X, Y = np.meshgrid(xs, xs)          # X: column coordinate, Y: row coordinate
    f_hi = np.zeros_like(X)
    in_can = (np.abs(X) <= cfg.can_half) & (np.abs(Y) <= cfg.can_half)
    mu_hi = np.where(in_can, cfg.bg_mu, 0.0)
    for idx in range(n_rod_total):
        if idx in empty:
            continue
        l, k = divmod(idx, nr)          # row-major: l = lattice row, k = lattice column
        cx = (k - 0.5 * (nr - 1)) * cfg.pitch
        cy = (l - 0.5 * (nr - 1)) * cfg.pitch
        # window of sub-samples that can lie inside this rod
        lo_c = max(0, int(np.searchsorted(xs, cx - cfg.rod_radius - 1.0)))
        hi_c = min(xs.size, int(np.searchsorted(xs, cx + cfg.rod_radius + 1.0)))
        lo_r = max(0, int(np.searchsorted(xs, cy - cfg.rod_radius - 1.0)))
        hi_r = min(xs.size, int(np.searchsorted(xs, cy + cfg.rod_radius + 1.0)))
        Xw = X[lo_r:hi_r, lo_c:hi_c]
        Yw = Y[lo_r:hi_r, lo_c:hi_c]
        inside = (Xw - cx) ** 2 + (Yw - cy) ** 2 <= cfg.rod_radius ** 2
        f_hi[lo_r:hi_r, lo_c:hi_c][inside] = rod_f[idx]
        mu_hi[lo_r:hi_r, lo_c:hi_c][inside] = rod_mu[idx]
    f = f_hi.reshape(n, sub, n, sub).mean(axis=(1, 3))
    mu = mu_hi.reshape(n, sub, n, sub).mean(axis=(1, 3))
    return f, mu


# ---- scanner geometry (physical units: millimetres)

@dataclass(frozen=True)
class ScannerConfig:
    """A slice in the geometry of the measurement device: two banks of 91
    detector elements whose readings interleave over a full turn to 182 bins
    at 2 mm, a 165 x 165 reconstruction grid, data generated on a grid
    ``oversample`` times finer.  Readings where the paper gives no number:
    pixels of the detector spacing, 2 mm (a 330 mm field inside the 364 mm
    detector span, the assembly a central section of the image), 360
    angles, collimator response a Gaussian of 1 bin (2 mm) standard
    deviation, a 9 x 9 lattice at 14.4 mm pitch with 5.5 mm rod radius, rod
    centres perturbed by U(-0.5, 0.5) mm per axis, water filling the
    field-of-view disk.  The full discrete model (``scanner_full_model``)
    adds a response widening to a Gaussian of 2 bins at the far side of the
    field and a vertical correction of the attenuation path growing to 1.05
    there, both linear in depth."""

    name: str = "scanner9x9_n165_a360_b182"
    n: int = 165
    pixel_mm: float = 2.0
    n_angles: int = 360
    n_bins: int = 182
    bin_mm: float = 2.0
    psf_sigma_bins: float = 1.0
    psf_sigma_far_bins: float = 2.0     # full model: response at the far side of the field
    depth_factor_far: float = 1.05      # full model: vertical correction there
    oversample: int = 2
    n_rods: int = 9
    pitch_mm: float = 14.4
    rod_radius_mm: float = 5.5
    jitter_mm: float = 0.5
    rod_f_range: Tuple[float, float] = (6.5e5 / 7e5, 1.0)      # emission, in units of 7e5
    rod_mu_range: Tuple[float, float] = (0.12, 0.14)            # 1/mm
    water_mu: float = 0.0085                                    # 1/mm
    noise: float = 0.02
    max_outer: int = 15
    n_cg: int = 30
    alpha: float = 1e-2


SCANNER_165 = ScannerConfig()


def scanner_geometry(cfg: ScannerConfig, oversample: int = 1, full_model: bool = False) -> dict:
    """Plan arguments of the device geometry on a grid `oversample` times
    finer than cfg.n: pixel size p = pixel_mm / oversample, bins and samples
    in pixel units, attenuation per mm (atten_scale = p), and the factor p
    that turns the plan's ray sums (step of one pixel) into millimetres.
    With the full model the collimator taps span 3 far-response sigmas."""
    p = cfg.pixel_mm / oversample
    d = dict(n=cfg.n * oversample, n_angles=cfg.n_angles, n_bins=cfg.n_bins,
             bin_size=cfg.bin_mm / p, step=1.0, psf_sigma=cfg.psf_sigma_bins,
             atten_scale=p, y_scale=p)
    if full_model:
        d["psf_radius"] = int(math.ceil(3.0 * cfg.psf_sigma_far_bins))
    return d


def scanner_full_model(cfg: ScannerConfig, n_samples: int):
    """Per-sample tables of the full discrete model for a plan of the device
    geometry with ``n_samples`` samples per ray: (depth factor, alpha of the
    far response, far taps), linear in depth from the detector side (1, 0)
    to the far side (depth_factor_far, 1)."""
    K = int(math.ceil(3.0 * cfg.psf_sigma_far_bins))
    alpha, far = collimator_depth_response(n_samples, K, cfg.psf_sigma_far_bins)
    depth = tuple(1.0 + (cfg.depth_factor_far - 1.0) * a for a in alpha)
    return depth, alpha, far


def scanner_phantom(cfg: ScannerConfig, seed: int = 0, kind: str = "missing", oversample: int = 1):
    """Emission f (units of 7e5) and attenuation mu (1/mm) of a 9 x 9
    assembly on the (oversample * n)^2 grid, 4 x 4 supersampled per pixel.

    kind: "full" (all rods), "missing" (1..6 rods replaced by water),
    "replaced" (5..6 rods without emission, attenuation kept), "medium"
    (1..20 rods missing or replaced, present rods' emission down to 70 % of
    the range's top).  Draws from ``default_rng([seed, 6])`` in this order:
    rod jitter (x then y, row-major), emission, attenuation, the number of
    changed rods, their indices, and (medium) which are replaced and the
    emission scale of the others."""
    rng = np.random.default_rng([seed, 6])
    nr = cfg.n_rods
    nt = nr * nr
    jx = rng.uniform(-cfg.jitter_mm, cfg.jitter_mm, size=nt)
    jy = rng.uniform(-cfg.jitter_mm, cfg.jitter_mm, size=nt)
    rod_f = rng.uniform(cfg.rod_f_range[0], cfg.rod_f_range[1], size=nt)
    rod_mu = rng.uniform(cfg.rod_mu_range[0], cfg.rod_mu_range[1], size=nt)
    missing, replaced = set(), set()
    if kind == "missing":
        missing = set(int(i) for i in rng.choice(nt, size=int(rng.integers(1, 7)), replace=False))
    elif kind == "replaced":
        replaced = set(int(i) for i in rng.choice(nt, size=int(rng.integers(5, 7)), replace=False))
    elif kind == "medium":
        changed = rng.choice(nt, size=int(rng.integers(1, 21)), replace=False)
        rep = rng.integers(0, 2, size=changed.size)
        missing = set(int(i) for i, r in zip(changed, rep) if not r)
        replaced = set(int(i) for i, r in zip(changed, rep) if r)
        rod_f = rod_f * rng.uniform(0.7, 1.0, size=nt)
    elif kind != "full":
        raise ValueError("kind must be full, missing, replaced or medium")
    n = cfg.n * oversample
    px = cfg.pixel_mm / oversample
    sub = 4
    off = ((np.arange(sub) + 0.5) / sub - 0.5) * px
    cc = (np.arange(n) - 0.5 * (n - 1)) * px
    xs = (cc[:, None] + off[None, :]).reshape(-1)
    X, Y = np.meshgrid(xs, xs)
    fov = X ** 2 + Y ** 2 <= (0.5 * cfg.n * cfg.pixel_mm) ** 2
    f_hi = np.zeros_like(X)
    mu_hi = np.where(fov, cfg.water_mu, 0.0)
    r = cfg.rod_radius_mm
    for idx in range(nt):
        if idx in missing:
            continue
        l, k = divmod(idx, nr)
        cx = (k - 0.5 * (nr - 1)) * cfg.pitch_mm + jx[idx]
        cy = (l - 0.5 * (nr - 1)) * cfg.pitch_mm + jy[idx]
        lo_c = max(0, int(np.searchsorted(xs, cx - r - px)))
        hi_c = min(xs.size, int(np.searchsorted(xs, cx + r + px)))
        lo_r = max(0, int(np.searchsorted(xs, cy - r - px)))
        hi_r = min(xs.size, int(np.searchsorted(xs, cy + r + px)))
        Xw = X[lo_r:hi_r, lo_c:hi_c]
        Yw = Y[lo_r:hi_r, lo_c:hi_c]
        inside = (Xw - cx) ** 2 + (Yw - cy) ** 2 <= r * r
        f_hi[lo_r:hi_r, lo_c:hi_c][inside] = 0.0 if idx in replaced else rod_f[idx]
        mu_hi[lo_r:hi_r, lo_c:hi_c][inside] = rod_mu[idx]
    f = f_hi.reshape(n, sub, n, sub).mean(axis=(1, 3))
    mu = mu_hi.reshape(n, sub, n, sub).mean(axis=(1, 3))
    return f, mu


def _outside_rods(n: int, px: float, centres, reach: float) -> np.ndarray:
    """1 where a pixel centre lies farther than `reach` from every centre."""
    cc = (np.arange(n) - 0.5 * (n - 1)) * px
    X, Y = np.meshgrid(cc, cc)
    out = np.ones((n, n))
    for cx, cy in centres:
        out[(X - cx) ** 2 + (Y - cy) ** 2 <= reach * reach] = 0.0
    return out


def scanner_rod_prior(cfg: ScannerConfig, margin_mm: Optional[float] = None):
    """Where the geometry prior applies (the paper's P1, P2: emission and
    attenuation away from every possible rod location of the known 9 x 9
    layout are penalised; no rod is assumed present).  Returns
    (outside, ref_f, ref_mu) on the reconstruction grid: `outside` is 1 for
    pixels whose centre is farther than rod radius + jitter + margin from
    every nominal rod centre (margin: one pixel by default, more than the
    pixel's half-diagonal, so that no such pixel overlaps a rod), the
    references are no emission there and water attenuation inside the field
    of view (0 outside it)."""
    if margin_mm is None:
        margin_mm = cfg.pixel_mm
    nr = cfg.n_rods
    centres = [((k - 0.5 * (nr - 1)) * cfg.pitch_mm, (l - 0.5 * (nr - 1)) * cfg.pitch_mm)
               for l in range(nr) for k in range(nr)]
    out = _outside_rods(cfg.n, cfg.pixel_mm, centres, cfg.rod_radius_mm + cfg.jitter_mm + margin_mm)
    ref_mu = np.where(fov_mask(cfg), cfg.water_mu, 0.0)
    return out, np.zeros_like(out), ref_mu


def lattice_rod_prior(cfg: SliceConfig, margin: float = 1.0):
    """The same for the rod-lattice phantoms (pixel units): 1 farther than
    rod radius + margin from every nominal centre; references no emission
    and the background attenuation inside the can (0 outside it)."""
    nr = cfg.n_rods
    centres = [((k - 0.5 * (nr - 1)) * cfg.pitch, (l - 0.5 * (nr - 1)) * cfg.pitch)
               for l in range(nr) for k in range(nr)]
    out = _outside_rods(cfg.n, 1.0, centres, cfg.rod_radius + margin)
    cc = np.arange(cfg.n) - 0.5 * (cfg.n - 1)
    X, Y = np.meshgrid(cc, cc)
    can = (np.abs(X) <= cfg.can_half) & (np.abs(Y) <= cfg.can_half)
    return out, np.zeros_like(out), np.where(can, cfg.bg_mu, 0.0)


def collimator_depth_response(n_samples: int, half_width: int, sigma_far: float):
    """A depth-dependent collimator response for the discrete model: the
    response at the far side of the field is a Gaussian of ``sigma_far``
    bins over the plan's 2K + 1 taps (normalised), and its weight alpha
    grows linearly from 0 at the sample nearest the detector to 1 at the
    farthest (sample 0), so the response widens with the emitter's
    distance.  Returns (alpha, far_taps) as tuples."""
    k = np.arange(-half_width, half_width + 1)
    t = np.exp(-(k ** 2) / (2.0 * sigma_far ** 2))
    t /= t.sum()
    alpha = 1.0 - np.arange(n_samples) / max(n_samples - 1, 1)
    return tuple(float(v) for v in alpha), tuple(float(v) for v in t)


def fov_mask(cfg: ScannerConfig) -> np.ndarray:
    """Pixels of the reconstruction grid whose centre lies in the field-of-view disk."""
    cc = np.arange(cfg.n) - 0.5 * (cfg.n - 1)
    X, Y = np.meshgrid(cc, cc)
    return X ** 2 + Y ** 2 <= (0.5 * cfg.n) ** 2


def gaussian_noise(y_clean: np.ndarray, level: float, seed: int = 0) -> np.ndarray:
    """y = y_clean + e, e white Gaussian with ||e|| about level * ||y_clean||
    (standard deviation level * rms(y_clean)); draws from default_rng([seed, 5])."""
    rng = np.random.default_rng([seed, 5])
    y_clean = np.asarray(y_clean, dtype=np.float64)
    sd = level * float(np.sqrt(np.mean(y_clean * y_clean)))
    return y_clean + sd * rng.standard_normal(y_clean.shape)


def poisson_counts(y_clean: np.ndarray, peak: float, seed: int = 0) -> np.ndarray:
    """y = Poisson(kappa * y_clean) / kappa with kappa = peak / max(y_clean)."""
    rng = np.random.default_rng([seed, 1])
    y_clean = np.asarray(y_clean, dtype=np.float64)
    kappa = peak / float(np.max(y_clean))
    return rng.poisson(np.maximum(kappa * y_clean, 0.0)).astype(np.float64) / kappa


def random_like(shape, seed: int, scale: float = 1.0, kind: str = "normal") -> np.ndarray:
    """Seeded test vectors (directions, cotangents)."""
    rng = np.random.default_rng([seed, 7])
    if kind == "normal":
        return scale * rng.standard_normal(shape)
    return scale * rng.uniform(0.0, 1.0, size=shape)


def arrival_times(rate: float, duration: float, seed: int = 0) -> np.ndarray:
    """Open-loop Poisson arrivals (seconds) at ``rate`` per second over ``duration``."""
    rng = np.random.default_rng([seed, 3])
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(t)
    return np.asarray(out)


def scaled(cfg: SliceConfig, **kw) -> SliceConfig:
    return replace(cfg, **kw)
