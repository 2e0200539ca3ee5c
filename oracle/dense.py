"""Dense brute-force formulation of the forward map (test infrastructure only).

An independent second reading of Sec. 2.1, eq. (d_fwd_model), for tiny grids:
every interpolation weight is written into an explicit matrix by summing the
tent product over *all* pixels (no four-neighbour shortcut), the attenuation
sums are a triangular matrix product, and the collimator blur is a banded
matrix.  Nothing is shared with the C oracle or the HIP library; it exists so
that the C oracle can be checked against it, and so that torch autograd can
differentiate the same formula to check the hand-derived Jacobian products.
"""
from __future__ import annotations

import math

import numpy as np


def lattice(n: int, n_angles: int, n_bins: int, angle0: float = 0.0,
            arc: float = 2.0 * math.pi, bin_size: float = 1.0, step: float = 1.0):
    """Sample points q[a, j, i] = s_j omega_perp(theta_a) + t_i omega(theta_a)."""
    n_t = 2 * math.ceil((n / math.sqrt(2.0) + 1.0) / step)
    th = angle0 + np.arange(n_angles) * arc / n_angles
    s = (np.arange(n_bins) - 0.5 * (n_bins - 1)) * bin_size
    t = (np.arange(n_t) - 0.5 * (n_t - 1)) * step
    qx = -s[None, :, None] * np.sin(th)[:, None, None] + t[None, None, :] * np.cos(th)[:, None, None]
    qy = s[None, :, None] * np.cos(th)[:, None, None] + t[None, None, :] * np.sin(th)[:, None, None]
    return qx, qy, n_t


def interpolation_matrix(n: int, qx: np.ndarray, qy: np.ndarray) -> np.ndarray:
    """W[(a, j, i), m] = tent(qx - x_m) * tent(qy - y_m), over every pixel m."""
    half = 0.5 * (n - 1)
    xm = np.tile(np.arange(n) - half, n)      # column coordinate of pixel m = r*n + c
    ym = np.repeat(np.arange(n) - half, n)    # row coordinate
    dx = qx.reshape(-1, 1) - xm[None, :]
    dy = qy.reshape(-1, 1) - ym[None, :]
    return np.maximum(0.0, 1.0 - np.abs(dx)) * np.maximum(0.0, 1.0 - np.abs(dy))


def beam_matrix(n_t: int) -> np.ndarray:
    """U[i, i'] = 1/2 if i' == i, 1 if i' > i (toward the detector), else 0."""
    return np.triu(np.ones((n_t, n_t)), k=1) + 0.5 * np.eye(n_t)


def psf_matrix(n_bins: int, sigma: float, radius: int = -1) -> np.ndarray:
    """K[j, j'] = kappa_{j - j'} for |j - j'| <= radius (Gaussian, normalised)."""
    if sigma <= 0.0:
        return np.eye(n_bins)
    K = radius if radius >= 0 else math.ceil(3.0 * sigma)
    k = np.arange(-K, K + 1)
    kap = np.exp(-(k ** 2) / (2.0 * sigma ** 2))
    kap /= kap.sum()
    d = np.arange(n_bins)[:, None] - np.arange(n_bins)[None, :]
    M = np.zeros((n_bins, n_bins))
    mask = np.abs(d) <= K
    M[mask] = kap[d[mask] + K]
    return M


def banded_matrix(n_bins: int, taps) -> np.ndarray:
    """M[j, j'] = taps[j - j' + R] for |j - j'| <= R, with 2R + 1 taps given."""
    taps = np.asarray(taps, dtype=np.float64)
    R = (len(taps) - 1) // 2
    M = np.zeros((n_bins, n_bins))
    for j in range(n_bins):
        for jj in range(max(0, j - R), min(n_bins, j + R + 1)):
            M[j, jj] = taps[j - jj + R]
    return M


class DenseModel:
    """All matrices of one tiny geometry."""

    def __init__(self, n, n_angles, n_bins, psf_sigma=1.5, psf_radius=-1,
                 angle0=0.0, arc=2.0 * math.pi, bin_size=1.0, step=1.0, atten_scale=1.0, depth=None,
                 resp=None, far_taps=None):
        qx, qy, n_t = lattice(n, n_angles, n_bins, angle0, arc, bin_size, step)
        self.n, self.n_angles, self.n_bins, self.n_t = n, n_angles, n_bins, n_t
        self.step = step
        # path factor per sample: atten_scale times the depth factor d_i
        self.c = atten_scale * (np.ones(n_t) if depth is None else np.asarray(depth, dtype=np.float64))
        self.W = interpolation_matrix(n, qx, qy)          # (A*J*T, n*n)
        self.U = beam_matrix(n_t)                          # (T, T)
        self.K = psf_matrix(n_bins, psf_sigma, psf_radius)  # (J, J)
        # depth response: sample i is seen through (1 - resp_i) K + resp_i K_far
        self.resp = None if resp is None else np.asarray(resp, dtype=np.float64)
        self.K_far = None if far_taps is None else banded_matrix(n_bins, far_taps)

    def forward(self, f, mu, xp=np):
        """y = K [step * sum_i lam_i exp(-c_i * step * (U mu_hat)_i)], any array module."""
        A, J, T = self.n_angles, self.n_bins, self.n_t
        W = xp.asarray(self.W) if xp is not np else self.W
        U = xp.asarray(self.U) if xp is not np else self.U
        K = xp.asarray(self.K) if xp is not np else self.K
        lam = (W @ f.reshape(-1)).reshape(A, J, T)
        mh = (W @ mu.reshape(-1)).reshape(A, J, T)
        B = self.step * (mh @ U.T)                     # B[a,j,i] = step * sum_i' U[i,i'] mh[a,j,i']
        c = xp.asarray(self.c) if xp is not np else self.c
        if self.resp is None:
            p = self.step * (lam * xp.exp(-c * B)).sum(-1)   # (A, J)
            return p @ K.T                                  # y[a, j] = sum_j' K[j, j'] p[a, j']
        # the response is linear in resp_i: split every ray sum into the part
        # seen through K and the part seen through K_far
        al = xp.asarray(self.resp) if xp is not np else self.resp
        Kf = xp.asarray(self.K_far) if xp is not np else self.K_far
        le = lam * xp.exp(-c * B)
        p_near = self.step * ((1.0 - al) * le).sum(-1)
        p_far = self.step * (al * le).sum(-1)
        return p_near @ K.T + p_far @ Kf.T
