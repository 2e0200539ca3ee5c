"""FP64 CPU oracle for the PGET Levenberg-Marquardt hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library: the operators live in ``pget_oracle.c`` (plain C,
double precision), the solver in :mod:`oracle.lm` (numpy, double precision),
and a dense brute-force formulation of the same operators in
:mod:`oracle.dense` (numpy, tiny grids only).

What it computes follows the paper (arXiv 2604.26745):

* Sec. 2.1, eq. (fwd_model) and its discrete form eq. (d_fwd_model): the
  attenuated ray transform of emission ``f`` (the paper's lambda) and
  attenuation ``mu`` with a collimator response, maps rotated per angle.
* Sec. 2.1, eq. (frechet): the two Frechet derivatives, and their adjoint.
* Sec. 2.1, eq. (lma_objective) and Sec. 2.2: the regularised least-squares
  objective, here with a gradient (Tikhonov) penalty.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pget_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpget_oracle.so")


def build_oracle(force: bool = False) -> str:
    """Compile ``pget_oracle.c`` with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CGeometry(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("n_angles", ctypes.c_int),
        ("n_bins", ctypes.c_int),
        ("psf_radius", ctypes.c_int),
        ("angle0", ctypes.c_double),
        ("arc", ctypes.c_double),
        ("bin_size", ctypes.c_double),
        ("step", ctypes.c_double),
        ("psf_sigma", ctypes.c_double),
        ("atten_scale", ctypes.c_double),
        ("depth", ctypes.POINTER(ctypes.c_double)),
        ("resp", ctypes.POINTER(ctypes.c_double)),
        ("far_taps", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_oracle()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_CGeometry)
        D = ctypes.POINTER(ctypes.c_double)
        lib.og_n_samples.argtypes = [P]
        lib.og_n_samples.restype = ctypes.c_int
        lib.og_psf_half_width.argtypes = [P]
        lib.og_psf_half_width.restype = ctypes.c_int
        lib.og_psf_taps.argtypes = [P, D]
        lib.og_forward.argtypes = [P, D, D, D]
        lib.og_forward_raw.argtypes = [P, D, D, D]
        lib.og_psf.argtypes = [P, D, D]
        lib.og_psf_transpose.argtypes = [P, D, D]
        lib.og_jvp.argtypes = [P, D, D, D, D, D]
        lib.og_vjp.argtypes = [P, D, D, D, D, D]
        lib.og_reg_energy.argtypes = [ctypes.c_int, ctypes.c_double, D]
        lib.og_reg_energy.restype = ctypes.c_double
        lib.og_reg_gradient.argtypes = [ctypes.c_int, ctypes.c_double, D, D]
        _lib = lib
    return _lib


@dataclass(frozen=True)
class Geometry:
    """Parallel-beam geometry of one slice (pixel units, radians)."""

    n: int
    n_angles: int
    n_bins: int
    angle0: float = 0.0
    arc: float = 2.0 * math.pi
    bin_size: float = 1.0
    step: float = 1.0
    psf_sigma: float = 1.5
    psf_radius: int = -1
    atten_scale: float = 1.0
    # per-sample depth factor d_i of the attenuation path (n_samples values,
    # sample 0 farthest from the detector), or None for d_i = 1
    depth: Optional[Tuple[float, ...]] = None
    # depth-dependent collimator response: sample i is seen through
    # (1 - resp_i) times the Gaussian taps plus resp_i times far_taps
    # (2K + 1 values); None for the same response at every depth
    resp: Optional[Tuple[float, ...]] = None
    far_taps: Optional[Tuple[float, ...]] = None

    def _c(self) -> _CGeometry:
        c = _CGeometry(
            self.n, self.n_angles, self.n_bins, self.psf_radius, self.angle0,
            self.arc, self.bin_size, self.step, self.psf_sigma, self.atten_scale, None, None, None,
        )
        keep = []
        for name in ("depth", "resp", "far_taps"):
            vals = getattr(self, name)
            if vals is not None:
                arr = (ctypes.c_double * len(vals))(*vals)
                setattr(c, name, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)))
                keep.append(arr)
        c._keep = keep
        lib = _load()
        if self.depth is not None and len(self.depth) != lib.og_n_samples(ctypes.byref(c)):
            raise ValueError("depth needs one value per sample along a ray")
        if (self.resp is None) != (self.far_taps is None):
            raise ValueError("resp and far_taps go together")
        if self.resp is not None:
            if len(self.resp) != lib.og_n_samples(ctypes.byref(c)):
                raise ValueError("resp needs one value per sample along a ray")
            if len(self.far_taps) != 2 * lib.og_psf_half_width(ctypes.byref(c)) + 1:
                raise ValueError("far_taps needs 2K + 1 values")
        return c

    @property
    def n_samples(self) -> int:
        return _load().og_n_samples(ctypes.byref(self._c()))

    @property
    def psf_half_width(self) -> int:
        return _load().og_psf_half_width(ctypes.byref(self._c()))

    @property
    def sino_shape(self):
        return (self.n_angles, self.n_bins)

    @property
    def image_shape(self):
        return (self.n, self.n)


def _d(a: np.ndarray, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def psf_taps(g: Geometry) -> np.ndarray:
    K = g.psf_half_width
    out = np.empty(2 * K + 1)
    _load().og_psf_taps(ctypes.byref(g._c()), _ptr(out))
    return out


def forward(g: Geometry, f, mu) -> np.ndarray:
    """y = A(f, mu), shape (n_angles, n_bins)."""
    f = _d(f, g.image_shape)
    mu = _d(mu, g.image_shape)
    y = np.empty(g.sino_shape)
    _load().og_forward(ctypes.byref(g._c()), _ptr(f), _ptr(mu), _ptr(y))
    return y


def forward_raw(g: Geometry, f, mu) -> np.ndarray:
    """Ray sums before the collimator blur."""
    f = _d(f, g.image_shape)
    mu = _d(mu, g.image_shape)
    p = np.empty(g.sino_shape)
    _load().og_forward_raw(ctypes.byref(g._c()), _ptr(f), _ptr(mu), _ptr(p))
    return p


def psf(g: Geometry, p) -> np.ndarray:
    p = _d(p, g.sino_shape)
    y = np.empty(g.sino_shape)
    _load().og_psf(ctypes.byref(g._c()), _ptr(p), _ptr(y))
    return y


def psf_transpose(g: Geometry, w) -> np.ndarray:
    w = _d(w, g.sino_shape)
    v = np.empty(g.sino_shape)
    _load().og_psf_transpose(ctypes.byref(g._c()), _ptr(w), _ptr(v))
    return v


def jvp(g: Geometry, f, mu, vf, vmu) -> np.ndarray:
    """J(f, mu) [vf, vmu], shape (n_angles, n_bins)."""
    args = [_d(x, g.image_shape) for x in (f, mu, vf, vmu)]
    out = np.empty(g.sino_shape)
    _load().og_jvp(ctypes.byref(g._c()), *[_ptr(x) for x in args], _ptr(out))
    return out


def vjp(g: Geometry, f, mu, w):
    """J(f, mu)^T w -> (g_f, g_mu), each (n, n)."""
    f = _d(f, g.image_shape)
    mu = _d(mu, g.image_shape)
    w = _d(w, g.sino_shape)
    gf = np.empty(g.image_shape)
    gm = np.empty(g.image_shape)
    _load().og_vjp(ctypes.byref(g._c()), _ptr(f), _ptr(mu), _ptr(w), _ptr(gf), _ptr(gm))
    return gf, gm


def reg_energy(alpha: float, x) -> float:
    """0.5 * alpha * ||grad x||^2 (forward differences, Neumann boundary)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    return float(_load().og_reg_energy(n, float(alpha), _ptr(x)))


def reg_gradient(alpha: float, x) -> np.ndarray:
    """alpha * grad^T grad x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    out = np.empty_like(x)
    _load().og_reg_gradient(n, float(alpha), _ptr(x), _ptr(out))
    return out


__all__ = [
    "Geometry", "build_oracle", "forward", "forward_raw", "psf", "psf_transpose",
    "psf_taps", "jvp", "vjp", "reg_energy", "reg_gradient",
]
