"""Thin ctypes binding of libpget (include/pget.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of ``libpget.so``.  torch tensors provide device memory and the
current HIP stream.  If the library is not built, every call raises
``RuntimeError`` -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpget.so")

PGET_OK = 0
STATUS_NAMES = {
    0: "ok", -1: "invalid argument", -2: "HIP runtime error", -3: "workspace missing or too small",
    -4: "non-finite value in the solver", -5: "unsupported geometry",
}
OP_FORWARD, OP_JVP, OP_VJP, OP_LM = 0, 1, 2, 3
STEP_CG, STEP_SGP = 0, 1
KC_MARCH, KC_JVP, KC_VJP, KC_VECTOR, KC_CONTROL, KC_GRADIENT = 0, 1, 2, 3, 4, 5
KERNEL_CLASS_NAMES = {KC_MARCH: "march", KC_JVP: "jvp", KC_VJP: "vjp", KC_VECTOR: "vector",
                      KC_CONTROL: "control", KC_GRADIENT: "gradient"}


class PgetError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s failed: %s (%d)" % (where, STATUS_NAMES.get(status, "?"), status))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_bins", ctypes.c_int32),
        ("psf_radius", ctypes.c_int32), ("angle0", ctypes.c_double), ("arc", ctypes.c_double),
        ("bin_size", ctypes.c_double), ("step", ctypes.c_double), ("psf_sigma", ctypes.c_double),
        ("atten_scale", ctypes.c_double),
    ]


class LMParams(ctypes.Structure):
    _fields_ = [
        ("max_outer", ctypes.c_int32), ("n_cg", ctypes.c_int32),
        ("alpha_f", ctypes.c_double), ("alpha_mu", ctypes.c_double),
        ("alpha_decay", ctypes.c_double), ("alpha_decay_until", ctypes.c_int32),
        ("beta0", ctypes.c_double), ("tau", ctypes.c_double), ("eta", ctypes.c_double),
        ("d_f", ctypes.c_double), ("d_mu", ctypes.c_double),
        ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double),
        ("mu_lo", ctypes.c_double), ("mu_hi", ctypes.c_double),
        ("tol", ctypes.c_double), ("replay", ctypes.POINTER(ctypes.c_int8)),
        ("w_f", ctypes.c_double), ("w_mu", ctypes.c_double), ("active_set", ctypes.c_int32),
        ("prior_w", ctypes.c_void_p), ("prior_ref", ctypes.c_void_p),
        ("trace_u", ctypes.c_void_p), ("trace_t", ctypes.c_void_p), ("step", ctypes.c_int32),
    ]


class LMReportC(ctypes.Structure):
    _fields_ = [
        ("scalars", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("rho", ctypes.c_void_p),
        ("beta", ctypes.c_void_p), ("pred", ctypes.c_void_p), ("ared", ctypes.c_void_p),
        ("gnorm", ctypes.c_void_p), ("accepted", ctypes.c_void_p),
        ("hook_accepted", ctypes.c_void_p), ("cg_rr", ctypes.c_void_p),
        ("hook_rho", ctypes.c_void_p), ("hook_pred", ctypes.c_void_p),
    ]


REFINE_FN = ctypes.CFUNCTYPE(
    ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
)

_lib = None


def load_library():
    """Load libpget.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libpget.so is not built (%s); run __graft_entry__.build() first" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.POINTER, ctypes.c_void_p
    lib.pget_plan_create.argtypes = [P(Geometry), ctypes.c_int, P(V)]
    lib.pget_plan_create.restype = ctypes.c_int
    lib.pget_plan_destroy.argtypes = [V]
    lib.pget_plan_destroy.restype = None
    lib.pget_plan_n_samples.argtypes = [V]
    lib.pget_plan_n_samples.restype = ctypes.c_int32
    lib.pget_plan_psf_half_width.argtypes = [V]
    lib.pget_plan_psf_half_width.restype = ctypes.c_int32
    lib.pget_plan_support_samples.argtypes = [V]
    lib.pget_plan_support_samples.restype = ctypes.c_int64
    lib.pget_plan_set_depth_factor.argtypes = [V, P(ctypes.c_double), ctypes.c_int32]
    lib.pget_plan_set_depth_factor.restype = ctypes.c_int
    lib.pget_plan_set_depth_response.argtypes = [V, P(ctypes.c_double), ctypes.c_int32, P(ctypes.c_double),
                                                 ctypes.c_int32]
    lib.pget_plan_set_depth_response.restype = ctypes.c_int
    lib.pget_timing_enable.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.pget_timing_enable.restype = ctypes.c_int
    lib.pget_timing_read.argtypes = [ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.pget_timing_read.restype = ctypes.c_int
    lib.pget_autotune.argtypes = [V, ctypes.c_int32, V, ctypes.c_size_t, V]
    lib.pget_autotune.restype = ctypes.c_int
    lib.pget_tuned_shape.argtypes = [V, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.pget_tuned_shape.restype = ctypes.c_int32
    lib.pget_set_shape.argtypes = [V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.pget_set_shape.restype = ctypes.c_int
    lib.pget_plan_set_band_staging.argtypes = [V, ctypes.c_int32]
    lib.pget_plan_set_band_staging.restype = ctypes.c_int
    lib.pget_plan_jvp_bands.argtypes = [V]
    lib.pget_plan_jvp_bands.restype = ctypes.c_int32
    lib.pget_workspace_bytes_multi.argtypes = [ctypes.c_int32, P(V)]
    lib.pget_workspace_bytes_multi.restype = ctypes.c_size_t
    lib.pget_lm_solve_multi.argtypes = [ctypes.c_int32, P(V), P(V), P(V), P(V), P(LMParams),
                                        P(LMReportC), V, ctypes.c_size_t, V]
    lib.pget_lm_solve_multi.restype = ctypes.c_int
    lib.pget_set_graphs.argtypes = [ctypes.c_int32]
    lib.pget_set_graphs.restype = ctypes.c_int
    lib.pget_workspace_bytes.argtypes = [V, ctypes.c_int32, ctypes.c_int32]
    lib.pget_workspace_bytes.restype = ctypes.c_size_t
    lib.pget_forward.argtypes = [V, V, V, V, V, V]
    lib.pget_forward.restype = ctypes.c_int
    lib.pget_forward_noalloc.argtypes = [V, V, V, V, V]
    lib.pget_forward_noalloc.restype = ctypes.c_int
    lib.pget_jvp.argtypes = [V, V, V, V, V, V, V, V, V]
    lib.pget_jvp.restype = ctypes.c_int
    lib.pget_vjp.argtypes = [V, V, V, V, V, V, V, V]
    lib.pget_vjp.restype = ctypes.c_int
    lib.pget_lm_solve.argtypes = [V, V, V, V, P(LMParams), REFINE_FN, V, P(LMReportC), V, V]
    lib.pget_lm_solve.restype = ctypes.c_int
    lib.pget_lm_solve_batched.argtypes = [V, ctypes.c_int32, P(V), P(V), P(V), P(LMParams),
                                          P(LMReportC), V, V]
    lib.pget_lm_solve_batched.restype = ctypes.c_int
    lib.pget_lm_pool_workspace_bytes.argtypes = [V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.pget_lm_pool_workspace_bytes.restype = ctypes.c_size_t
    lib.pget_lm_pool_create.argtypes = [V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, V,
                                        ctypes.c_size_t, V, P(V)]
    lib.pget_lm_pool_create.restype = ctypes.c_int
    lib.pget_lm_pool_destroy.argtypes = [V]
    lib.pget_lm_pool_destroy.restype = None
    lib.pget_lm_pool_load.argtypes = [V, ctypes.c_int32, V, V, V, P(LMParams), V]
    lib.pget_lm_pool_load.restype = ctypes.c_int
    lib.pget_lm_pool_step.argtypes = [V, V, V]
    lib.pget_lm_pool_step.restype = ctypes.c_int
    lib.pget_lm_pool_fetch.argtypes = [V, ctypes.c_int32, V, V, P(LMReportC), V]
    lib.pget_lm_pool_fetch.restype = ctypes.c_int
    lib.pget_status_string.argtypes = [ctypes.c_int]
    lib.pget_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(rc: int, where: str):
    if rc != PGET_OK:
        raise PgetError(rc, where)


@dataclass
class SolverParams:
    """Mirror of pget_lm_params (defaults: the readings of the paper used here)."""

    max_outer: int = 15
    n_cg: int = 30
    alpha_f: float = 1e-2
    alpha_mu: float = 1e-2
    alpha_decay: float = 1.0
    alpha_decay_until: int = 0
    beta0: float = 0.0
    tau: float = 1e-3
    eta: float = 1e-3
    d_f: float = 1.0
    d_mu: float = 1.0
    f_lo: float = 0.0
    f_hi: float = math.inf
    mu_lo: float = 0.0
    mu_hi: float = math.inf
    tol: float = 0.0
    replay: Optional[Sequence[int]] = None
    w_f: float = 1.0          # CG preconditioner W = diag(w_f I, w_mu I)
    w_mu: float = 1.0
    active_set: int = 0       # 1: CG on the variables not held at a bound
    prior_w: object = None    # geometry prior: CUDA float32 (2, N, N) weights, or None
    prior_ref: object = None  # its reference maps (2, N, N), or None (zero)
    trace_u: object = None    # iterate trace: CUDA float32 (max_outer, 2, N, N) receiving u_k, or None
    trace_t: object = None    # the same receiving the trial points u'_k, or None
    step: int = 0             # damped-step solver: STEP_CG (0) or STEP_SGP (1, scaled gradient projection)

    def to_c(self, n: Optional[int] = None):
        p = LMParams()
        for k, _ in LMParams._fields_:
            if k in ("replay", "prior_w", "prior_ref", "trace_u", "trace_t"):
                continue
            setattr(p, k, getattr(self, k))
        keep = []
        if self.replay is not None:
            # the library reads max_outer entries
            if len(self.replay) < self.max_outer:
                raise ValueError("replay holds %d decisions, max_outer is %d" % (len(self.replay), self.max_outer))
            arr = (ctypes.c_int8 * len(self.replay))(*[int(v) for v in self.replay])
            keep.append(arr)
            p.replay = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int8))
        for name in ("prior_w", "prior_ref"):
            t = getattr(self, name)
            if t is None:
                continue
            if not (t.is_cuda and t.dtype == _torch().float32 and t.is_contiguous()):
                raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)
            if n is not None and t.numel() != 2 * n * n:
                raise ValueError("%s must hold 2 x %d x %d values" % (name, n, n))
            keep.append(t)
            setattr(p, name, t.data_ptr())
        for name in ("trace_u", "trace_t"):
            t = getattr(self, name)
            if t is None:
                continue
            if not (t.is_cuda and t.dtype == _torch().float32 and t.is_contiguous()):
                raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)
            if n is not None and t.numel() != self.max_outer * 2 * n * n:
                raise ValueError("%s must hold max_outer x 2 x %d x %d values" % (name, n, n))
            keep.append(t)
            setattr(p, name, t.data_ptr())
        return p, keep


@dataclass
class LMReport:
    status: int = 0
    iters_run: int = 0
    beta_final: float = 0.0
    stop_reason: int = 0
    phi: List[float] = field(default_factory=list)
    rho: List[float] = field(default_factory=list)
    beta: List[float] = field(default_factory=list)
    pred: List[float] = field(default_factory=list)
    ared: List[float] = field(default_factory=list)
    gnorm: List[float] = field(default_factory=list)
    accepted: List[int] = field(default_factory=list)
    hook_accepted: List[int] = field(default_factory=list)
    cg_rr: List[List[float]] = field(default_factory=list)
    hook_rho: List[float] = field(default_factory=list)
    hook_pred: List[float] = field(default_factory=list)


class _ReportBuffers:
    """Device buffers one report is written into."""

    def __init__(self, max_outer: int, n_cg: int, device):
        torch = _torch()
        f64 = dict(dtype=torch.float64, device=device)
        self.max_outer, self.n_cg = max_outer, n_cg
        self.scalars = torch.zeros(4, **f64)
        self.phi = torch.full((max_outer + 1,), math.nan, **f64)
        self.rho = torch.zeros(max_outer, **f64)
        self.beta = torch.zeros(max_outer, **f64)
        self.pred = torch.zeros(max_outer, **f64)
        self.ared = torch.zeros(max_outer, **f64)
        self.gnorm = torch.zeros(max_outer, **f64)
        self.accepted = torch.zeros(max_outer, dtype=torch.int8, device=device)
        self.hook_accepted = torch.zeros(max_outer, dtype=torch.int8, device=device)
        self.cg_rr = torch.zeros(max_outer * n_cg, **f64)
        self.hook_rho = torch.full((max_outer,), math.nan, **f64)
        self.hook_pred = torch.full((max_outer,), math.nan, **f64)

    def c(self):
        r = LMReportC()
        for k, _ in LMReportC._fields_:
            setattr(r, k, getattr(self, k).data_ptr())
        return r

    def to_report(self) -> LMReport:
        sc = self.scalars.cpu().tolist()
        k = int(sc[1])
        return LMReport(
            status=int(sc[0]), iters_run=k, beta_final=sc[2], stop_reason=int(sc[3]),
            phi=self.phi.cpu().tolist()[: k + 1], rho=self.rho.cpu().tolist()[:k],
            beta=self.beta.cpu().tolist()[:k], pred=self.pred.cpu().tolist()[:k],
            ared=self.ared.cpu().tolist()[:k], gnorm=self.gnorm.cpu().tolist()[:k],
            accepted=self.accepted.cpu().tolist()[:k],
            hook_accepted=self.hook_accepted.cpu().tolist()[:k],
            cg_rr=self.cg_rr.view(self.max_outer, self.n_cg).cpu().tolist()[:k],
            hook_rho=self.hook_rho.cpu().tolist()[:k], hook_pred=self.hook_pred.cpu().tolist()[:k],
        )


class Plan:
    """A slice shape: geometry tables on the device plus cached workspaces."""

    def __init__(self, n: int, n_angles: int, n_bins: int, angle0: float = 0.0,
                 arc: float = 2.0 * math.pi, bin_size: float = 1.0, step: float = 1.0,
                 psf_sigma: float = 1.5, psf_radius: int = -1, atten_scale: float = 1.0,
                 storage: str = "fp32"):
        self.lib = load_library()
        self.geom = Geometry(n, n_angles, n_bins, psf_radius, angle0, arc, bin_size, step,
                             psf_sigma, atten_scale)
        if storage not in ("fp32", "bf16"):
            raise ValueError("storage must be 'fp32' or 'bf16'")
        self.storage = storage
        h = ctypes.c_void_p()
        _check(self.lib.pget_plan_create(ctypes.byref(self.geom), 0 if storage == "fp32" else 1,
                                          ctypes.byref(h)), "pget_plan_create")
        self.handle = h
        self.n, self.n_angles, self.n_bins = n, n_angles, n_bins
        self._ws = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.pget_plan_destroy(h)
            self.handle = None

    @property
    def n_samples(self) -> int:
        return int(self.lib.pget_plan_n_samples(self.handle))

    @property
    def psf_half_width(self) -> int:
        return int(self.lib.pget_plan_psf_half_width(self.handle))

    @property
    def support_samples(self) -> int:
        return int(self.lib.pget_plan_support_samples(self.handle))

    def workspace_bytes(self, op: int, batch: int = 1) -> int:
        return int(self.lib.pget_workspace_bytes(self.handle, op, batch))

    def workspace(self, op: int, batch: int = 1):
        torch = _torch()
        key = (op, batch)
        if key not in self._ws:
            nbytes = self.workspace_bytes(op, batch)
            if nbytes == 0:
                raise PgetError(-1, "pget_workspace_bytes")
            self._ws[key] = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self._ws[key]

    # -- operators ----------------------------------------------------------
    def _img(self, t):
        torch = _torch()
        if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != (self.n, self.n):
            raise ValueError("expected a float32 CUDA tensor of shape (%d, %d)" % (self.n, self.n))
        return t.contiguous()

    def _sino(self, t):
        torch = _torch()
        if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != (self.n_angles, self.n_bins):
            raise ValueError("expected a float32 CUDA tensor of shape (%d, %d)"
                             % (self.n_angles, self.n_bins))
        return t.contiguous()

    def forward(self, f, mu):
        torch = _torch()
        f, mu = self._img(f), self._img(mu)
        y = torch.empty((self.n_angles, self.n_bins), dtype=torch.float32, device=f.device)
        ws = self.workspace(OP_FORWARD)
        _check(self.lib.pget_forward(self.handle, _ptr(f), _ptr(mu), _ptr(y), _ptr(ws), _stream()),
               "pget_forward")
        return y

    def forward_noalloc(self, f, mu, y):
        """pget_forward_noalloc into the caller's y (n_angles x n_bins): the
        library allocates nothing for it."""
        f, mu, y = self._img(f), self._img(mu), self._sino(y)
        _check(self.lib.pget_forward_noalloc(self.handle, _ptr(f), _ptr(mu), _ptr(y), _stream()),
               "pget_forward_noalloc")
        return y

    def jvp(self, f, mu, vf, vmu, want_y: bool = False):
        torch = _torch()
        f, mu, vf, vmu = (self._img(t) for t in (f, mu, vf, vmu))
        jv = torch.empty((self.n_angles, self.n_bins), dtype=torch.float32, device=f.device)
        y = torch.empty_like(jv) if want_y else None
        ws = self.workspace(OP_JVP)
        _check(self.lib.pget_jvp(self.handle, _ptr(f), _ptr(mu), _ptr(vf), _ptr(vmu), _ptr(jv),
                                 _ptr(y), _ptr(ws), _stream()), "pget_jvp")
        return (jv, y) if want_y else jv

    def vjp(self, f, mu, w):
        torch = _torch()
        f, mu, w = self._img(f), self._img(mu), self._sino(w)
        gf = torch.empty_like(f)
        gm = torch.empty_like(f)
        ws = self.workspace(OP_VJP)
        _check(self.lib.pget_vjp(self.handle, _ptr(f), _ptr(mu), _ptr(w), _ptr(gf), _ptr(gm),
                                 _ptr(ws), _stream()), "pget_vjp")
        return gf, gm

    # -- solver -------------------------------------------------------------
    def lm_solve(self, y, f0, mu0, params: SolverParams, hook=None, sync: bool = True):
        """Reconstruct one slice.  ``hook(f, mu, s_f, s_mu) -> (f~, mu~)`` takes
        and returns torch tensors (the learned refinement of Alg. 2)."""
        torch = _torch()
        y = self._sino(y)
        f = self._img(f0).clone()
        mu = self._img(mu0).clone()
        prm, keep = params.to_c(self.n)
        rb = _ReportBuffers(params.max_outer, params.n_cg, f.device)
        rc_struct = rb.c()
        ws = self.workspace(OP_LM, 1)
        n = self.n
        cb = REFINE_FN(0)
        if hook is not None:
            def _cb(user, pf, pm, psf, psm, pft, pmt, stream):
                try:
                    tens = [_wrap_device(p, (n, n)) for p in (pf, pm, psf, psm, pft, pmt)]
                    ft, mt = hook(tens[0], tens[1], tens[2], tens[3])
                    tens[4].copy_(ft)
                    tens[5].copy_(mt)
                    return 0
                except Exception:
                    return 1
            cb = REFINE_FN(_cb)
        _check(self.lib.pget_lm_solve(self.handle, _ptr(y), _ptr(f), _ptr(mu), ctypes.byref(prm),
                                      cb, None, ctypes.byref(rc_struct), _ptr(ws), _stream()),
               "pget_lm_solve")
        del keep
        if sync:
            torch.cuda.current_stream().synchronize()
        return f, mu, rb

    def set_depth_factor(self, depth=None):
        """Per-sample depth factor d of the attenuation path (sample 0
        farthest from the detector): exp(-atten_scale * d[i] * B_i).  None
        restores d = 1."""
        if depth is None:
            _check(self.lib.pget_plan_set_depth_factor(self.handle, None, 0), "pget_plan_set_depth_factor")
            return
        arr = (ctypes.c_double * len(depth))(*[float(v) for v in depth])
        _check(self.lib.pget_plan_set_depth_factor(self.handle, arr, len(depth)), "pget_plan_set_depth_factor")

    def set_depth_response(self, alpha=None, far_taps=None):
        """Depth-dependent collimator response: sample i of every ray (sample
        0 farthest from the detector) is seen through (1 - alpha[i]) times the
        plan's Gaussian taps plus alpha[i] times ``far_taps`` (2K + 1
        symmetric values).  None restores the depth-independent response.
        The workspaces grow; the cached ones are dropped."""
        self._ws.clear()
        if alpha is None:
            _check(self.lib.pget_plan_set_depth_response(self.handle, None, 0, None, 0),
                   "pget_plan_set_depth_response")
            return
        a = (ctypes.c_double * len(alpha))(*[float(v) for v in alpha])
        t = (ctypes.c_double * len(far_taps))(*[float(v) for v in far_taps])
        _check(self.lib.pget_plan_set_depth_response(self.handle, a, len(alpha), t, len(far_taps)),
               "pget_plan_set_depth_response")

    def autotune(self, batch: int = 1):
        """Pick the fastest launch shapes for solves of `batch` slices."""
        ws = self.workspace(OP_LM, batch)
        _check(self.lib.pget_autotune(self.handle, batch, _ptr(ws), ws.numel(), _stream()),
               "pget_autotune")
        return self.tuned_shape(batch)

    def set_band_staging(self, enable: bool = True) -> int:
        """Band staging of maps too large for LDS (pget_plan_set_band_staging):
        for plans solved in large batches.  Returns the bands the product
        walks (1: none)."""
        _check(self.lib.pget_plan_set_band_staging(self.handle, int(bool(enable))), "pget_plan_set_band_staging")
        self._ws.clear()
        return int(self.lib.pget_plan_jvp_bands(self.handle))

    def set_shape(self, batch: int = 1, jvp_angle_slots: int = 0, vjp_fine_groups: int = 0):
        """Fix the launch shapes of solves of `batch` slices (0 keeps a default)."""
        _check(self.lib.pget_set_shape(self.handle, batch, jvp_angle_slots, vjp_fine_groups), "pget_set_shape")
        return self.tuned_shape(batch)

    def tuned_shape(self, batch: int = 1):
        ja, vg = ctypes.c_int32(), ctypes.c_int32()
        tuned = self.lib.pget_tuned_shape(self.handle, batch, ctypes.byref(ja), ctypes.byref(vg))
        return {"jvp_angle_slots": ja.value, "vjp_angle_groups": vg.value, "tuned": bool(tuned)}

    def lm_solve_batched(self, ys, f0s, mu0s, params: Sequence[SolverParams], sync: bool = True,
                         ws=None):
        """Solve a batch of slices of this shape.  ``ws`` is an optional
        caller-owned workspace (uint8 CUDA tensor of at least
        ``workspace_bytes(OP_LM, len(ys))`` bytes); concurrent solves on
        different streams need distinct workspaces."""
        torch = _torch()
        B = len(ys)
        if not (len(f0s) == len(mu0s) == len(params) == B):
            raise ValueError("lm_solve_batched: ys, f0s, mu0s and params differ in length")
        if B == 0:   # nothing to solve (the C call requires n_slices >= 1)
            return [], [], []
        ys = [self._sino(t) for t in ys]
        fs = [self._img(t).clone() for t in f0s]
        ms = [self._img(t).clone() for t in mu0s]
        arr = ctypes.c_void_p * B
        cp = (LMParams * B)()
        keeps = []
        for i, p in enumerate(params):
            c, k = p.to_c(self.n)
            cp[i] = c
            keeps.append(k)
        rbs = [_ReportBuffers(params[0].max_outer, params[0].n_cg, fs[0].device) for _ in range(B)]
        reps = (LMReportC * B)(*[r.c() for r in rbs])
        if ws is None:
            ws = self.workspace(OP_LM, B)
        elif ws.numel() < self.workspace_bytes(OP_LM, B):
            raise PgetError(-3, "lm_solve_batched")
        _check(self.lib.pget_lm_solve_batched(
            self.handle, B, arr(*[t.data_ptr() for t in ys]), arr(*[t.data_ptr() for t in fs]),
            arr(*[t.data_ptr() for t in ms]), cp, reps, _ptr(ws), _stream()),
            "pget_lm_solve_batched")
        del keeps
        if sync:
            torch.cuda.current_stream().synchronize()
        return fs, ms, rbs


_multi_ws = {}


def lm_solve_multi(plans: Sequence["Plan"], ys, f0s, mu0s, params: Sequence[SolverParams],
                   sync: bool = True):
    """Slices of mixed shapes: slice s uses plans[s]; slices sharing a plan are
    batched and the groups run concurrently (pget_lm_solve_multi)."""
    torch = _torch()
    lib = load_library()
    n = len(plans)
    arr = ctypes.c_void_p * n
    handles = arr(*[p.handle.value for p in plans])
    ys = [p._sino(t) for p, t in zip(plans, ys)]
    fs = [p._img(t).clone() for p, t in zip(plans, f0s)]
    ms = [p._img(t).clone() for p, t in zip(plans, mu0s)]
    cp = (LMParams * n)()
    keeps = []
    for i, p in enumerate(params):
        c, k = p.to_c(plans[i].n)
        cp[i] = c
        keeps.append(k)
    rbs = [_ReportBuffers(p.max_outer, p.n_cg, fs[0].device) for p in params]
    reps = (LMReportC * n)(*[r.c() for r in rbs])
    nbytes = lib.pget_workspace_bytes_multi(n, handles)
    if nbytes == 0:
        raise PgetError(-1, "pget_workspace_bytes_multi")
    key = tuple(p.handle.value for p in plans)
    ws = _multi_ws.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _multi_ws[key] = ws
    _check(lib.pget_lm_solve_multi(
        n, handles, arr(*[t.data_ptr() for t in ys]), arr(*[t.data_ptr() for t in fs]),
        arr(*[t.data_ptr() for t in ms]), cp, reps, _ptr(ws), ws.numel(), _stream()),
        "pget_lm_solve_multi")
    del keeps
    if sync:
        torch.cuda.current_stream().synchronize()
    return fs, ms, rbs


def _wrap_device(ptr, shape):
    """A torch view of device memory owned by the library (hook arguments)."""
    torch = _torch()
    n = 1
    for s in shape:
        n *= s

    class _Holder:
        pass

    h = _Holder()
    h.__cuda_array_interface__ = {
        "shape": tuple(shape), "typestr": "<f4", "data": (int(ptr), False), "version": 2,
        "strides": None,
    }
    return torch.as_tensor(h, device="cuda")


def set_graphs(enable: bool) -> None:
    """Replay the solver's kernel sequence as a HIP graph (default) or not."""
    _check(load_library().pget_set_graphs(1 if enable else 0), "pget_set_graphs")


def timing_enable(classes: int, capacity: int) -> None:
    """Bracket later launches of the kernel classes in the bit mask with HIP events."""
    _check(load_library().pget_timing_enable(classes, capacity), "pget_timing_enable")


def timing_read(kernel_class: int):
    """(summed device milliseconds, launches) of one kernel class."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load_library().pget_timing_read(kernel_class, ctypes.byref(ms), ctypes.byref(n)),
           "pget_timing_read")
    return ms.value, n.value


# C-ABI names, for callers who prefer them
def pget_forward(plan: Plan, f, mu):
    return plan.forward(f, mu)


def pget_jvp(plan: Plan, f, mu, vf, vmu, want_y: bool = False):
    return plan.jvp(f, mu, vf, vmu, want_y)


def pget_vjp(plan: Plan, f, mu, w):
    return plan.vjp(f, mu, w)


def pget_lm_solve(plan: Plan, y, f0, mu0, params: SolverParams, hook=None):
    return plan.lm_solve(y, f0, mu0, params, hook)


def pget_lm_solve_batched(plan: Plan, ys, f0s, mu0s, params):
    return plan.lm_solve_batched(ys, f0s, mu0s, params)


class LMPool:
    """A slot pool of one plan (pget_lm_pool_*): continuous batching at
    outer-iteration boundaries.  All calls go to the stream current at
    construction (or `stream`).  Argument marshalling only."""

    def __init__(self, plan: "Plan", capacity: int, max_outer: int, n_cg: int, stream=None, step: int = 0):
        torch = _torch()
        self.plan, self.lib = plan, plan.lib
        self.capacity, self.max_outer, self.n_cg = capacity, max_outer, n_cg
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = self.lib.pget_lm_pool_workspace_bytes(plan.handle, capacity, max_outer, n_cg)
        if nbytes == 0:
            raise PgetError(-1, "pget_lm_pool_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.finished = torch.zeros(capacity, dtype=torch.int32).pin_memory()
        self.keep = [None] * capacity      # per slot: inputs, parameters, report buffers
        self.handle = ctypes.c_void_p()
        _check(self.lib.pget_lm_pool_create(plan.handle, capacity, max_outer, n_cg, step, _ptr(self.ws), nbytes,
                                            self.stream.cuda_stream, ctypes.byref(self.handle)),
               "pget_lm_pool_create")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and getattr(self, "lib", None) is not None:
            self.lib.pget_lm_pool_destroy(h)
            self.handle = ctypes.c_void_p()

    def load(self, slot: int, y, f0, mu0, params: SolverParams):
        p = self.plan
        y, f0, mu0 = p._sino(y), p._img(f0), p._img(mu0)
        prm, keep = params.to_c(p.n)
        self.keep[slot] = (y, f0, mu0, prm, keep)
        _check(self.lib.pget_lm_pool_load(self.handle, slot, _ptr(y), _ptr(f0), _ptr(mu0), ctypes.byref(prm),
                                          self.stream.cuda_stream), "pget_lm_pool_load")

    def step(self, timing: bool = False):
        """Enqueue one outer iteration; returns an event recorded after it
        (the `finished` flags are valid once it has completed; with timing,
        the event can measure elapsed time)."""
        torch = _torch()
        _check(self.lib.pget_lm_pool_step(self.handle, ctypes.c_void_p(self.finished.data_ptr()),
                                          self.stream.cuda_stream), "pget_lm_pool_step")
        ev = torch.cuda.Event(enable_timing=timing)
        ev.record(self.stream)
        return ev

    def fetch(self, slot: int, report: bool = True):
        """Maps (and report buffers) of a slot, which becomes free."""
        torch = _torch()
        n = self.plan.n
        f = torch.empty((n, n), dtype=torch.float32, device="cuda")
        mu = torch.empty_like(f)
        held = self.keep[slot] if 0 <= slot < self.capacity else None
        mo = held[3].max_outer if held is not None else self.max_outer
        rb = _ReportBuffers(mo, self.n_cg, "cuda") if report else None
        rc = rb.c() if rb is not None else None
        _check(self.lib.pget_lm_pool_fetch(self.handle, slot, _ptr(f), _ptr(mu),
                                           ctypes.byref(rc) if rc is not None else None, self.stream.cuda_stream),
               "pget_lm_pool_fetch")
        if 0 <= slot < self.capacity:
            self.keep[slot] = None
        return f, mu, rb
