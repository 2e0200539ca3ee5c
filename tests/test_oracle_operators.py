"""Pins of the FP64 oracle's operators to facts outside the oracle itself.

Each test names what fixes the expected value: a closed form, an invariant,
an independent brute-force formulation, or automatic differentiation.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle.dense import DenseModel


def raster_disk(n, R, cx=0.0, cy=0.0, sub=8):
    off = (np.arange(sub) + 0.5) / sub - 0.5
    cc = np.arange(n) - 0.5 * (n - 1)
    xs = (cc[:, None] + off[None, :]).reshape(-1)
    X, Y = np.meshgrid(xs, xs)
    inside = ((X - cx) ** 2 + (Y - cy) ** 2) <= R * R
    return inside.astype(float).reshape(n, sub, n, sub).mean(axis=(1, 3))


def smooth_bump(n, R):
    cc = np.arange(n) - 0.5 * (n - 1)
    X, Y = np.meshgrid(cc, cc)
    r2 = (X ** 2 + Y ** 2) / R ** 2
    return np.where(r2 < 1.0, (1.0 - r2) ** 2, 0.0)


def bins(g):
    return (np.arange(g.n_bins) - 0.5 * (g.n_bins - 1)) * g.bin_size


# ---------------------------------------------------------------- collimator
def test_psf_taps_normalised_symmetric():
    g = O.Geometry(16, 4, 40, psf_sigma=1.5)
    k = O.psf_taps(g)
    assert g.psf_half_width == 5          # ceil(3 * 1.5)
    assert k.shape == (11,)
    assert abs(k.sum() - 1.0) < 1e-15
    assert np.array_equal(k, k[::-1])
    # Gaussian shape: ratio of neighbouring taps is exp(-(2k+1)/(2 sigma^2))
    assert abs(k[6] / k[5] - math.exp(-1.0 / (2 * 1.5 ** 2))) < 1e-14


def test_psf_impulse_response_and_transpose():
    g = O.Geometry(16, 3, 40, psf_sigma=1.5)
    p = np.zeros(g.sino_shape)
    p[1, 20] = 1.0
    y = O.psf(g, p)
    assert np.allclose(y[1, 15:26], O.psf_taps(g), rtol=0, atol=1e-16)
    assert np.all(y[0] == 0) and np.all(y[2] == 0)
    # adjoint identity of the blur, including the truncated border
    rng = np.random.default_rng(1)
    a = rng.standard_normal(g.sino_shape)
    b = rng.standard_normal(g.sino_shape)
    lhs = np.sum(O.psf(g, a) * b)
    rhs = np.sum(a * O.psf_transpose(g, b))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_psf_sigma_zero_is_identity():
    g = O.Geometry(16, 3, 20, psf_sigma=0.0)
    p = np.random.default_rng(2).standard_normal(g.sino_shape)
    assert np.array_equal(O.psf(g, p), p)


# ------------------------------------------------------- closed-form transforms
def test_radon_of_smooth_bump_second_order():
    """mu = 0, no blur: the Radon transform of (1 - |x|^2/R^2)^2 is
    (16 R / 15) (1 - s^2/R^2)^(5/2); midpoint sampling of a bilinear
    interpolant converges at second order."""
    errs = []
    for n in (32, 64):
        g = O.Geometry(n, 12, int(1.5 * n), psf_sigma=0.0)
        R = 0.4 * n
        y = O.forward(g, smooth_bump(n, R), np.zeros((n, n)))
        s = bins(g)
        ex = np.where(np.abs(s) < R, (16 * R / 15) * np.clip(1 - s ** 2 / R ** 2, 0, None) ** 2.5, 0.0)
        errs.append(np.linalg.norm(y - ex[None, :]) / (np.linalg.norm(ex) * math.sqrt(g.n_angles)))
    assert errs[1] < 1e-3
    rate = math.log2(errs[0] / errs[1])
    assert 1.8 < rate < 2.2


def test_constant_attenuation_disks():
    """f = 1 on a disk R_e, mu = mu0 on a concentric disk R_a:
    y(s) = (2/mu0) exp(-mu0 L_a) sinh(mu0 L_e), L = sqrt(R^2 - s^2).
    First-order convergence (sharp disk edges).  Getting the self-attenuation
    of a sample wrong by half a step biases every ray by ~exp(-mu0/2), i.e.
    ~5 % at mu0 = 0.1, far outside the tolerance."""
    mu0 = 0.1
    errs = []
    for n in (64, 128):
        g = O.Geometry(n, 12, int(1.5 * n), psf_sigma=0.0)
        Re, Ra = 0.25 * n, 0.4 * n
        y = O.forward(g, raster_disk(n, Re), mu0 * raster_disk(n, Ra))
        s = bins(g)
        Le = np.sqrt(np.clip(Re ** 2 - s ** 2, 0, None))
        La = np.sqrt(np.clip(Ra ** 2 - s ** 2, 0, None))
        ex = (2.0 / mu0) * np.exp(-mu0 * La) * np.sinh(mu0 * Le)
        errs.append(np.linalg.norm(y - ex[None, :]) / (np.linalg.norm(ex) * math.sqrt(g.n_angles)))
    assert errs[1] < 0.01
    assert errs[0] / errs[1] > 1.6


def test_small_attenuation_limit_is_radon():
    n = 48
    g = O.Geometry(n, 8, 72, psf_sigma=0.0)
    f = smooth_bump(n, 0.4 * n)
    y0 = O.forward(g, f, np.zeros((n, n)))
    y1 = O.forward(g, f, 1e-9 * raster_disk(n, 0.45 * n))
    assert np.abs(y1 - y0).max() <= 1e-7 * np.abs(y0).max()


def test_point_source_orientation_and_detector_side():
    """A single emitting pixel at p inside an attenuating disk: the peak bin
    of angle a is the bin nearest <p, omega_perp>, and the detected mass is
    ~exp(-mu0 d_a), d_a the distance from p to the disk edge in the +omega
    (detector) direction.  Attenuating toward -omega instead would give
    exp(-mu0 d'_a), d'_a = sqrt(R^2 - s^2) + <p, omega>."""
    n, na, nb = 64, 24, 96
    g = O.Geometry(n, na, nb, psf_sigma=0.0)
    r, c = 40, 15
    px, py = c - 0.5 * (n - 1), r - 0.5 * (n - 1)
    f = np.zeros((n, n))
    f[r, c] = 1.0
    mu0, Ra = 0.05, 28.0
    y = O.forward(g, f, mu0 * raster_disk(n, Ra))
    th = np.arange(na) * 2 * np.pi / na
    sp = -px * np.sin(th) + py * np.cos(th)
    tp = px * np.cos(th) + py * np.sin(th)
    pos = sp / g.bin_size + 0.5 * (nb - 1)
    clear = np.abs(pos - np.floor(pos) - 0.5) > 0.1
    assert np.array_equal(np.argmax(y, axis=1)[clear], np.round(pos).astype(int)[clear])
    mass = y.sum(axis=1) * g.bin_size
    d = np.sqrt(Ra ** 2 - sp ** 2) - tp
    ratio = mass / np.exp(-mu0 * d)
    assert np.all(np.abs(ratio - 1.0) < 0.12)
    d_wrong = np.sqrt(Ra ** 2 - sp ** 2) + tp
    wrong = mass / np.exp(-mu0 * d_wrong)
    far = np.abs(tp) > 10
    assert np.all(np.abs(wrong[far] - 1.0) > 0.3)


# ---------------------------------------------------------------- symmetries
def test_rotation_by_quarter_turn_shifts_angles():
    """Rotating both maps by +90 degrees, new[r][c] = old[N-1-c][r], gives
    y_new[a] = y_old[a - n_a/4] when n_a is a multiple of 4 over a full turn."""
    n, na = 20, 16
    g = O.Geometry(n, na, 30, psf_sigma=1.5)
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.1, (n, n))
    rot = lambda m: np.array([[m[n - 1 - cc, rr] for cc in range(n)] for rr in range(n)])
    y = O.forward(g, f, mu)
    yr = O.forward(g, rot(f), rot(mu))
    assert np.abs(yr - np.roll(y, na // 4, axis=0)).max() <= 1e-12 * np.abs(y).max()


def test_opposite_angles_mirror_without_attenuation():
    n, na = 20, 16
    g = O.Geometry(n, na, 31, psf_sigma=1.5)
    f = np.random.default_rng(4).uniform(0, 1, (n, n))
    y = O.forward(g, f, np.zeros((n, n)))
    assert np.abs(y[na // 2:] - y[: na // 2, ::-1]).max() <= 1e-12 * np.abs(y).max()


def test_linear_in_emission():
    n = 16
    g = O.Geometry(n, 10, 24)
    rng = np.random.default_rng(5)
    f1, f2 = rng.uniform(0, 1, (2, n, n))
    mu = rng.uniform(0, 0.2, (n, n))
    lhs = O.forward(g, 2.0 * f1 - 3.0 * f2, mu)
    rhs = 2.0 * O.forward(g, f1, mu) - 3.0 * O.forward(g, f2, mu)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()


# -------------------------------------------- brute force and differentiation
@pytest.mark.parametrize("n,na,nb,sigma", [(8, 8, 12, 1.5), (7, 5, 11, 0.0), (9, 6, 10, 1.0)])
def test_matches_dense_brute_force(n, na, nb, sigma):
    """The dense formulation sums tent weights over every pixel and forms the
    beam sums with a triangular matrix; the oracle must agree to rounding."""
    g = O.Geometry(n, na, nb, psf_sigma=sigma)
    D = DenseModel(n, na, nb, psf_sigma=sigma)
    assert D.n_t == g.n_samples
    rng = np.random.default_rng(6)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.3, (n, n))
    y = O.forward(g, f, mu)
    assert np.abs(y - D.forward(f, mu)).max() <= 1e-13 * np.abs(y).max()


def test_jvp_vjp_match_torch_autograd_of_dense_model():
    torch = pytest.importorskip("torch")
    n, na, nb = 8, 8, 12
    g = O.Geometry(n, na, nb, psf_sigma=1.5)
    D = DenseModel(n, na, nb, psf_sigma=1.5)
    rng = np.random.default_rng(7)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.3, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    fn = lambda a, b: D.forward(a, b, xp=torch)
    T = lambda a: torch.tensor(a, dtype=torch.float64)
    _, jt = torch.func.jvp(fn, (T(f), T(mu)), (T(vf), T(vm)))
    jv = O.jvp(g, f, mu, vf, vm)
    assert np.abs(jt.numpy() - jv).max() <= 1e-13 * np.abs(jv).max()
    _, back = torch.func.vjp(fn, T(f), T(mu))
    tf, tm = back(T(w))
    gf, gm = O.vjp(g, f, mu, w)
    assert np.abs(tf.numpy() - gf).max() <= 1e-13 * np.abs(gf).max()
    assert np.abs(tm.numpy() - gm).max() <= 1e-13 * np.abs(gm).max()


def test_jvp_central_differences():
    n = 16
    g = O.Geometry(n, 12, 24)
    rng = np.random.default_rng(8)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.15, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    h = 1e-5 * math.sqrt(np.sum(f ** 2) + np.sum(mu ** 2)) / math.sqrt(np.sum(vf ** 2) + np.sum(vm ** 2))
    fd = (O.forward(g, f + h * vf, mu + h * vm) - O.forward(g, f - h * vf, mu - h * vm)) / (2 * h)
    jv = O.jvp(g, f, mu, vf, vm)
    assert np.linalg.norm(fd - jv) <= 1e-8 * np.linalg.norm(jv)
    # the emission part is exact: F is linear in f
    fd_f = (O.forward(g, f + vf, mu) - O.forward(g, f - vf, mu)) / 2.0
    jv_f = O.jvp(g, f, mu, vf, np.zeros((n, n)))
    assert np.abs(fd_f - jv_f).max() <= 1e-12 * np.abs(jv_f).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_identity(seed):
    n = 16
    g = O.Geometry(n, 14, 23, psf_sigma=1.5)
    rng = np.random.default_rng(9 + seed)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.15, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal(g.sino_shape)
    lhs = np.sum(O.jvp(g, f, mu, vf, vm) * w)
    gf, gm = O.vjp(g, f, mu, w)
    rhs = np.sum(vf * gf) + np.sum(vm * gm)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-300)


# --------------------------------------------------------------- regulariser
def test_regulariser_gradient_and_nullspace():
    n = 12
    rng = np.random.default_rng(11)
    x = rng.standard_normal((n, n))
    alpha = 0.37
    # the gradient of a quadratic is exact under central differences
    v = rng.standard_normal((n, n))
    fd = (O.reg_energy(alpha, x + v) - O.reg_energy(alpha, x - v)) / 2.0
    assert abs(fd - np.sum(O.reg_gradient(alpha, x) * v)) <= 1e-12 * abs(fd)
    # constants are free (Neumann boundary) and a ramp costs alpha/2 per edge
    assert np.abs(O.reg_gradient(alpha, np.full((n, n), 3.0))).max() == 0.0
    ramp = np.tile(np.arange(n, dtype=float), (n, 1))
    assert abs(O.reg_energy(alpha, ramp) - 0.5 * alpha * n * (n - 1)) < 1e-12


# ------------------------------------------------- depth factor of the path
def _depth(n_t, seed):
    """A smooth depth factor >= 1, largest far from the detector (sample 0)."""
    rng = np.random.default_rng(seed)
    t = np.linspace(1.0, 0.0, n_t)
    return tuple(1.0 + 0.8 * t + 0.05 * rng.uniform(size=n_t))


def test_depth_factor_matches_dense_and_autograd():
    """With a per-sample factor d_i on the attenuation path (c_i = c d_i),
    the oracle agrees with the dense formulation and its Jacobian products
    with torch autograd of that formulation (where c_i enters the
    exponential of every sample separately)."""
    torch = pytest.importorskip("torch")
    n, na, nb = 8, 8, 12
    n_t = O.Geometry(n, na, nb).n_samples
    d = _depth(n_t, 0)
    g = O.Geometry(n, na, nb, psf_sigma=1.5, atten_scale=0.7, depth=d)
    D = DenseModel(n, na, nb, psf_sigma=1.5, atten_scale=0.7, depth=d)
    rng = np.random.default_rng(17)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.3, (n, n))
    y = O.forward(g, f, mu)
    assert np.abs(y - D.forward(f, mu)).max() <= 1e-13 * np.abs(y).max()
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    fn = lambda a, b: D.forward(a, b, xp=torch)
    T = lambda a: torch.tensor(a, dtype=torch.float64)
    _, jt = torch.func.jvp(fn, (T(f), T(mu)), (T(vf), T(vm)))
    jv = O.jvp(g, f, mu, vf, vm)
    assert np.abs(jt.numpy() - jv).max() <= 1e-13 * np.abs(jv).max()
    _, back = torch.func.vjp(fn, T(f), T(mu))
    tf, tm = back(T(w))
    gf, gm = O.vjp(g, f, mu, w)
    assert np.abs(tf.numpy() - gf).max() <= 1e-13 * np.abs(gf).max()
    assert np.abs(tm.numpy() - gm).max() <= 1e-13 * np.abs(gm).max()
    # the factor matters: without it the attenuation part differs
    g0 = O.Geometry(n, na, nb, psf_sigma=1.5, atten_scale=0.7)
    assert np.abs(O.forward(g0, f, mu) - y).max() > 1e-3 * np.abs(y).max()


def test_uniform_depth_is_a_scaled_attenuation():
    """d_i = 2 everywhere is the constant factor c = 2 exactly."""
    n, na, nb = 12, 10, 18
    n_t = O.Geometry(n, na, nb).n_samples
    g2 = O.Geometry(n, na, nb, atten_scale=2.0)
    gd = O.Geometry(n, na, nb, depth=(2.0,) * n_t)
    rng = np.random.default_rng(18)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.2, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    assert np.array_equal(O.forward(g2, f, mu), O.forward(gd, f, mu))
    assert np.array_equal(O.jvp(g2, f, mu, vf, vm), O.jvp(gd, f, mu, vf, vm))
    for a, b in zip(O.vjp(g2, f, mu, w), O.vjp(gd, f, mu, w)):
        assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        O.Geometry(n, na, nb, depth=(1.0,) * (n_t - 1)).n_samples


def test_depth_adjoint_identity():
    n = 16
    n_t = O.Geometry(n, 14, 23).n_samples
    g = O.Geometry(n, 14, 23, psf_sigma=1.5, depth=_depth(n_t, 1))
    rng = np.random.default_rng(19)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.15, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal(g.sino_shape)
    lhs = np.sum(O.jvp(g, f, mu, vf, vm) * w)
    gf, gm = O.vjp(g, f, mu, w)
    assert abs(lhs - (np.sum(vf * gf) + np.sum(vm * gm))) <= 1e-12 * abs(lhs)


# ------------------------------------- depth-dependent collimator response
def _gauss_taps(sigma, K):
    k = np.arange(-K, K + 1)
    t = np.exp(-(k ** 2) / (2.0 * sigma ** 2))
    return tuple(t / t.sum())


def _alpha(n_t, seed=None):
    """Weight of the far response: 1 at sample 0 (farthest from the
    detector), 0 at the last sample, linear in between; optionally jittered."""
    a = 1.0 - np.arange(n_t) / (n_t - 1)
    if seed is not None:
        a = np.clip(a + 0.1 * np.random.default_rng(seed).uniform(-1, 1, n_t), 0.0, 1.0)
    return tuple(a)


def test_depth_response_matches_dense_and_autograd():
    """The oracle spreads every sample with its own response; the dense
    formulation splits each ray sum into the parts seen through the near
    and the far response.  They agree, and the oracle's Jacobian products
    agree with torch autograd of the dense formulation, with and without a
    depth factor on the attenuation path."""
    torch = pytest.importorskip("torch")
    n, na, nb = 8, 8, 14
    n_t = O.Geometry(n, na, nb).n_samples
    K = O.Geometry(n, na, nb, psf_sigma=1.5).psf_half_width
    far = _gauss_taps(2.5, K)
    al = _alpha(n_t, seed=3)
    rng = np.random.default_rng(31)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.3, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    T = lambda a: torch.tensor(a, dtype=torch.float64)
    for depth in (None, _depth(n_t, 2)):
        g = O.Geometry(n, na, nb, psf_sigma=1.5, atten_scale=0.7, depth=depth, resp=al, far_taps=far)
        D = DenseModel(n, na, nb, psf_sigma=1.5, atten_scale=0.7, depth=depth, resp=al, far_taps=far)
        y = O.forward(g, f, mu)
        assert np.abs(y - D.forward(f, mu)).max() <= 1e-13 * np.abs(y).max()
        fn = lambda a, b: D.forward(a, b, xp=torch)
        _, jt = torch.func.jvp(fn, (T(f), T(mu)), (T(vf), T(vm)))
        jv = O.jvp(g, f, mu, vf, vm)
        assert np.abs(jt.numpy() - jv).max() <= 1e-13 * np.abs(jv).max()
        _, back = torch.func.vjp(fn, T(f), T(mu))
        tf, tm = back(T(w))
        gf, gm = O.vjp(g, f, mu, w)
        assert np.abs(tf.numpy() - gf).max() <= 1e-13 * np.abs(gf).max()
        assert np.abs(tm.numpy() - gm).max() <= 1e-13 * np.abs(gm).max()
        # the response matters
        g0 = O.Geometry(n, na, nb, psf_sigma=1.5, atten_scale=0.7, depth=depth)
        assert np.abs(O.forward(g0, f, mu) - y).max() > 1e-3 * np.abs(y).max()


def test_depth_response_reduces_to_one_gaussian():
    """alpha = 0 everywhere is the plain model; alpha = 1 everywhere is the
    plain model whose Gaussian is the far one (same truncation)."""
    n, na, nb = 12, 10, 20
    g = O.Geometry(n, na, nb, psf_sigma=1.2)
    n_t, K = g.n_samples, g.psf_half_width
    far = _gauss_taps(2.0, K)
    g_near = O.Geometry(n, na, nb, psf_sigma=1.2, resp=(0.0,) * n_t, far_taps=far)
    g_far = O.Geometry(n, na, nb, psf_sigma=1.2, resp=(1.0,) * n_t, far_taps=far)
    g_ref = O.Geometry(n, na, nb, psf_sigma=2.0, psf_radius=K)
    rng = np.random.default_rng(32)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.2, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    for a, b in ((g_near, g), (g_far, g_ref)):
        y = O.forward(b, f, mu)
        assert np.abs(O.forward(a, f, mu) - y).max() <= 1e-13 * np.abs(y).max()
        jv = O.jvp(b, f, mu, vf, vm)
        assert np.abs(O.jvp(a, f, mu, vf, vm) - jv).max() <= 1e-13 * np.abs(jv).max()
        for p, q in zip(O.vjp(a, f, mu, w), O.vjp(b, f, mu, w)):
            assert np.abs(p - q).max() <= 1e-13 * np.abs(q).max()


def test_depth_response_is_affine_in_alpha():
    """Every output is affine in the per-sample weights: the midpoint of two
    weight profiles gives the mean of their outputs."""
    n, na, nb = 10, 9, 16
    g = O.Geometry(n, na, nb, psf_sigma=1.5)
    n_t, K = g.n_samples, g.psf_half_width
    far = _gauss_taps(3.0, K)
    a1, a2 = np.array(_alpha(n_t, seed=4)), np.random.default_rng(5).uniform(0, 1, n_t)
    gs = [O.Geometry(n, na, nb, psf_sigma=1.5, resp=tuple(a), far_taps=far) for a in (a1, a2, 0.5 * (a1 + a2))]
    rng = np.random.default_rng(33)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.2, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal((na, nb))
    y = [O.forward(x, f, mu) for x in gs]
    assert np.abs(y[2] - 0.5 * (y[0] + y[1])).max() <= 1e-13 * np.abs(y[2]).max()
    j = [O.jvp(x, f, mu, vf, vm) for x in gs]
    assert np.abs(j[2] - 0.5 * (j[0] + j[1])).max() <= 1e-13 * np.abs(j[2]).max()
    v = [O.vjp(x, f, mu, w) for x in gs]
    for c in range(2):
        assert np.abs(v[2][c] - 0.5 * (v[0][c] + v[1][c])).max() <= 1e-13 * np.abs(v[2][c]).max()


def test_depth_response_point_emitter_width():
    """A single emitting pixel at angle 0 without attenuation: pixel centres
    fall on lattice points, so exactly one sample sees it, and its profile
    across bins is that sample's response.  The profile keeps unit mass, and
    its variance is (1 - alpha) Var(kappa) + alpha Var(kappa_far) with alpha
    of the pixel's own depth: wider for the emitter far from the detector
    (the detector lies toward +x at angle 0)."""
    n, nb = 16, 24
    g = O.Geometry(n, 4, nb, psf_sigma=1.0)
    n_t, K = g.n_samples, g.psf_half_width
    far = _gauss_taps(2.5, K)
    al = _alpha(n_t)
    gr = O.Geometry(n, 4, nb, psf_sigma=1.0, resp=al, far_taps=far)
    k = np.arange(-K, K + 1)
    var_near = float(np.sum(k ** 2 * np.array(O.psf_taps(g))))
    var_far = float(np.sum(k ** 2 * np.array(far)))
    widths = []
    for c in (2, 13):                       # far from / near to the detector
        f = np.zeros((n, n))
        r = 8
        f[r, c] = 1.0
        y = O.forward(gr, f, np.zeros((n, n)))[0]
        j0 = r - (n - 1) / 2 + (nb - 1) / 2     # bin whose centre is the pixel's row
        i0 = int(c - (n - 1) / 2 + (n_t - 1) / 2)   # sample whose point is the pixel
        a = al[i0]
        var = float(np.sum((np.arange(nb) - j0) ** 2 * y))
        assert abs(y.sum() - 1.0) <= 1e-13
        assert abs(var - ((1 - a) * var_near + a * var_far)) <= 1e-12
        widths.append((a, var))
    (a_far, w_far), (a_near, w_near) = widths
    assert a_far > a_near and w_far - w_near > 0.9 * (a_far - a_near) * (var_far - var_near)


def test_depth_response_adjoint_identity_and_arguments():
    n = 16
    g0 = O.Geometry(n, 14, 23, psf_sigma=1.5)
    n_t, K = g0.n_samples, g0.psf_half_width
    g = O.Geometry(n, 14, 23, psf_sigma=1.5, depth=_depth(n_t, 1), resp=_alpha(n_t, seed=6),
                   far_taps=_gauss_taps(2.8, K))
    rng = np.random.default_rng(34)
    f = rng.uniform(0, 1, (n, n))
    mu = rng.uniform(0, 0.15, (n, n))
    vf, vm = rng.standard_normal((2, n, n))
    w = rng.standard_normal(g.sino_shape)
    lhs = np.sum(O.jvp(g, f, mu, vf, vm) * w)
    gf, gm = O.vjp(g, f, mu, w)
    assert abs(lhs - (np.sum(vf * gf) + np.sum(vm * gm))) <= 1e-12 * abs(lhs)
    with pytest.raises(ValueError):
        O.Geometry(n, 14, 23, resp=(0.5,) * n_t).n_samples
    with pytest.raises(ValueError):
        O.Geometry(n, 14, 23, resp=(0.5,) * (n_t - 1), far_taps=_gauss_taps(2.0, K)).n_samples
    with pytest.raises(ValueError):
        O.Geometry(n, 14, 23, resp=(0.5,) * n_t, far_taps=_gauss_taps(2.0, K + 1)).n_samples
