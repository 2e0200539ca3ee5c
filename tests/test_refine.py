"""The learned refinement network and its training pieces, on the CPU: the
parameter count of the reading (3x3 kernels, 5x5 L), the output's
non-negativity and masking, the augmentation rotation (exact at 0 degrees,
a quarter turn equals numpy's rot90 up to the interpolation of the corners
outside the inscribed disk), and that one training stage lowers its loss.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2604_26745_amd import refine  # noqa: E402


def test_parameter_count():
    m = refine.build_cnn()
    # encoders 2 x (152 + 1168 + 4640), decoder 9248 + 4624 + 1160 + 146, L 2*2*25
    assert refine.n_params(m) == 2 * (152 + 1168 + 4640) + 9248 + 4624 + 1160 + 146 + 100 == 27198


def test_output_nonnegative_and_masked():
    torch.manual_seed(0)
    n = 24
    cc = np.arange(n) - 0.5 * (n - 1)
    X, Y = np.meshgrid(cc, cc)
    mask = (X ** 2 + Y ** 2 <= (0.5 * n) ** 2).astype(np.float64)
    m = refine.build_cnn(mask=mask)
    u = torch.rand(3, 2, n, n)
    s = torch.randn(3, 2, n, n)
    with torch.no_grad():
        out = m(u, s)
    assert out.shape == (3, 2, n, n)
    assert float(out.min()) >= 0.0
    assert float(out[:, :, mask == 0].abs().max()) == 0.0


def test_rotation():
    torch.manual_seed(1)
    x = torch.rand(2, 2, 20, 20, dtype=torch.float64)
    assert torch.allclose(refine.rotate(x, [0.0, 0.0]), x, atol=1e-12)
    r = refine.rotate(x, [90.0, 90.0]).numpy()
    cc = np.arange(20) - 9.5
    X, Y = np.meshgrid(cc, cc)
    disk = X ** 2 + Y ** 2 <= 8.0 ** 2
    # one of the two quarter turns, whichever orientation the grid convention gives
    ok = [np.abs((r - np.rot90(x.numpy(), k, axes=(2, 3)))[:, :, disk]).max() < 1e-9 for k in (1, 3)]
    assert any(ok)


def test_training_stage_lowers_loss():
    torch.manual_seed(2)
    n = 16
    Ut = torch.rand(8, 2, n, n)
    U = 0.5 * Ut
    S = 0.3 * Ut
    m = refine.build_cnn()
    with torch.no_grad():
        before = float(torch.mean((m(U, S) - Ut) ** 2))
    refine.train_stage(m, U, S, Ut, epochs=30, batch=4, lr=5e-3, max_rot=0.0)
    with torch.no_grad():
        after = float(torch.mean((m(U, S) - Ut) ** 2))
    assert after < 0.5 * before
