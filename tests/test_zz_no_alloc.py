"""The allocation-free forward map (pget_forward_noalloc) called through the
C ABI gives the bits of pget_forward with a workspace, on consecutive calls
whose bordered map copies live in the library's static scratch (a 256^2
map, then a smaller 150^2 one; both too large for LDS), and on a map staged
in LDS (64^2, no scratch)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2604_26745_amd import inputs, pget  # noqa: E402


def test_forward_noalloc_equals_forward():
    for n, na, nb, seed in ((256, 90, 256, 0), (150, 60, 160, 1), (64, 120, 96, 2)):
        print("noalloc forward: %d^2, %d x %d" % (n, na, nb), flush=True)
        sys.stdout.flush()
        plan = pget.Plan(n, na, nb)
        f = torch.tensor(inputs.random_like((n, n), seed, kind="uniform"), dtype=torch.float32, device="cuda")
        mu = 0.02 * torch.tensor(inputs.random_like((n, n), seed + 10, kind="uniform"), dtype=torch.float32,
                                 device="cuda")
        y_ref = plan.forward(f, mu)
        y = torch.full((na, nb), float("nan"), dtype=torch.float32, device="cuda")
        plan.forward_noalloc(f, mu, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), n
        assert float(y_ref.abs().max()) > 0.0
