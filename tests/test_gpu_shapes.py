"""Default launch shapes of the Jacobian product (angle slots per block).

When a plan reads the map pair whole (staged in LDS, or from the bordered
HBM copy with band staging off), the default takes the fewest angle slots
per block that minimise ceil(blocks / CUs) x (slots per block + c0), with
c0 = 2 (LDS) or 0.5 (HBM copy).  The expected picks below are the ones
measured fastest on one MI355X (256 CUs) per LM solve of 15 x 30; plans
with band staging on keep the rule that fills the chip twice.  Shapes change
no result bit (tests/test_gpu_invariance.py); these tests pin the choice.
Most slots per block: 8 for a 128^2 map in LDS (the rows of the block's
slots share LDS with the staged map), 16 otherwise here.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2604_26745_amd import pget  # noqa: E402


def expected(slots, batch, max_slots, c0, cus):
    best, pick = None, 1
    for j in range(1, max_slots + 1):
        blocks = batch * -(-slots // j)
        cost = -(-blocks // cus) * (j + c0)
        if best is None or cost < best * (1 - 1e-9):
            best, pick = cost, j
    return pick


@pytest.fixture(scope="module")
def cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


# (grid, angles, bins, batch, measured pick on 256 CUs)
LDS_CASES = [(128, 360, 192, 1, 1), (128, 360, 192, 4, 3), (128, 360, 192, 8, 6), (128, 360, 192, 13, 5),
             (128, 360, 192, 64, 8), (64, 360, 96, 12, 9), (96, 360, 144, 13, 10), (64, 120, 96, 64, 15)]
HBM_CASES = [(192, 360, 288, 4, 3), (192, 360, 288, 11, 8), (256, 360, 384, 15, 11), (256, 360, 384, 64, 15)]


@pytest.mark.parametrize("n,na,nb,batch,pick", LDS_CASES, ids=["%dx%d_b%d" % (c[0], c[1], c[3]) for c in LDS_CASES])
def test_product_slots_map_in_lds(cus, n, na, nb, batch, pick):
    plan = pget.Plan(n, na, nb)
    got = plan.tuned_shape(batch)
    assert not got["tuned"]
    max_slots = 8 if n == 128 else 16
    assert got["jvp_angle_slots"] == expected(na // 2, batch, max_slots, 2.0, cus)
    if cus == 256:
        assert got["jvp_angle_slots"] == pick


@pytest.mark.parametrize("n,na,nb,batch,pick", HBM_CASES, ids=["%dx%d_b%d" % (c[0], c[1], c[3]) for c in HBM_CASES])
def test_product_slots_map_in_hbm(cus, n, na, nb, batch, pick):
    plan = pget.Plan(n, na, nb)
    assert plan.set_band_staging(False) == 1
    got = plan.tuned_shape(batch)
    assert got["jvp_angle_slots"] == expected(na // 2, batch, 16, 0.5, cus)
    if cus == 256:
        assert got["jvp_angle_slots"] == pick



def test_widest_blocks_keep_every_bit():
    """The 64^2 x 120-angle plan at 15 angle slots per block (the default for
    64 slices) gives the same bits as one slot per block: a Jacobian product
    and a short solve."""
    import numpy as np
    from paper_2604_26745_amd import inputs
    n, na, nb = 64, 120, 96
    plan = pget.Plan(n, na, nb)
    cfg = inputs.SMALL_64
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")
    f_true, mu_true = inputs.rod_lattice(cfg, 1)
    y = T(inputs.poisson_counts(plan.forward(T(f_true), T(mu_true)).double().cpu().numpy(), 1e4, 1))
    f0 = torch.full((n, n), float(f_true.mean()), device="cuda")
    m0 = torch.zeros((n, n), device="cuda")
    rng = np.random.default_rng(4)
    vf, vm = T(rng.standard_normal((n, n))), T(0.05 * rng.standard_normal((n, n)))
    prm = pget.SolverParams(max_outer=3, n_cg=8, w_mu=0.05 ** 2, d_mu=1 / 0.05 ** 2, active_set=1)
    runs = []
    for slots in (1, 15):
        assert plan.set_shape(1, jvp_angle_slots=slots)["jvp_angle_slots"] == slots
        jv = plan.jvp(f0, T(0.02 * f_true), vf, vm)
        runs.append((jv, plan.lm_solve(y, f0, m0, prm)))
    (jv1, (f1, m1, _)), (jv2, (f2, m2, _)) = runs
    assert torch.equal(jv1, jv2)
    assert torch.equal(f1, f2) and torch.equal(m1, m2)
