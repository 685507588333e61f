"""The collision-time calibrated contact coefficients (the paper's sand
parameters e_n = 0.97, e_t = 0.39, mu_c = 0.15, T_c = 10 dt_f) in the step,
through the C ABI, against the oracle: full steps of the 50-sphere and
512-sphere beds (FP64 1e-11, FP32 1e-5) and a head-on collision followed
substep by substep."""
import numpy as np
import pytest

from helpers import fields_for, oracle_params, prs_params, rel_err
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}
TINY = W.small("tiny", 40, 10, (4.0, 6.0, 4.0), seed=11, bed_u_std=0.1)
SAND = dict(contact_model=1, t_c=10 * W.PHYS["dt_f"], e_n=0.97, e_t=0.39, mu=0.15)


@pytest.fixture(scope="module")
def P():
    import torch

    import paper_2108_01814_amd as P

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle

    oracle.lib()
    return oracle


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("w", [TINY, W.C1], ids=["tiny", "c1"])
def test_step_with_calibrated_contacts(P, orc, precision, w):
    import torch

    bed = W.make_bed(w)
    dt = torch.float64 if precision == 1 else torch.float32
    g = [a.to(device="cuda", dtype=dt).contiguous() for a in fields_for(w, bed)]
    x, u, om = dev(bed.x), dev(bed.u), dev(bed.om)
    with P.Context(prs_params(P, w, precision, **SAND)) as ctx:
        H = P.History.zeros(w.n)
        f = [torch.zeros_like(a) for a in g]
        for _ in range(2):
            Fh, Th, st = ctx.step(g, f, x, u, om, H, zero_f=True)
        got = dict(x=x.cpu().numpy(), u=u.cpu().numpy(), om=om.cpu().numpy(),
                   partner=H.partner.cpu().numpy(), dt=H.delta_t.cpu().numpy())
    uh = [np.ascontiguousarray(a.double().cpu().numpy()) for a in g]
    p = oracle_params(orc, w, **SAND)
    xo, uo, oo = bed.x.copy(), bed.u.copy(), bed.om.copy()
    Ho = orc.History(w.n)
    for _ in range(2):
        fo = [np.zeros_like(a) for a in uh]
        rc, out = orc.step(p, uh, fo, xo, uo, oo, Ho)
        assert rc == 0
    tol = TOL[precision]
    assert np.array_equal(got["partner"], Ho.partner)
    assert np.abs(got["x"] - xo).max() < tol
    assert rel_err(got["u"], uo) < tol
    assert rel_err(got["om"], oo) < tol
    assert rel_err(got["dt"], Ho.dt) < max(tol, 1e-10)


def test_head_on_collision_substeps(P, orc):
    """Two spheres approaching at unit speed, one substep per call (no fluid
    force), followed through the contact: device and oracle states agree to
    1e-11 after every substep, and the collision returns e_n = 0.97."""
    import torch

    w = W.small("pair", 2, 0, (8.0, 10.0, 8.0))
    kw = dict(SAND, n_sub=1, dt_f=W.PHYS["dt_f"] / 50, n_iter=0, g=(0.0, 0.0, 0.0))
    x0 = np.array([[3.0, 5.0, 4.0], [3.0 + 1.0 - 1e-9, 5.0, 4.0]])
    u0 = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    p = oracle_params(orc, w, **kw)
    xo, uo, oo = x0.copy(), u0.copy(), np.zeros((2, 3))
    Ho = orc.History(2)
    Z = np.zeros((2, 3))
    with P.Context(prs_params(P, w, P.F64, n=2, **kw)) as ctx:
        shapes = ctx.grid_shapes()
        g = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in shapes]
        f = [torch.zeros_like(a) for a in g]
        x, u, om = dev(x0), dev(u0), dev(np.zeros((2, 3)))
        H = P.History.zeros(2)
        for k in range(600):
            ctx.step(g, f, x, u, om, H, zero_f=True)
            rc, _, _ = orc.dem(p, xo, uo, oo, Z, Z, Ho)
            assert rc == 0
            assert np.abs(x.cpu().numpy() - xo).max() < 1e-11, k
            assert np.abs(u.cpu().numpy() - uo).max() < 1e-11, k
            if k > 10 and int(H.count.sum()) == 0:
                break
    assert (uo[1, 0] - uo[0, 0]) == pytest.approx(0.97, abs=0.01)
