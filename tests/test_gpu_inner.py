"""Fluid inside the spheres and the Runge-Kutta coupling of the step, through
the C ABI, against the oracle: the inner-fluid integrals (identical node
sets, sums in a different order), and a fluid step of two Runge-Kutta
substeps (alpha_1 = 1 forcing only, then alpha_2 = 1/2 with the particle
substeps), each with the inner-fluid term, in FP64 (1e-11) and FP32
(1e-5)."""
import numpy as np
import pytest

from helpers import fields_for, oracle_params, prs_params, rel_err
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}
TINY = W.small("tiny", 40, 10, (4.0, 6.0, 4.0), seed=11, bed_u_std=0.1)


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
def test_inner_fluid_integrals(P, orc, precision, w):
    import torch

    bed = W.make_bed(w)
    dt = torch.float64 if precision == 1 else torch.float32
    g = [a.to(device="cuda", dtype=dt).contiguous() for a in fields_for(w, bed)]
    with P.Context(prs_params(P, w, precision)) as ctx:
        got = ctx.inner_fluid(g, dev(bed.x)).cpu().numpy()
    ref = orc.inner_fluid(oracle_params(orc, w), [a.double().cpu().numpy() for a in g], bed.x)
    assert np.abs(ref).max() > 0
    assert rel_err(got[:, :3], ref[:, :3]) < 1e-12
    assert rel_err(got[:, 3:], ref[:, 3:]) < 1e-12


@pytest.mark.parametrize("precision", [1, 0])
def test_runge_kutta_fluid_step(P, orc, precision):
    import torch

    w = TINY
    bed = W.make_bed(w)
    dt = torch.float64 if precision == 1 else torch.float32
    g = [a.to(device="cuda", dtype=dt).contiguous() for a in fields_for(w, bed)]
    uh = [np.ascontiguousarray(a.double().cpu().numpy()) for a in g]
    p = oracle_params(orc, w)
    # device: I0 of the initial field, substep 1 (forcing only), substep 2
    x, u, om = dev(bed.x), dev(bed.u), dev(bed.om)
    with P.Context(prs_params(P, w, precision)) as ctx:
        H = P.History.zeros(w.n)
        f = [torch.zeros_like(a) for a in g]
        I0 = ctx.inner_fluid(g, x)
        I1 = torch.empty_like(I0)
        I2 = torch.empty_like(I0)
        Fh1, Th1, st1 = ctx.step(g, f, x, u, om, H, zero_f=True, alpha=1.0, advance=False,
                                 inner_prev=I0, inner_out=I1)
        Fh1, Th1 = Fh1.cpu().numpy(), Th1.cpu().numpy()
        x1 = x.cpu().numpy()
        Fh2, Th2, st2 = ctx.step(g, f, x, u, om, H, zero_f=True, alpha=0.5, advance=True,
                                 inner_prev=I1, inner_out=I2)
        got = dict(Fh1=Fh1, Th1=Th1, Fh2=Fh2.cpu().numpy(), Th2=Th2.cpu().numpy(),
                   x=x.cpu().numpy(), u=u.cpu().numpy(), om=om.cpu().numpy(),
                   I1=I1.cpu().numpy(), I2=I2.cpu().numpy(), x1=x1,
                   partner=H.partner.cpu().numpy())
    # oracle: the same sequence
    xo, uo, oo = bed.x.copy(), bed.u.copy(), bed.om.copy()
    Ho = orc.History(w.n)
    I0o = orc.inner_fluid(p, uh, xo)
    fo = [np.zeros_like(a) for a in uh]
    rc, o1 = orc.step_ex(p, 1.0, False, uh, fo, xo, uo, oo, Ho, inner_prev=I0o, want_inner=True)
    assert rc == 0
    assert np.array_equal(xo, bed.x)
    fo = [np.zeros_like(a) for a in uh]
    rc, o2 = orc.step_ex(p, 0.5, True, uh, fo, xo, uo, oo, Ho, inner_prev=o1["inner"],
                         want_inner=True)
    assert rc == 0
    tol = TOL[precision]
    assert np.array_equal(got["x1"], bed.x)            # the first substep moves nothing
    assert rel_err(got["I1"], o1["inner"]) < tol
    assert rel_err(got["Fh1"], o1["Fh"]) < tol
    assert rel_err(got["Th1"], o1["Th"]) < tol
    assert rel_err(got["I2"], o2["inner"]) < tol
    assert rel_err(got["Fh2"], o2["Fh"]) < tol
    assert rel_err(got["Th2"], o2["Th"]) < tol
    assert np.abs(got["x"] - xo).max() < tol
    assert rel_err(got["u"], uo) < tol
    assert rel_err(got["om"], oo) < tol
    assert np.array_equal(got["partner"], Ho.partner)
