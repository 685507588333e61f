"""Edge cases of the step against the oracle (FP64 1e-11, FP32 1e-5):
marker counts at the extremes of a workgroup (a ragged 37, exactly one
wave, the maximum 1024), and the brick shapes of the interpolation (14 nodes
at D/h = 10 and 20 at D/h = 16, compiled with the edge known, and 16 at
D/h = 12, the general path)."""
import numpy as np
import pytest

from helpers import fields_for, oracle_params, prs_params, rel_err
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}


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


def run_both(P, orc, w, precision, stale=0.0):
    import torch

    bed = W.make_bed(w)
    dt = torch.float64 if precision == 1 else torch.float32
    g = [a.to(device="cuda", dtype=dt).contiguous() for a in fields_for(w, bed)]
    x, u, om = (torch.as_tensor(a).cuda() for a in (bed.x, bed.u, bed.om))
    print(f"{w.name}: {w.n} spheres, D/h {w.d_over_h}, {w.n_markers} markers, "
          f"precision {precision}, f on entry {stale}", flush=True)
    with P.Context(prs_params(P, w, precision)) as ctx:
        H = P.History.zeros(w.n)
        f = [torch.full_like(a, stale) for a in g]
        Fh, Th, st = ctx.step(g, f, x, u, om, H, zero_f=True)
        gpu = dict(Fh=Fh.cpu().numpy(), Th=Th.cpu().numpy(), x=x.cpu().numpy(),
                   f=[a.double().cpu().numpy() for a in f], st=st)
    uh = [np.ascontiguousarray(a.double().cpu().numpy()) for a in g]
    fo = [np.zeros_like(a) for a in uh]
    xo, uo, oo = bed.x.copy(), bed.u.copy(), bed.om.copy()
    rc, out = orc.step(oracle_params(orc, w), uh, fo, xo, uo, oo, orc.History(w.n))
    assert rc == 0
    return gpu, dict(Fh=out["Fh"], Th=out["Th"], x=xo, f=fo, slip=out["slip"])


def check(gpu, ref, tol):
    assert np.allclose(gpu["st"]["rel_slip"], ref["slip"], rtol=10 * tol, atol=0)
    assert rel_err(gpu["Fh"], ref["Fh"]) < tol
    assert rel_err(gpu["Th"], ref["Th"]) < tol
    for c in range(3):
        assert rel_err(gpu["f"][c], ref["f"][c]) < tol
    assert np.abs(gpu["x"] - ref["x"]).max() < tol


@pytest.mark.parametrize("nl", [37, 64, 1024])
@pytest.mark.parametrize("precision", [1, 0])
def test_marker_count_extremes(P, orc, nl, precision):
    # (fewer than about 20 markers is no test of the method: the marker volume
    # then exceeds 16 h^3 and the Jacobi forcing amplifies the slip by
    # |1 - dV/(8h^3)| > 1 per pass)
    w = W.small(f"nl{nl}", 40, 10, (4.0, 6.0, 4.0), n_markers=nl, seed=21, bed_u_std=0.1)
    gpu, ref = run_both(P, orc, w, precision)
    check(gpu, ref, TOL[precision])


@pytest.mark.parametrize("d_over_h,nl", [(16, 804), (12, 452)], ids=["brick20", "brick16"])
@pytest.mark.parametrize("precision", [1, 0])
def test_brick_shapes(P, orc, d_over_h, nl, precision):
    w = W.small(f"dh{d_over_h}", 30, 8, (4.0, 5.0, 4.0), d_over_h=d_over_h, n_markers=nl,
                seed=23, bed_u_std=0.1)
    gpu, ref = run_both(P, orc, w, precision)
    check(gpu, ref, TOL[precision])


@pytest.mark.parametrize("precision", [1, 0])
def test_zero_f_overwrites_a_stale_field(P, orc, precision):
    # zero_f: the first spreading pass stores every node of f instead of
    # adding to it, so NaN left in f on entry must not survive anywhere
    w = W.small("stale", 40, 10, (4.0, 6.0, 4.0), seed=25, bed_u_std=0.1)
    gpu, ref = run_both(P, orc, w, precision, stale=float("nan"))
    for c in range(3):
        assert np.isfinite(gpu["f"][c]).all()
    check(gpu, ref, TOL[precision])


@pytest.mark.parametrize("kw", [dict(n_iter=0), dict(tol_mode=1, tol=2.0, max_iter=5)],
                         ids=["no_iterations", "tolerance_met_at_once"])
def test_zero_f_without_a_spreading_pass_clears_f(P, kw):
    # no spreading pass runs: the field is cleared on its own
    import torch

    w = W.small("nospread", 20, 10, (4.0, 6.0, 4.0), seed=26)
    bed = W.make_bed(w)
    g = [a.to(device="cuda").contiguous() for a in fields_for(w, bed)]
    x, u, om = (torch.as_tensor(a).cuda() for a in (bed.x, bed.u, bed.om))
    with P.Context(prs_params(P, w, P.F64, **kw)) as ctx:
        f = [torch.full_like(a, float("nan")) for a in g]
        _, _, st = ctx.step(g, f, x, u, om, P.History.zeros(w.n), zero_f=True)
    assert st["iterations"] == 0
    for a in f:
        assert bool((a == 0).all())
