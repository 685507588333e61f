"""Parity at full size: the 1,048,576-sphere C3 bed with FP32 fields, in the
launch configuration bench.py times (3 forcing iterations, 20 substeps, skin
0.1), and the 22,000-sphere C2 bed (D/h = 16, 804 markers) in both
precisions (FP64 fields 1e-11, FP32 fields 1e-5).

The oracle cannot run the whole bed, so it runs a 12D x Ly x 12D column of
it (the spheres with centres in the column, the same FP32 field on the
column plus a 1D margin) and the spheres at least 4D inside the column are
compared: what a sphere's step depends on reaches a few diameters (three
forcing passes of stencil width, contacts a few neighbours deep with
geometrically decaying weight), so the column's missing surroundings do not
reach them.  The force field f is compared on the node columns at least
F_CORE_MARGIN inside the column (they receive spreading only from spheres at
least F_CORE_MARGIN - D inside).  Contact detection is compared bit-exactly
on the whole bed (the oracle's cell-list detector is linear in the sphere
count)."""
import math

import numpy as np
import pytest

from helpers import rel_err
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu

WIDTH, CORE_MARGIN, FIELD_MARGIN, F_CORE_MARGIN = 12.0, 4.0, 1.0, 5.0


def column(w):
    """Corner of the compared column and the node window of its field."""
    h = w.h
    x0 = 0.5 * (w.domain[0] - WIDTH)
    z0 = 0.5 * (w.domain[2] - WIDTH)
    wi0 = int(math.floor((x0 - FIELD_MARGIN) / h))
    wk0 = int(math.floor((z0 - FIELD_MARGIN) / h))
    wnx = wnz = int(math.ceil((WIDTH + 2 * FIELD_MARGIN) / h))
    return x0, z0, wi0, wnx, wk0, wnz


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


CASES = {"c3-f32": (W.C3, 0), "c2-f32": (W.C2, 0), "c2-f64": (W.C2, 1)}


@pytest.fixture(scope="module", params=list(CASES))
def full(P, request):
    """A bed, its field in the case's precision, and the GPU step on the
    whole bed."""
    import torch

    from paper_2108_01814_amd import learned as L

    w, precision = CASES[request.param]
    dt = torch.float32 if precision == 0 else torch.float64
    bed = W.make_bed(w)
    modes = W.flow_modes(w, bed.bed_top)
    g = W.fluid_field(w, modes, device="cuda", dtype=dt)
    x = torch.as_tensor(bed.x, device="cuda")
    u = torch.as_tensor(bed.u, device="cuda")
    om = torch.as_tensor(bed.om, device="cuda")
    print(f"{w.name} step on {w.n} spheres, grid {w.grid}, precision {precision}", flush=True)
    with P.Context(L.params_for(w, precision, w.n, skin=0.1)) as ctx:
        H = P.History.zeros(w.n)
        f = [torch.zeros_like(a) for a in g]
        Fh, Th, st = ctx.step(g, f, x, u, om, H, zero_f=True)
        out = dict(Fh=Fh.cpu().numpy(), Th=Th.cpu().numpy(), x=x.cpu().numpy(),
                   u=u.cpu().numpy(), om=om.cpu().numpy(), partner=H.partner.cpu().numpy(),
                   count=H.count.cpu().numpy().astype(np.int32), st=st)
        out["f_window"] = window_field(w, f, *column(w)[2:])
        del f
    yield w, bed, g, out, precision
    del g
    torch.cuda.empty_cache()


def window_field(w, g, wi0, wnx, wk0, wnz):
    """The FP32 field on node columns wi0.. (wnx) and wk0.. (wnz), periodic, as
    FP64 host arrays (the generator's values as the device stores them)."""
    import torch

    nx, _, nz = w.grid
    ix = torch.as_tensor((wi0 + np.arange(wnx)) % nx, device=g[0].device)
    kz = torch.as_tensor((wk0 + np.arange(wnz)) % nz, device=g[0].device)
    return [np.ascontiguousarray(a.index_select(2, ix).index_select(0, kz).double().cpu().numpy())
            for a in g]


def test_step_matches_oracle_inside_a_column(P, orc, full):
    w, bed, g, gpu, precision = full
    assert gpu["st"]["iterations"] == w.n_iter and gpu["st"]["flags"] == 0
    ph = W.PHYS
    nx, ny, nz = w.grid
    h = w.h
    x0, z0, wi0, wnx, wk0, wnz = column(w)
    sel = ((bed.x[:, 0] >= x0) & (bed.x[:, 0] < x0 + WIDTH) &
           (bed.x[:, 2] >= z0) & (bed.x[:, 2] < z0 + WIDTH))
    win = np.nonzero(sel)[0]
    xs, us, oms = (np.ascontiguousarray(a[sel]) for a in (bed.x, bed.u, bed.om))
    uh = window_field(w, g, wi0, wnx, wk0, wnz)
    po = orc.make_params(nx=nx, ny=ny, nz=nz, h=h, wi0=wi0 % nx, wnx=wnx, wk0=wk0 % nz, wnz=wnz,
                         R=0.5 * ph["D"], nl=w.n_markers, g=ph["g"], rho_p=ph["rho_p"],
                         rho_f=ph["rho_f"], dt_f=ph["dt_f"], alpha=ph["alpha"], n_iter=w.n_iter,
                         n_sub=ph["n_sub"], k_n=ph["k_n"], e_n=ph["e_n"], mu=ph["mu"],
                         kt_ratio=ph["kt_ratio"], dt_ratio=ph["dt_ratio"], use_cells=1)
    f = [np.zeros_like(a) for a in uh]
    H = orc.History(len(xs))
    print(f"oracle on {len(xs)} spheres of the column", flush=True)
    rc, out = orc.step(po, uh, f, xs, us, oms, H)
    assert rc == 0
    core = ((bed.x[win, 0] >= x0 + CORE_MARGIN) & (bed.x[win, 0] < x0 + WIDTH - CORE_MARGIN) &
            (bed.x[win, 2] >= z0 + CORE_MARGIN) & (bed.x[win, 2] < z0 + WIDTH - CORE_MARGIN))
    assert core.sum() > 150
    gi = win[core]
    tol = 1e-5 if precision == 0 else 1e-11
    print(f"{w.name} column core:" + " %d spheres; errors F_h %.2e T_h %.2e x %.2e u %.2e om %.2e" % (
        core.sum(), rel_err(gpu["Fh"][gi], out["Fh"][core]), rel_err(gpu["Th"][gi], out["Th"][core]),
        np.abs(gpu["x"][gi] - xs[core]).max(), rel_err(gpu["u"][gi], us[core]),
        rel_err(gpu["om"][gi], oms[core])), flush=True)
    assert rel_err(gpu["Fh"][gi], out["Fh"][core]) < tol
    assert rel_err(gpu["Th"][gi], out["Th"][core]) < tol
    assert np.abs(gpu["x"][gi] - xs[core]).max() < tol
    assert rel_err(gpu["u"][gi], us[core]) < tol
    assert rel_err(gpu["om"][gi], oms[core]) < tol
    # the force field on the core node columns (every component, every row)
    i0 = int(math.ceil((x0 + F_CORE_MARGIN) / h)) - wi0
    i1 = int(math.floor((x0 + WIDTH - F_CORE_MARGIN) / h)) - wi0
    k0 = int(math.ceil((z0 + F_CORE_MARGIN) / h)) - wk0
    k1 = int(math.floor((z0 + WIDTH - F_CORE_MARGIN) / h)) - wk0
    assert i1 - i0 >= 15 and k1 - k0 >= 15
    for c in range(3):
        a = gpu["f_window"][c][k0:k1, :, i0:i1]
        b = f[c][k0:k1, :, i0:i1]
        assert np.abs(b).max() > 0
        print(f"{w.name} column core f[{c}]: error {rel_err(a, b):.2e}", flush=True)
        assert rel_err(a, b) < tol
    # contact histories: the same partners (window indices mapped to the bed's)
    assert np.array_equal(gpu["count"][gi], H.cnt[core])
    for a, b, n in zip(gpu["partner"][gi], H.partner[core], H.cnt[core]):
        mapped = np.where(b[:n] >= 0, win[np.maximum(b[:n], 0)], b[:n])
        assert np.array_equal(a[:n], mapped)


def test_contact_list_bit_exact(P, orc, full):
    import torch

    w, bed, g, gpu, precision = full
    if precision == 1:
        pytest.skip("the contact list does not depend on the field precision")
    nx, ny, nz = w.grid
    x = np.ascontiguousarray(bed.x)
    with P.Context(P.make_params(nx=nx, ny=ny, nz=nz, h=w.h, radius=0.5 * W.PHYS["D"],
                                 n_markers=w.n_markers, precision=P.F32,
                                 max_particles=w.n)) as ctx:
        pairs = ctx.contacts(torch.as_tensor(x, device="cuda")).cpu().numpy()
    po = orc.make_params(nx=nx, ny=ny, nz=nz, h=w.h, R=0.5 * W.PHYS["D"], nl=w.n_markers,
                         use_cells=1)
    rc, ref, n_ref = orc.contacts(po, x)
    assert rc == 0 and n_ref == len(ref)
    print(f"{len(pairs)} contacts on the whole bed", flush=True)
    assert len(pairs) > w.n
    assert np.array_equal(pairs, ref)
