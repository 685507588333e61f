"""Shared test set-up: the same seeded inputs and parameters for the HIP path
and the oracle."""
from __future__ import annotations

import numpy as np

from paper_2108_01814_amd import workloads as W


def phys_kw(w: W.Workload, **kw):
    P = W.PHYS
    d = dict(h=w.h, nl=w.n_markers, rho_p=P["rho_p"], rho_f=P["rho_f"], g=P["g"],
             dt_f=P["dt_f"], alpha=P["alpha"], n_iter=w.n_iter, n_sub=P["n_sub"], k_n=P["k_n"],
             e_n=P["e_n"], mu=P["mu"], kt_ratio=P["kt_ratio"], dt_ratio=P["dt_ratio"])
    d.update(kw)
    return d


def oracle_params(orc, w: W.Workload, **kw):
    d = phys_kw(w, **kw)
    nx, ny, nz = w.grid
    d.setdefault("use_cells", 1)
    return orc.make_params(nx=nx, ny=ny, nz=nz, R=0.5 * W.PHYS["D"], **d)


def prs_params(P, w: W.Workload, precision, n=None, **kw):
    d = phys_kw(w, **kw)
    nx, ny, nz = w.grid
    d["gravity"] = d.pop("g")
    d["n_markers"] = d.pop("nl")
    return P.make_params(nx=nx, ny=ny, nz=nz, radius=0.5 * W.PHYS["D"], precision=precision,
                         max_particles=n if n is not None else w.n, **d)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    if den == 0:
        return float(np.abs(a).max())
    return float(np.abs(a - b).max() / den)


def fields_for(w: W.Workload, bed: W.Bed, step: int = 0):
    """u-hat of the workload as float64 CPU tensors."""
    modes = W.flow_modes(w, bed.bed_top)
    return W.fluid_field(w, modes, step=step)
