"""Settle the periodic bed patches of the synthetic workloads with the oracle's DEM.

Test infrastructure like the rest of ``oracle/``: it writes the files under
``paper_2108_01814_amd/beds/``, which the input generator tiles into beds.
The paper builds its beds by letting spheres settle under gravity with its
own DEM (sec. 4.1); this script does the same with the plain FP64 DEM of
this oracle (linear spring-dashpot, tangential spring and Coulomb cap,
App. A), in a box that is periodic in x and z with a wall at y = 0:

1. random sequential addition of the patch's spheres into a tall column,
   at rest;
2. DEM substeps under buoyant gravity only (no fluid force), with a low
   normal restitution so that the pile comes to rest quickly and a larger
   substep than a coupled run's (still 25 per contact duration);
3. stop once the largest sphere speed has stayed below a threshold for a
   whole chunk of substeps.

The stiffness, gravity, densities and friction are those of the workloads,
so a settled patch is at rest under the coupled runs' contact law too (its
overlaps and tangential springs balance the same weights).  The contact
history at rest (partners, tangential displacements, impact velocities) is
stored with the positions, so a run can start from the settled state
itself rather than from unloaded tangential springs.  Usage:

    python -m oracle.settle_beds [name ...]
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

from . import History, dem, make_params
from paper_2108_01814_amd import workloads as W

OUT_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2108_01814_amd", "beds")

# patch name -> (patch edge in x and z in D, spheres, seed)
PATCHES = {
    "patch12-1946": (12.0, 1946, 31),
    "patch16-2500": (16.0, 2500, 32),
    "patch8-384": (8.0, 384, 33),
}

E_SETTLE = 0.1          # normal restitution while settling
SUB_PER_CONTACT = 25    # substeps per contact duration while settling
V_REST = 5e-3           # largest speed (D per unit time) taken as rest
COLUMN_PHI = 0.2        # volume fraction of the initial column


def settle(edge: float, n: int, seed: int, log=print):
    D = W.PHYS["D"]
    rng = np.random.default_rng(seed)
    height = n * (math.pi / 6.0) * D ** 3 / (COLUMN_PHI * edge * edge)
    Ly = math.ceil(height + 2.0)
    x = W._rsa(rng, n, edge, edge, 0.5 * D + 1e-3, height, D)
    u = np.zeros_like(x)
    om = np.zeros_like(x)
    # contact duration of a sphere pair at the workloads' stiffness
    m = W.PHYS["rho_p"] * math.pi / 6.0 * D ** 3
    t_c = math.pi * math.sqrt(0.5 * m / W.PHYS["k_n"])
    n_sub = 20
    h = 0.1
    p = make_params(nx=int(round(edge / h)), ny=int(round(Ly / h)), nz=int(round(edge / h)), h=h,
                    R=0.5 * D, rho_p=W.PHYS["rho_p"], rho_f=W.PHYS["rho_f"], g=W.PHYS["g"],
                    k_n=W.PHYS["k_n"], e_n=E_SETTLE, mu=W.PHYS["mu"],
                    kt_ratio=W.PHYS["kt_ratio"], dt_ratio=W.PHYS["dt_ratio"],
                    dt_f=n_sub * t_c / SUB_PER_CONTACT, n_sub=n_sub, use_cells=1)
    hist = History(n)
    Fh = np.zeros((n, 3))
    t0 = time.time()
    calls, rest = 0, 0
    while True:
        rc, _, _ = dem(p, x, u, om, Fh, Fh, hist)
        if rc:
            raise RuntimeError(f"oracle DEM returned {rc}")
        calls += 1
        vmax = float(np.sqrt((u * u).sum(axis=1)).max())
        rest = rest + 1 if vmax < V_REST else 0
        if calls % 200 == 0:
            log(f"  {calls * n_sub} substeps, t = {calls * p.dt_f:.2f}, max speed {vmax:.3g}, "
                f"top {x[:, 1].max() + 0.5 * D:.2f} D, {time.time() - t0:.0f} s")
        if rest >= 20:
            break
        if calls > 20000:
            raise RuntimeError("bed did not come to rest")
    contacts = int(hist.cnt.sum())
    log(f"  at rest after {calls * n_sub} substeps: coordination {contacts / n:.2f}, "
        f"top {x[:, 1].max() + 0.5 * D:.2f} D")
    return x, hist


def write_patch(name: str):
    edge, n, seed = PATCHES[name]
    print(f"{name}: {n} spheres, {edge} x {edge} D, seed {seed}")
    x, hist = settle(edge, n, seed)
    order = np.lexsort((x[:, 2], x[:, 0], x[:, 1]))
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    os.makedirs(OUT_DIR, exist_ok=True)
    path = os.path.join(OUT_DIR, name + ".txt")
    header = (f"bed patch {name}: {n} spheres of diameter 1, periodic {edge} x {edge} in x and z, "
              f"wall at y = 0; settled under buoyant gravity by the oracle's DEM "
              f"(python -m oracle.settle_beds {name}, seed {seed}); columns x y z")
    np.savetxt(path, x[order], fmt="%.17g", header=header)
    # the contact history at rest, one row per contact slot, sphere indices
    # in the order of the positions file; partner -1: the bottom wall
    rows = []
    for i in range(n):
        p = order[i]
        for k in range(hist.cnt[p]):
            q = int(hist.partner[p, k])
            rows.append([i, rank[q] if q >= 0 else q, *hist.dt[p, k], hist.uin[p, k]])
    hpath = os.path.join(OUT_DIR, name + ".hist.txt")
    hheader = (f"contact history of bed patch {name} at rest (python -m oracle.settle_beds "
               f"{name}); columns: sphere, partner (-1 bottom wall), delta_t x y z, u_in")
    np.savetxt(hpath, np.array(rows), fmt=["%d", "%d", "%.12g", "%.12g", "%.12g", "%.12g"],
               header=hheader)
    print(f"  wrote {path} and {hpath}")


if __name__ == "__main__":
    names = sys.argv[1:] or list(PATCHES)
    for nm in names:
        write_patch(nm)
