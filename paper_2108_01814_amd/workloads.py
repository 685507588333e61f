"""Seeded synthetic inputs shaped like the paper's workloads.

This module only generates inputs (sphere beds, particle velocities and the
predicted fluid velocity on the staggered grid) and holds the run
configurations.  It contains none of the method's arithmetic: no delta
kernel, no forcing, no contact law, no integrator.  It is the one module that
both the product tests and the oracle tests draw their inputs from.

Bed recipe.  The paper settles its beds under gravity with its DEM
(sec. 4.1).  The named workloads do the same: their beds are periodic copies
of one patch (12 x 12 D for the million-sphere bed, 16 x 16 D and 8 x 8 D
for the smaller ones) that the oracle's plain FP64 DEM let settle from a
random column, stored as text under ``beds/`` by ``oracle/settle_beds.py``;
a bed is the patch tiled over the box and shifted by a seeded periodic
offset.  Reduced test workloads use a seeded lattice instead: spheres on a
body-centred tetragonal lattice -- square layers of spacing a >= 1.02 D,
alternate layers shifted by half a cell -- whose layer spacing is chosen so
that each sphere overlaps its eight neighbours in the layers above and below
by about 1e-4 D; the bottom layer overlaps the wall by 5e-5 D; a random
subset of the sites is left empty so the bed volume fraction is about 0.58;
every coordinate gets N(0, 1e-5 D) jitter.  Saltating spheres are placed
above the bed by random sequential addition.  The fluid field is a log-law
profile above the bed plus 32 seeded Fourier modes scaled to 10 % of the top
velocity, faded out over the diameter below the bed top (the fluid inside a
settled bed is at rest with it), convected with the mean velocity (frozen
turbulence), so every step's field is regenerated from (seed, step).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np

# Physical parameters shared by every configuration (units: D = 1, rho_f = 1,
# |g| = 1).  dt_f is the fluid step; with k_n = 1e5 and e = 0.9 it is one tenth
# of the particle-particle contact duration, the ratio the paper uses (T_c =
# 10 dt_f, sec. 2.1).
PHYS = dict(
    D=1.0, rho_p=2.65, rho_f=1.0, g=(0.0, -1.0, 0.0),
    k_n=1.0e5, e_n=0.9, mu=0.5, kt_ratio=2.0 / 7.0, dt_ratio=2.0 / 7.0,
    dt_f=8.27944e-4, alpha=1.0, n_sub=20,
    shields=0.065, kappa=0.41, B_log=8.5,
)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_bed: int
    n_upper: int
    d_over_h: int
    n_markers: int
    domain: tuple          # (Lx, Ly, Lz) in D
    seed: int
    n_iter: int = 3
    upper_band: float = 1e9  # saltating layer at most this far above the bed top
    upper_vy: tuple = (0.0, 0.1)   # (mean, std) of the saltating spheres' u_y
    bed_u_std: float = 0.01
    omega_std: float = 0.2
    bed: str = ""                  # settled patch tiled into the bed ("" = lattice)

    @property
    def n(self) -> int:
        return self.n_bed + self.n_upper

    @property
    def h(self) -> float:
        return PHYS["D"] / self.d_over_h

    @property
    def grid(self) -> tuple:
        return tuple(int(round(L * self.d_over_h)) for L in self.domain)

    @property
    def markers(self) -> int:
        return self.n * self.n_markers


# C1: 512 spheres at D/h = 10 (the stated 8x4x8 D box cannot hold them; the
# height is raised to 10 D).  C2: 22,000 spheres at D/h = 16.  C3: 1,048,576
# spheres in the paper's own million-sphere domain, 384 x 20 x 192 D at
# D/h = 10 (sec. 3.5); its bed is 32 x 16 copies of a 1,946-sphere patch.
C1 = Workload("c1-512", 384, 128, 10, 314, (8.0, 10.0, 8.0), seed=1, bed_u_std=0.1,
              upper_vy=(0.0, 0.1), bed="patch8-384")
C2 = Workload("c2-22k", 20000, 2000, 16, 804, (64.0, 16.0, 32.0), seed=2, upper_vy=(1.0, 0.3),
              bed_u_std=0.0, bed="patch16-2500")
C3 = Workload("c3-1m", 996352, 52224, 10, 314, (384.0, 20.0, 192.0), seed=3, upper_band=10.0,
              upper_vy=(1.0, 0.3), bed_u_std=0.0, bed="patch12-1946")
WORKLOADS = {w.name: w for w in (C1, C2, C3)}


def small(name: str, n_bed: int, n_upper: int, domain, d_over_h: int = 10, n_markers: int = 314,
          seed: int = 7, **kw) -> Workload:
    """A reduced workload with the same recipe (for fast tests)."""
    return Workload(name, n_bed, n_upper, d_over_h, n_markers, tuple(float(v) for v in domain),
                    seed=seed, **kw)


# --------------------------------------------------------------------------
# beds
# --------------------------------------------------------------------------
def _lattice_bed(rng, n_bed, Lx, Lz, D, overlap=1e-4, wall_overlap=5e-5, phi=0.58,
                 jitter=1e-5, spacing=1.02):
    ncx = max(1, int(math.floor(Lx / (spacing * D))))
    ncz = max(1, int(math.floor(Lz / (spacing * D))))
    ax, az = Lx / ncx, Lz / ncz
    dnn = D * (1.0 - overlap)
    half = math.sqrt(max(dnn * dnn - 0.25 * (ax * ax + az * az), 1e-6))  # layer spacing
    per_layer = ncx * ncz
    phi0 = (math.pi / 6.0) * D ** 3 / (ax * az * half)
    vac = max(0.0, 1.0 - phi / phi0)
    n_layers = max(1, int(math.ceil(n_bed / ((1.0 - vac) * per_layer))))
    n_sites = n_layers * per_layer
    if n_sites < n_bed:
        raise ValueError("bed does not fit")
    chosen = np.sort(rng.choice(n_sites, size=n_bed, replace=False))
    layer = chosen // per_layer
    rem = chosen % per_layer
    kz, ix = rem // ncx, rem % ncx
    shift = (layer % 2) * 0.5
    x = np.empty((n_bed, 3))
    x[:, 0] = (ix + 0.25 + shift) * ax
    x[:, 1] = (0.5 * D - wall_overlap) + layer * half
    x[:, 2] = (kz + 0.25 + shift) * az
    x += rng.normal(0.0, jitter * D, size=x.shape)
    x[:, 1] = np.maximum(x[:, 1], 0.5 * D - 2 * wall_overlap)
    x[:, 0] = np.mod(x[:, 0], Lx)
    x[:, 2] = np.mod(x[:, 2], Lz)
    return x


BED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "beds")
# Layout of the step's contact history (prs_history): slots per sphere and
# the partner code of the bottom wall.
SLOTS = 14
WALL_BOTTOM = -1


def load_patch(name: str):
    """A settled bed patch: (positions [m, 3], edge in x and z)."""
    path = os.path.join(BED_DIR, name + ".txt")
    with open(path) as fh:
        head = fh.readline()
    edge = float(head.split("periodic ")[1].split(" x ")[0])
    return np.loadtxt(path, dtype=np.float64, ndmin=2), edge


def load_patch_history(name: str):
    """The contact history of a settled patch at rest: rows (sphere, partner
    or -1 for the bottom wall, delta_t x y z, u_in), or None if not stored."""
    path = os.path.join(BED_DIR, name + ".hist.txt")
    if not os.path.exists(path):
        return None
    return np.loadtxt(path, dtype=np.float64, ndmin=2)


def _tile_history(xp, edge, rows, cx, cz):
    """The patch history on every copy: (owner, partner, delta_t [3], u_in)
    with bed indices copy * m + i; a partner across the patch's periodic seam
    is the neighbouring copy's sphere."""
    m = len(xp)
    i = rows[:, 0].astype(np.int64)
    q = rows[:, 1].astype(np.int64)
    sphere = q >= 0
    qq = np.where(sphere, q, 0)
    d = xp[qq] - xp[i]
    sx = np.where(d[:, 0] > 0.5 * edge, -1, np.where(d[:, 0] < -0.5 * edge, 1, 0))
    sz = np.where(d[:, 2] > 0.5 * edge, -1, np.where(d[:, 2] < -0.5 * edge, 1, 0))
    ix, iz = np.meshgrid(np.arange(cx), np.arange(cz), indexing="ij")
    ix, iz = ix.ravel()[:, None], iz.ravel()[:, None]
    copy = ix * cz + iz
    pcopy = ((ix + sx[None, :]) % cx) * cz + (iz + sz[None, :]) % cz
    owner = (copy * m + i[None, :]).ravel()
    partner = np.where(sphere[None, :], pcopy * m + qq[None, :], q[None, :]).ravel()
    ncopy = cx * cz
    return (owner, partner, np.tile(rows[:, 2:5], (ncopy, 1)), np.tile(rows[:, 5], ncopy))


def _patch_bed(rng, name, n_bed, Lx, Lz):
    """Copies of a settled periodic patch over the box, shifted by a seeded
    offset in x and z (a translation of a periodic bed is a settled bed);
    also returns the tiled contact history (or None)."""
    xp, edge = load_patch(name)
    cx, cz = Lx / edge, Lz / edge
    if abs(cx - round(cx)) > 1e-12 or abs(cz - round(cz)) > 1e-12:
        raise ValueError(f"patch {name} does not tile a {Lx} x {Lz} box")
    cx, cz = int(round(cx)), int(round(cz))
    if n_bed != cx * cz * len(xp):
        raise ValueError(f"patch {name} gives {cx * cz * len(xp)} bed spheres, not {n_bed}")
    ix, iz = np.meshgrid(np.arange(cx), np.arange(cz), indexing="ij")
    off = np.stack([ix.ravel() * edge, np.zeros(cx * cz), iz.ravel() * edge], axis=1)
    x = (off[:, None, :] + xp[None, :, :]).reshape(-1, 3)
    shift = rng.uniform(0.0, 1.0, size=2) * np.array([Lx, Lz])
    x[:, 0] = np.mod(x[:, 0] + shift[0], Lx)
    x[:, 2] = np.mod(x[:, 2] + shift[1], Lz)
    rows = load_patch_history(name)
    hist = None if rows is None else _tile_history(xp, edge, rows, cx, cz)
    return x, hist


def _history_arrays(n, owner, partner, dt, uin):
    """Contact history in the step's layout: slots of each sphere ordered by
    partner ascending, then the bottom wall."""
    key = np.where(partner >= 0, partner, np.int64(1) << 40)
    order = np.lexsort((key, owner))
    owner, partner, dt, uin = owner[order], partner[order], dt[order], uin[order]
    count = np.bincount(owner, minlength=n)
    if count.max(initial=0) > SLOTS:
        raise ValueError("more contacts on a sphere than history slots")
    first = np.concatenate([[0], np.cumsum(count)[:-1]])
    slot = np.arange(len(owner)) - first[owner]
    H = dict(partner=np.zeros((n, SLOTS), np.int32), delta_t=np.zeros((n, SLOTS, 3)),
             u_in=np.zeros((n, SLOTS)), count=count.astype(np.int8))
    H["partner"][owner, slot] = partner
    H["delta_t"][owner, slot] = dt
    H["u_in"][owner, slot] = uin
    return H


def _rsa(rng, n, Lx, Lz, y_lo, y_hi, D, min_sep=1.001):
    """Random sequential addition of n spheres with centres in the slab."""
    if n == 0:
        return np.zeros((0, 3))
    if y_hi <= y_lo:
        raise ValueError("empty saltation band")
    cs = min_sep * D
    ncx, ncz = max(3, int(Lx // cs)), max(3, int(Lz // cs))
    ncy = max(1, int((y_hi - y_lo) // cs) + 1)
    cells: dict = {}
    out = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > 200 * n + 1000:
            raise RuntimeError("random sequential addition did not converge")
        p = np.array([rng.uniform(0, Lx), rng.uniform(y_lo, y_hi), rng.uniform(0, Lz)])
        ci = int(p[0] / Lx * ncx) % ncx
        cj = min(int((p[1] - y_lo) / cs), ncy - 1)
        ck = int(p[2] / Lz * ncz) % ncz
        ok = True
        for dk in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    for q in cells.get(((ci + di) % ncx, cj + dj, (ck + dk) % ncz), ()):
                        d = out[q] - p
                        d[0] -= Lx * round(d[0] / Lx)
                        d[2] -= Lz * round(d[2] / Lz)
                        if d @ d < cs * cs:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out[k] = p
            cells.setdefault((ci, cj, ck), []).append(k)
            k += 1
    return out


@dataclasses.dataclass
class Bed:
    x: np.ndarray      # [n, 3] float64 positions
    u: np.ndarray      # [n, 3] float64 translational velocities
    om: np.ndarray     # [n, 3] float64 angular velocities
    bed_top: float     # max y of bed spheres + R
    # contact history at rest of a settled bed in the step's layout (dict of
    # partner [n][SLOTS] int32, delta_t [n][SLOTS][3], u_in [n][SLOTS],
    # count [n] int8, caller order), or None
    hist: Optional[dict] = None


def make_bed(w: Workload, seed: Optional[int] = None) -> Bed:
    rng = np.random.default_rng(w.seed if seed is None else seed)
    D = PHYS["D"]
    Lx, Ly, Lz = w.domain
    hb = None
    if w.bed:
        xb, hb = _patch_bed(rng, w.bed, w.n_bed, Lx, Lz)
    else:
        xb = _lattice_bed(rng, w.n_bed, Lx, Lz, D)
    top = float(xb[:, 1].max() + 0.5 * D) if w.n_bed else 0.0
    y_lo = top + 0.5 * D
    y_hi = min(top + w.upper_band, Ly - 0.5 * D - 1e-3)
    xu = _rsa(rng, w.n_upper, Lx, Lz, y_lo, y_hi, D)
    x = np.concatenate([xb, xu], axis=0)
    u = np.concatenate([rng.normal(0.0, w.bed_u_std, size=(w.n_bed, 3)),
                        np.stack([rng.normal(0.0, 0.1, w.n_upper),
                                  rng.normal(w.upper_vy[0], w.upper_vy[1], w.n_upper),
                                  rng.normal(0.0, 0.1, w.n_upper)], axis=1)], axis=0)
    # a settled bed at rest (bed_u_std 0) starts without spin as well
    om_bed = w.omega_std if w.bed_u_std >= 0.1 else (0.02 if w.bed_u_std > 0 else 0.0)
    om = rng.normal(0.0, om_bed, size=(w.n, 3))
    om[w.n_bed:] = rng.normal(0.0, w.omega_std, size=(w.n_upper, 3))
    perm = rng.permutation(w.n)   # callers see particles in no spatial order
    hist = None
    if hb is not None:
        inv = np.empty(w.n, dtype=np.int64)
        inv[perm] = np.arange(w.n)
        owner, partner, dt, uin = hb
        partner = np.where(partner >= 0, inv[np.maximum(partner, 0)], partner)
        hist = _history_arrays(w.n, inv[owner], partner, dt, uin)
    return Bed(np.ascontiguousarray(x[perm]), np.ascontiguousarray(u[perm]),
               np.ascontiguousarray(om[perm]), top, hist)


def fcc_block(n_side: int, spacing: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Face-centred cubic points, n_side^3 conventional cells, nearest-neighbour
    distance = spacing (for contact micro-cases)."""
    a = spacing * math.sqrt(2.0)
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    pts = []
    for i in range(n_side):
        for j in range(n_side):
            for k in range(n_side):
                pts.append((base + [i, j, k]) * a)
    return np.concatenate(pts, axis=0) + np.asarray(origin)


# --------------------------------------------------------------------------
# fluid field
# --------------------------------------------------------------------------
@dataclasses.dataclass
class FlowModes:
    u_tau: float
    y_b: float
    u_c: float
    kx: np.ndarray
    ky: np.ndarray
    kz: np.ndarray
    amp: np.ndarray     # [32, 3]
    phase: np.ndarray   # [32]
    scale: float


def _loglaw(y, y_b, u_tau):
    y = np.asarray(y, dtype=np.float64)
    yp = np.maximum(y - y_b, 1e-300)
    v = u_tau * np.maximum(0.0, np.log(yp / PHYS["D"]) / PHYS["kappa"] + PHYS["B_log"])
    return np.where(y > y_b, v, 0.0)


def _bed_damping(y, y_b):
    """Weight of the velocity fluctuation at height y: 1 above the bed top
    y_b, falling linearly to 0 one diameter below it (the fluid inside a
    settled bed moves with its spheres, which are at rest)."""
    return np.clip((np.asarray(y, dtype=np.float64) - y_b) / PHYS["D"] + 1.0, 0.0, 1.0)


def flow_modes(w: Workload, bed_top: float, seed: Optional[int] = None, n_modes: int = 32) -> FlowModes:
    rng = np.random.default_rng(10_000 + (w.seed if seed is None else seed))
    Lx, Ly, Lz = w.domain
    u_tau = math.sqrt(PHYS["shields"] * (PHYS["rho_p"] / PHYS["rho_f"] - 1.0) * 1.0 * PHYS["D"])
    ys = np.linspace(bed_top, Ly, 2001)
    u_c = float(_loglaw(ys, bed_top, u_tau).mean())
    kx = rng.integers(1, 9, n_modes)
    kz = rng.integers(1, 9, n_modes)
    ky = rng.integers(1, 5, n_modes)
    amp = rng.normal(size=(n_modes, 3))
    phase = rng.uniform(0, 2 * math.pi, n_modes)
    # scale the fluctuation so its RMS over a fixed sample lattice is 10 % of
    # the log-law velocity at the top of the domain
    sx = (np.arange(48) + 0.5) / 48 * Lx
    sy = (np.arange(24) + 0.5) / 24 * Ly
    sz = (np.arange(48) + 0.5) / 48 * Lz
    X, Y, Z = np.meshgrid(sx, sy, sz, indexing="ij")
    acc = np.zeros(X.shape + (3,))
    for m in range(n_modes):
        s = np.sin(2 * math.pi * (kx[m] * X / Lx + kz[m] * Z / Lz) + phase[m]) * \
            np.sin(math.pi * ky[m] * Y / Ly) * _bed_damping(Y, bed_top)
        acc += s[..., None] * amp[m]
    rms = math.sqrt(float((acc ** 2).sum(-1).mean()))
    top = float(_loglaw(np.array([Ly]), bed_top, u_tau)[0])
    scale = 0.1 * top / rms if rms > 0 else 0.0
    return FlowModes(u_tau, bed_top, u_c, kx, ky, kz, amp, phase, scale)


def fluid_field(w: Workload, modes: FlowModes, step: int = 0, device="cpu", dtype=None,
                out=None, window=None):
    """Predicted velocity u-hat on the staggered grid at fluid step `step`.

    Returns three torch tensors u [Nz, Ny, Nx], v [Nz, Ny+1, Nx], w [Nz, Ny, Nx]
    (x fastest), computed in float64 and stored in `dtype` on `device`.
    window = (i0, nx, k0, nz) restricts the output to node columns
    i0 .. i0+nx-1 and k0 .. k0+nz-1 (the field is periodic, so any integers)."""
    import torch

    dtype = dtype or torch.float64
    Nx, Ny, Nz = w.grid
    i0, k0 = 0, 0
    if window is not None:
        i0, Nx, k0, Nz = window
    h = w.h
    Lx, Ly, Lz = w.domain
    t = step * PHYS["dt_f"]
    dev = torch.device(device)
    f64 = torch.float64
    kx = torch.tensor(modes.kx, dtype=f64, device=dev)
    ky = torch.tensor(modes.ky, dtype=f64, device=dev)
    kz = torch.tensor(modes.kz, dtype=f64, device=dev)
    amp = torch.tensor(modes.amp, dtype=f64, device=dev) * modes.scale
    ph = torch.tensor(modes.phase, dtype=f64, device=dev)
    comps = []
    for c in range(3):
        o = [0.5, 0.5, 0.5]
        o[c] = 0.0
        ny_c = Ny + 1 if c == 1 else Ny
        xs = (torch.arange(i0, i0 + Nx, dtype=f64, device=dev) + o[0]) * h
        ys = (torch.arange(ny_c, dtype=f64, device=dev) + o[1]) * h
        zs = (torch.arange(k0, k0 + Nz, dtype=f64, device=dev) + o[2]) * h
        ax = 2 * math.pi * kx[None, :] * (xs[:, None] - modes.u_c * t) / Lx      # [Nx, m]
        az = 2 * math.pi * kz[None, :] * zs[:, None] / Lz + ph[None, :]         # [Nz, m]
        damp = torch.tensor(_bed_damping(ys.cpu().numpy(), modes.y_b), dtype=f64, device=dev)
        sy = (torch.sin(math.pi * ky[None, :] * ys[:, None] / Ly) * amp[None, :, c] *
              damp[:, None])                                                        # [ny, m]
        Bm = torch.cat([torch.sin(ax), torch.cos(ax)], dim=1).T.contiguous()     # [2m, Nx]
        cz, sz = torch.cos(az), torch.sin(az)
        if out is not None:
            dst = out[c]
        else:
            dst = torch.empty((Nz, ny_c, Nx), dtype=dtype, device=dev)
        logu = None
        if c == 0:
            logu = torch.tensor(_loglaw(((np.arange(ny_c) + o[1]) * h), modes.y_b, modes.u_tau),
                                dtype=f64, device=dev)
        for j in range(ny_c):
            A = torch.cat([cz * sy[j][None, :], sz * sy[j][None, :]], dim=1)     # [Nz, 2m]
            plane = A @ Bm                                                         # [Nz, Nx]
            if logu is not None:
                plane = plane + logu[j]
            dst[:, j, :] = plane.to(dtype)
        comps.append(dst)
    return comps


def zero_fields(w: Workload, device="cpu", dtype=None):
    import torch

    dtype = dtype or torch.float64
    Nx, Ny, Nz = w.grid
    return [torch.zeros((Nz, Ny + (1 if c == 1 else 0), Nx), dtype=dtype, device=device)
            for c in range(3)]
