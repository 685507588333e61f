"""The settled bed patches of the named workloads, and their tiling into beds.

The patches were written by ``oracle/settle_beds.py`` (spheres settled under
gravity by the oracle's DEM, as the paper builds its beds, sec. 4.1).  These
CPU tests check that a stored patch is a settled bed: every sphere rests on
the floor through a chain of contacts (the bed detection of sec. 4.3.1 marks
them all), overlaps are of the size the weights produce, the coordination is
that of a frictional random packing, and no sphere hangs without a support
below it.  The tiling test checks that copies of a patch join across the
patch edges exactly as the patch joins itself across its periodic seams.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2108_01814_amd import workloads as W

PATCHES = sorted({w.bed for w in W.WORKLOADS.values() if w.bed})


def _params(edge, Ly, h=0.1):
    return O.make_params(nx=int(round(edge / h)), ny=int(round(Ly / h)), nz=int(round(edge / h)),
                         h=h, R=0.5, use_cells=1)


def _separation(x, i, j, Lx, Lz):
    d = x[j] - x[i]
    d[0] -= Lx * round(d[0] / Lx)
    d[2] -= Lz * round(d[2] / Lz)
    return d


@pytest.mark.parametrize("name", PATCHES)
def test_patch_is_settled(name):
    x, edge = W.load_patch(name)
    n = len(x)
    Ly = math.ceil(x[:, 1].max() + 2.0)
    p = _params(edge, Ly)
    rc, pairs, npairs = O.contacts(p, x)
    assert rc == 0 and npairs == len(pairs)
    # nearly every sphere reaches the floor through contacts (the rest are
    # rattlers)
    rc, flags, n_bed = O.bed_flags(p, x)
    assert rc == 0 and n_bed >= 0.99 * n
    sphere = pairs[pairs[:, 1] >= 0]
    wall = pairs[pairs[:, 1] == -1]
    assert len(pairs[pairs[:, 1] == -2]) == 0          # nothing touches the top
    # overlaps: positive for every listed contact, at most a few 1e-4 D
    # (the weight of the column above at k_n = 1e5 in these units)
    ov = np.array([1.0 - np.linalg.norm(_separation(x, i, j, edge, edge)) for i, j in sphere])
    assert ov.min() > 0.0 and ov.max() < 2e-3
    assert (0.5 - x[wall[:, 0], 1]).max() < 2e-3
    # coordination (contacts per sphere, each sphere pair listed once,
    # walls included) of a frictional random packing
    z = (2 * len(sphere) + len(wall)) / n
    assert 4.0 < z < 6.0, z
    # nearly every sphere has a contact with a lower centre (or the floor);
    # a settled frictional packing keeps a few rattlers (spheres loose in
    # their cage) and a few spheres held sideways by friction
    lower = np.zeros(n, dtype=bool)
    for i, j in sphere:
        lower[i if x[j, 1] < x[i, 1] else j] = True
    lower[wall[:, 0]] = True
    assert (~lower).sum() <= 0.01 * n


def test_tiled_bed_joins_across_patch_edges():
    w = W.C2
    xp, edge = W.load_patch(w.bed)
    Ly = w.domain[1]
    rc, pp, _ = O.contacts(_params(edge, Ly), xp)
    assert rc == 0
    bed = W.make_bed(w)
    # the bed spheres only (the saltating spheres sit above bed_top)
    is_bed = bed.x[:, 1] < bed.bed_top - 0.5 + 1e-9
    xb = np.ascontiguousarray(bed.x[is_bed])
    assert len(xb) == w.n_bed
    Lx, _, Lz = w.domain
    p = O.make_params(nx=int(round(Lx * 10)), ny=int(round(Ly * 10)), nz=int(round(Lz * 10)),
                      h=0.1, R=0.5, use_cells=1)
    rc, pb, _ = O.contacts(p, xb)
    assert rc == 0
    copies = w.n_bed // len(xp)
    assert len(pb) == copies * len(pp)
    assert (pb[:, 1] == -1).sum() == copies * (pp[:, 1] == -1).sum()


def test_seed_shifts_the_tiling():
    w = W.C1
    a, b = W.make_bed(w, seed=5), W.make_bed(w, seed=6)
    assert not np.allclose(np.sort(a.x[:, 0]), np.sort(b.x[:, 0]))
    # a periodic translation: the same bed heights
    ha = np.sort(a.x[:, 1])[: w.n_bed]
    hb = np.sort(b.x[:, 1])[: w.n_bed]
    assert np.array_equal(ha, hb)


def _pairs_of_history(h):
    """Sphere pairs (i < j) and wall rows of a history in the step's layout."""
    n = len(h["count"])
    owner = np.repeat(np.arange(n), h["count"].astype(np.int64))
    slot = np.concatenate([np.arange(c) for c in h["count"].astype(np.int64)]) if n else []
    partner = h["partner"][owner, slot]
    sp = partner >= 0
    pairs = {(int(a), int(b)) for a, b in zip(owner[sp], partner[sp])}
    walls = {int(a) for a in owner[partner == W.WALL_BOTTOM]}
    return pairs, walls, h["count"]


@pytest.mark.parametrize("w", [W.C1, W.C2], ids=["c1", "c2"])
def test_bed_history_is_the_settled_contact_set(w):
    """The tiled history at rest: symmetric, slots in the step's order, and
    the contacts of the bed's positions (a contact within the last
    settling substep's motion of touching may differ)."""
    bed = W.make_bed(w)
    h = bed.hist
    assert h is not None
    pairs, walls, count = _pairs_of_history(h)
    assert all((b, a) in pairs for a, b in pairs)
    # slots: partners ascending, then the bottom wall; unused slots zero
    for i in np.flatnonzero(count):
        p = h["partner"][i, : count[i]]
        sp = p[p >= 0]
        assert np.all(np.diff(sp) > 0) and np.all(p[len(sp):] == W.WALL_BOTTOM)
        assert np.all(h["partner"][i, count[i]:] == 0)
    Lx, Ly, Lz = w.domain
    p = O.make_params(nx=int(round(Lx * 10)), ny=int(round(Ly * 10)), nz=int(round(Lz * 10)),
                      h=0.1, R=0.5, use_cells=1)
    rc, ref, _ = O.contacts(p, bed.x)
    assert rc == 0
    ref_pairs = {(int(a), int(b)) for a, b in ref if b >= 0}
    ref_pairs |= {(b, a) for a, b in ref_pairs}
    ref_walls = {int(a) for a, b in ref if b == -1}
    diff = len(pairs ^ ref_pairs) + len(walls ^ ref_walls)
    assert diff <= 0.002 * (len(ref_pairs) + len(ref_walls)), diff
    # the settled bed has no initial velocities
    assert w.bed_u_std > 0 or np.count_nonzero(bed.u[bed.x[:, 1] < bed.bed_top - 0.5 + 1e-9]) == 0
