"""Pins of the oracle's bed / flying detection (sec. 4.3.1, step (1)), no GPU:
hand-built configurations whose answer is fixed by the definition (a chain
of touching spheres down to the bottom layer, a detached cluster, lone
spheres either side of the one-diameter line, the periodic seam), and random
beds against connected components of the brute-force contact graph computed
by scipy (a sphere is bed exactly when its component holds a sphere with
y < D)."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

L = (6.0, 8.0, 6.0)


def params(orc, **kw):
    return orc.make_params(nx=60, ny=80, nz=60, h=0.1, nl=10, **kw)


def flags(orc, x, use_cells=1):
    rc, f, nb = orc.bed_flags(params(orc, use_cells=use_cells), np.asarray(x, dtype=float))
    assert rc == 0
    assert nb == int(f.sum())
    return f


def test_chain_to_the_floor_is_bed(orc):
    # a vertical chain, each sphere 0.98 D above the previous, from y = 0.6
    x = np.array([[3.0, 0.6 + 0.98 * k, 3.0] for k in range(6)])
    assert flags(orc, x).tolist() == [1] * 6


def test_detached_cluster_is_flying(orc):
    x = np.array([[1.0, 0.55, 1.0],                       # bottom layer
                  [4.0, 4.0, 4.0], [4.0, 4.95, 4.0], [4.9, 4.5, 4.0]])   # touching, aloft
    assert flags(orc, x).tolist() == [1, 0, 0, 0]


def test_one_diameter_line(orc):
    # lone spheres: below y = D bed, at or above it flying (y < D strictly)
    x = np.array([[1.0, 0.999, 1.0], [3.0, 1.0, 3.0], [5.0, 1.3, 5.0], [1.0, 7.6, 5.0]])
    assert flags(orc, x).tolist() == [1, 0, 0, 0]      # the last touches the top wall only


def test_chain_across_the_periodic_seam(orc):
    x = np.array([[0.2, 0.55, 3.0], [L[0] - 0.6, 1.1, 3.0], [L[0] - 0.9, 1.95, 3.0],
                  [L[0] - 0.9, 3.5, 3.0]])                # the last is detached
    assert flags(orc, x).tolist() == [1, 1, 1, 0]


def contact_graph(x, R=0.5):
    d = x[None, :, :] - x[:, None, :]
    d[..., 0] -= L[0] * np.round(d[..., 0] / L[0])
    d[..., 2] -= L[2] * np.round(d[..., 2] / L[2])
    d2 = (d ** 2).sum(-1)
    i, j = np.nonzero((d2 < (2 * R) ** 2) & ~np.eye(len(x), dtype=bool))
    return coo_matrix((np.ones(len(i)), (i, j)), shape=(len(x), len(x)))


@pytest.mark.parametrize("seed", range(6))
def test_random_beds_match_connected_components(orc, seed):
    rng = np.random.default_rng(seed)
    n = 120
    x = np.stack([rng.uniform(0, L[0], n), rng.uniform(0.5, 7.5, n), rng.uniform(0, L[2], n)], 1)
    # thin out to at most 12 touching partners per sphere
    keep = np.ones(n, bool)
    while True:
        A = contact_graph(x[keep]).tocsr()
        deg = np.asarray(A.sum(1)).ravel()
        if deg.max() <= 12:
            break
        keep[np.nonzero(keep)[0][deg.argmax()]] = False
    x = x[keep]
    ncomp, lab = connected_components(contact_graph(x), directed=False)
    seeded = np.zeros(ncomp, bool)
    seeded[np.unique(lab[x[:, 1] < 1.0])] = True
    ref = seeded[lab].astype(np.int32)
    assert 0 < ref.sum() < len(x)
    assert np.array_equal(flags(orc, x, use_cells=1), ref)
    assert np.array_equal(flags(orc, x, use_cells=0), ref)
