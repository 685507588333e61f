"""The bound behind the fixed-point spreading (no GPU): at any grid node, the
stencil weights of one sphere's markers sum to at most

    (2/3)^3 * min(N_L, ceil(1.5 * A / (4 pi R^2 / N_L)) + 4),
    A = 2 pi R (R - sqrt(R^2 - rho^2)),  rho = 1.5 sqrt(3) h,

the product of the largest 3-point kernel value per axis and a count of the
markers that can lie within reach of one node (the cap of the sphere inside a
ball of radius rho, with a factor 1.5 for the Fibonacci points' departure
from uniform and 4 for the cap's rim).  The weight sums are computed by brute
force from the oracle's template and the 3-point kernel's closed form, for
several marker counts and sub-grid offsets of the centre.  (The bound is
loose -- about 15x the largest sums found, 0.74 at D/h = 10 with 314
markers -- which costs the fixed point about 4 of its 30 bits; it only has
to be safe.)"""
import math

import numpy as np
import pytest


def phi(r):
    r = np.abs(r)
    out = np.zeros_like(r)
    a = r <= 0.5
    out[a] = (1.0 + np.sqrt(1.0 - 3.0 * r[a] ** 2)) / 3.0
    b = (r > 0.5) & (r <= 1.5)
    out[b] = (5.0 - 3.0 * r[b] - np.sqrt(np.maximum(1.0 - 3.0 * (1.0 - r[b]) ** 2, 0.0))) / 6.0
    return out


def bound(nl, R, h):
    rho = 1.5 * math.sqrt(3.0) * h
    area = 2 * math.pi * R * (R - math.sqrt(R * R - rho * rho)) if rho < R else 4 * math.pi * R * R
    per_marker = 4 * math.pi * R * R / nl
    return (8.0 / 27.0) * min(nl, math.ceil(1.5 * area / per_marker) + 4)


@pytest.mark.parametrize("d_over_h,nl", [(10, 314), (16, 804), (12, 452), (10, 1024), (10, 64),
                                         (6, 113)])
def test_weight_sum_bound(orc, d_over_h, nl):
    h = 1.0 / d_over_h
    R = 0.5
    t, _ = orc.template(nl, R, h)
    rng = np.random.default_rng(nl)
    worst = 0.0
    for _ in range(6):
        c = rng.uniform(0, h, 3) + 2.0          # centre at a random sub-grid offset
        X = c + R * t                           # markers [nl, 3]
        # nodes (node centres at integer multiples of h; a staggering only
        # shifts the node lattice, which the random offset already covers)
        lo = np.floor((c - R) / h).astype(int) - 2
        hi = np.ceil((c + R) / h).astype(int) + 2
        axes = [np.arange(lo[a], hi[a] + 1) * h for a in range(3)]
        # separable weights: w[m, i] per axis
        w = [phi((X[:, a][:, None] - axes[a][None, :]) / h) for a in range(3)]
        # sum over markers of the product, for every node
        s = np.einsum("mi,mj,mk->ijk", w[0], w[1], w[2], optimize=True)
        worst = max(worst, float(s.max()))
    b = bound(nl, R, h)
    print(f"D/h {d_over_h}, {nl} markers: largest weight sum {worst:.3f}, bound {b:.3f}")
    assert worst <= b
