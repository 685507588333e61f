"""Pins of the oracle's learned-warm-start helpers (no GPU).

- features: closed form for affine fields (the interpolation reproduces them
  exactly away from walls), zero slip for a rigid motion of the sphere;
- initial force: closed form for a bias-only network (independent of the
  features) and for a single-path network whose every BF16 rounding point is
  written out by hand, which fixes the index of each standardisation
  statistic and where the forward pass rounds;
- gradient: the same single-path network, its gradient written out by hand
  with the rounding of the back-propagated errors, which fixes where the
  backward pass rounds;
- the premise of the dyadic network of mlp_cases (saturated hidden units,
  exact layer sums), on which the GPU parity tests need no tie allowance;
- the rejection rule on hand-written slip sequences.

The network is not part of the paper; these pin the library's own definition
of it."""
import math

import numpy as np
import pytest

import mlp_cases

RNG = np.random.default_rng(2024)
H = 0.1
R = 0.5


def bf16(x):
    """Round to the nearest BF16 value (ties to even), through FP32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + math.erf(z / math.sqrt(2.0))) + z * math.exp(-0.5 * z * z) / math.sqrt(
        2.0 * math.pi)


def staggered_affine(p, a, B):
    """The field a_c + B_c . x sampled at the staggered nodes of component c."""
    out = []
    for c in range(3):
        nyc = p.ny + (1 if c == 1 else 0)
        k, j, i = np.meshgrid(np.arange(p.nz), np.arange(nyc), np.arange(p.nx), indexing="ij")
        o = [0.5, 0.5, 0.5]
        o[c] = 0.0
        X = (i + o[0]) * H
        Y = (j + o[1]) * H
        Z = (k + o[2]) * H
        out.append(np.ascontiguousarray(a[c] + B[c, 0] * X + B[c, 1] * Y + B[c, 2] * Z))
    return out


def fib(nl):
    l = np.arange(nl)
    zp = 1.0 - (2.0 * l + 1.0) / nl
    rho = np.sqrt(1.0 - zp * zp)
    th = l * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(th), zp, rho * np.sin(th)], 1)


def test_features_of_affine_field_in_closed_form(orc):
    nl = 50
    p = orc.make_params(nx=40, ny=40, nz=40, h=H, nl=nl)
    a = RNG.normal(size=3)
    Bm = RNG.normal(size=(3, 3))
    uh = staggered_affine(p, a, Bm)
    x = np.array([[2.03, 1.97, 2.11], [1.21, 2.4, 2.83]])
    up = RNG.normal(size=(2, 3))
    om = RNG.normal(size=(2, 3))
    F = orc.learned_features(p, uh, x, up, om)
    t = fib(nl)
    for s in range(2):
        r = R * t
        X = x[s] + r
        Ud = up[s] + np.cross(om[s], r)
        slip = Ud - (a + X @ Bm.T)
        assert np.abs(F[s, :, 0:3] - slip).max() < 1e-12
        assert np.abs(F[s, :, 3:6] - t).max() < 1e-13   # libm vs numpy cos, sin
        assert np.array_equal(F[s, :, 6:9], np.broadcast_to(up[s], (nl, 3)))
        assert np.abs(F[s, :, 9:12] - R * om[s]).max() == 0.0
        assert np.all(F[s, :, 12:] == 0.0)


def test_rigid_motion_has_zero_slip(orc):
    p = orc.make_params(nx=40, ny=40, nz=40, h=H, nl=80)
    xc = np.array([[2.0, 2.05, 1.95]])
    U = RNG.normal(size=3)
    Om = RNG.normal(size=3)
    # u(x) = U + Om x (x - xc): a = U - Om x xc, B = [Om]_x
    Bm = np.array([[0, -Om[2], Om[1]], [Om[2], 0, -Om[0]], [-Om[1], Om[0], 0]])
    uh = staggered_affine(p, U - Bm @ xc[0], Bm)
    F = orc.learned_features(p, uh, xc, U[None], Om[None])
    assert np.abs(F[..., 0:3]).max() < 1e-12


def norm_vec(mean, std, tmean, tstd):
    return np.concatenate([mean, std, tmean, tstd])


def test_initial_force_of_bias_only_network(orc):
    nparam = orc.mlp_nparam()
    P = np.zeros(nparam)
    b = np.array([0.3, -1.2, 2.5])
    P[6272:6275] = b
    mean, std = RNG.normal(size=16), RNG.uniform(0.5, 2.0, 16)
    tmean, tstd = np.array([0.1, -0.7, 0.4]), np.array([0.9, 2.5, 0.3])
    adt = 8.27944e-4
    feat = RNG.normal(size=(3, 7, 16))
    F0 = orc.learned_initial_force(P, norm_vec(mean, std, tmean, tstd), feat, adt)
    ref = (b * tstd + tmean) / adt
    assert F0.shape == (3, 7, 3)
    assert np.abs(F0 - ref).max() <= 1e-15 * np.abs(ref).max()


def single_path(k0=5, i0=17, j0=40, o0=1):
    P = np.zeros(6288)
    vals = dict(w1=0.7071, c1=0.13, w2=-1.3137, c2=0.37, w3=0.91723, c3=-0.211)
    P[0 + i0 * 16 + k0] = vals["w1"]
    P[1024 + i0] = vals["c1"]
    P[1088 + j0 * 64 + i0] = vals["w2"]
    P[5184 + j0] = vals["c2"]
    P[5248 + o0 * 64 + j0] = vals["w3"]
    P[6272 + o0] = vals["c3"]
    return P, vals, (k0, i0, j0, o0)


def test_initial_force_of_single_path_network(orc):
    """Feature k0 -> hidden i0 -> hidden j0 -> output o0, every rounding of the
    forward pass written out: the standardised input, each weight and each
    activation are rounded to BF16; biases and sums are exact."""
    P, v, (k0, i0, j0, o0) = single_path()
    mean, std = RNG.normal(size=16), RNG.uniform(0.5, 2.0, 16)
    tmean, tstd = np.array([0.1, -0.7, 0.4]), np.array([0.9, 2.5, 0.3])
    adt = 8.27944e-4
    feat = RNG.normal(size=(11, 16)) * 2.0
    F0 = orc.learned_initial_force(P, norm_vec(mean, std, tmean, tstd), feat, adt)
    for m in range(feat.shape[0]):
        xs = bf16((feat[m, k0] - mean[k0]) / std[k0])
        a1 = bf16(gelu(bf16(v["w1"]) * xs + v["c1"]))
        a2 = bf16(gelu(bf16(v["w2"]) * a1 + v["c2"]))
        y = bf16(v["w3"]) * a2 + v["c3"]
        ref = tmean / adt
        ref[o0] = (y * tstd[o0] + tmean[o0]) / adt
        assert np.abs(F0[m] - ref).max() <= 1e-13 * np.abs(ref).max(), m
    # the rounding points matter here: without them the prediction moves
    Y_plain = orc.mlp_forward(P, (feat - mean) / std, emulate_bf16=False)[:, o0]
    Y_emu = orc.mlp_forward(P, (feat - mean) / std, emulate_bf16=True)[:, o0]
    assert np.abs(Y_plain - Y_emu).max() > 1e-4


def test_gradient_of_single_path_network(orc):
    """The gradient of the single-path network with the rounding of the
    back-propagated errors written out: dy, dz2 and dz1 enter the weight
    gradients and the next layer's product rounded to BF16, the bias
    gradients take them unrounded."""
    P, v, (k0, i0, j0, o0) = single_path()
    B = 3
    X = np.zeros((B, 16))
    X[:, :12] = RNG.normal(size=(B, 12))
    T = RNG.normal(size=(B, 3))
    loss, g = orc.mlp_loss_grad(P, X, T, emulate_bf16=True)
    d = {k: np.zeros(s) for k, s in mlp_cases.SHAPES}
    lsum = 0.0
    w1, w2, w3 = bf16(v["w1"]), bf16(v["w2"]), bf16(v["w3"])
    for b in range(B):
        xb = bf16(X[b])
        z1 = w1 * xb[k0] + v["c1"]
        a1 = bf16(gelu(z1))
        z2 = w2 * a1 + v["c2"]
        a2 = bf16(gelu(z2))
        y = np.zeros(3)
        y[o0] = w3 * a2 + v["c3"]
        e = y - T[b]
        lsum += (e ** 2).sum()
        dy = 2.0 * e / (3.0 * B)
        dyb = bf16(dy)
        d["W3"][:3, j0] += dyb * a2
        d["b3"][:3] += dy
        dz2 = w3 * dyb[o0] * gelu_d(z2)
        d["W2"][j0, i0] += bf16(dz2) * a1
        d["b2"][j0] += dz2
        dz1 = w2 * bf16(dz2) * gelu_d(z1)
        d["W1"][i0, :] += bf16(dz1) * xb
        d["b1"][i0] += dz1
    ref = mlp_cases.pack(d)
    assert loss == pytest.approx(lsum / (3 * B), rel=1e-14)
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()
    # the hidden units that carry nothing get exactly zero gradient
    assert np.count_nonzero(g) == np.count_nonzero(ref)


def test_dyadic_case_saturates_every_hidden_unit():
    """The premise of the dyadic network used by the GPU parity tests: every
    hidden pre-activation is at least 6 away from zero (GELU is the identity
    or below 1e-8 there, in single precision), the layer sums are dyadic
    rationals small enough to be exact in FP32, and the targets sit 3 d off
    the outputs with d a multiple of 1/8."""
    P, X = mlp_cases.dyadic_network(3, B=512)
    d = {}
    o = 0
    for k, s in mlp_cases.SHAPES:
        n = int(np.prod(s))
        d[k] = P[o:o + n].reshape(s)
        o += n
    z1 = X @ d["W1"].T + d["b1"]
    assert np.abs(z1).min() >= 6.0
    a1 = np.where(z1 > 0, bf16(z1), 0.0)
    z2 = a1 @ d["W2"].T + d["b2"]
    assert np.abs(z2).min() >= 6.0
    for v, q in ((z1, 64), (z2, 4096)):   # exact multiples of 1/q, < 2^24 / q
        assert np.array_equal(v * q, np.round(v * q)) and np.abs(v).max() * q < 2 ** 24
    Y = np.zeros((X.shape[0], 16))
    Y[:, :3] = np.where(z2 > 0, bf16(z2), 0.0) @ d["W3"][:3].T + d["b3"][:3]
    T = mlp_cases.dyadic_targets(3, Y)
    dd = (Y[:, :3] - T) / 3.0
    assert np.array_equal(dd * 8, np.round(dd * 8))


@pytest.mark.parametrize("slips,reject", [
    ([], False),
    ([0.5], False),
    ([0.5, 0.3, 0.2], False),
    ([0.5, 0.5, 0.4], False),        # equal is not growth
    ([1.0], True),                    # no better than zero forcing
    ([1.2, 0.5], True),
    ([0.4, 0.41], True),              # growth between consecutive passes
    ([0.4, 0.2, 0.1, 0.11], True),
    ([float("nan")], True),
])
def test_rejection_rule(orc, slips, reject):
    assert orc.reject_learned(slips) is reject
