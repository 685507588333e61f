"""Pins of the oracle's learned-warm-start network (no GPU): BF16 rounding on
known values, analytic gradient vs central finite differences, the loss at
zero weights, and Adam's first steps in closed form."""
import math

import numpy as np
import pytest

RNG = np.random.default_rng(99)


def random_params(orc, scale=0.3):
    d = {}
    for k, s in orc.MLP_SHAPES:
        fan_in = s[1] if len(s) == 2 else 64
        d[k] = RNG.uniform(-1, 1, size=s) * (scale if k.startswith("b") else 1 / math.sqrt(fan_in))
    d["W1"][:, 12:] = 0.0
    return orc.mlp_pack(d)


def batch(n=8):
    X = np.zeros((n, 16))
    X[:, :12] = RNG.normal(size=(n, 12))
    T = RNG.normal(size=(n, 3))
    return X, T


@pytest.mark.parametrize("x,expect", [
    (1.0, 1.0), (-2.5, -2.5), (0.0, 0.0),
    (1.0 + 2 ** -8, 1.0),                    # tie -> even (1.0)
    (1.0 + 3 * 2 ** -8, 1.0 + 2 ** -6),      # tie -> even (upper)
    (1.0 + 2 ** -8 + 2 ** -20, 1.0 + 2 ** -7),
    (3.140625, 3.140625), (1e-3, 0.00099945068359375),
])
def test_bf16_rounding_known_values(orc, x, expect):
    assert orc.bf16(x) == expect


def test_gradient_matches_finite_differences(orc):
    P = random_params(orc)
    X, T = batch(6)
    loss, g = orc.mlp_loss_grad(P, X, T, emulate_bf16=False)
    idx = np.concatenate([RNG.choice(P.size, 60, replace=False),
                          [0, 15, 1024 + 3, 1088 + 100, 5184 + 2, 6272 + 1, 6272 + 7]])
    for i in idx:
        hstep = 1e-6 * max(1.0, abs(P[i]))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += hstep
        Pm[i] -= hstep
        lp, _ = orc.mlp_loss_grad(Pp, X, T, emulate_bf16=False)
        lm, _ = orc.mlp_loss_grad(Pm, X, T, emulate_bf16=False)
        fd = (lp - lm) / (2 * hstep)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_padding_outputs_and_inputs_get_no_gradient(orc):
    P = random_params(orc)
    X, T = batch(5)
    _, g = orc.mlp_loss_grad(P, X, T)
    d = orc.mlp_unpack(g)
    assert np.all(d["W3"][3:] == 0) and np.all(d["b3"][3:] == 0)
    assert np.all(d["W1"][:, 12:] == 0)


def test_zero_network_loss_is_mean_square_target(orc):
    P = np.zeros(orc.mlp_nparam())
    X, T = batch(10)
    loss, g = orc.mlp_loss_grad(P, X, T)
    assert loss == pytest.approx((T ** 2).mean(), rel=1e-14)
    d = orc.mlp_unpack(g)
    assert np.allclose(d["b3"][:3], -2 * T.mean(0) / 3, rtol=1e-12)


def test_forward_matches_loss_path(orc):
    P = random_params(orc)
    X, T = batch(7)
    Y = orc.mlp_forward(P, X)
    loss, _ = orc.mlp_loss_grad(P, X, T)
    assert loss == pytest.approx(((Y[:, :3] - T) ** 2).mean(), rel=1e-13)


def test_bf16_emulation_changes_little(orc):
    P = random_params(orc)
    X, T = batch(32)
    Ya = orc.mlp_forward(P, X, emulate_bf16=True)
    Yb = orc.mlp_forward(P, X, emulate_bf16=False)
    rel = np.abs(Ya - Yb).max() / np.abs(Yb).max()
    assert 1e-5 < rel < 3e-2


def test_adam_first_steps_closed_form(orc):
    n = 5
    P = np.zeros(n)
    m = np.zeros(n)
    v = np.zeros(n)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -4.0])
    lr = 1e-3
    orc.mlp_adam(P, m, v, g, 1, lr=lr)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> lr * g / (|g| + eps)
    assert np.allclose(P, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    orc.mlp_adam(P, m, v, g, 2, lr=lr)
    # constant gradient: m_hat = g, v_hat = g^2 again
    assert np.allclose(P, -2 * lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
