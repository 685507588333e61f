"""Parity of the learned warm-start network on MFMA with the FP64 oracle that
rounds the same values to BF16 (forward, backward, Adam), the training-set
statistics and standardisation, and a training sanity check.

Two kinds of input:
- the dyadic network of mlp_cases, on which every value the network rounds
  to BF16 is exact in FP32 on both sides, so the rounding decisions agree and
  the only difference is FP32 against FP64 accumulation: forward, gradient
  and Adam step within 1e-5;
- seeded random networks, where a BF16 rounding of an activation computed in
  FP32 (device) or FP64 (oracle) can land on the other side of a tie: the
  gradient over a batch of 65,536 within 1e-5 in norm, and looser element
  maxima as tie bounds."""
import numpy as np
import pytest

import mlp_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    import paper_2108_01814_amd as P

    assert torch.cuda.is_available()
    P.lib()
    return P


@pytest.fixture(scope="module")
def orc():
    import oracle

    oracle.lib()
    return oracle


def setup(P, seed=3, B=1000):
    import torch

    rng = np.random.default_rng(seed)
    params = P.Mlp.init_params(seed)
    params[1024:1088] = rng.uniform(-0.2, 0.2, 64)        # b1
    params[5184:5248] = rng.uniform(-0.2, 0.2, 64)        # b2
    params[6272:6275] = rng.uniform(-0.2, 0.2, 3)         # b3
    norm = np.concatenate([np.zeros(16), np.ones(16), np.zeros(3), np.ones(3)]).astype(np.float32)
    X = np.zeros((B, 16), np.float32)
    X[:, :12] = rng.normal(size=(B, 12))
    T = rng.normal(size=(B, 3)).astype(np.float32)
    net = P.Mlp(params, norm)
    return net, params, norm, X, T, torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()


def test_forward_parity(P, orc):
    net, params, norm, X, T, Xd, Td = setup(P, B=1003)
    Y = net.forward(Xd, raw=False).cpu().numpy()
    ref = orc.mlp_forward(params.astype(np.float64), X.astype(np.float64))[:, :3]
    err = np.abs(Y - ref)
    assert np.median(err) / np.abs(ref).max() < 1e-5
    assert err.max() / np.abs(ref).max() < 2e-2


def test_forward_raw_units(P):
    import torch

    net, params, _, X, T, Xd, Td = setup(P, B=64)
    mean = np.linspace(-1, 1, 16).astype(np.float32)
    std = np.linspace(0.5, 2, 16).astype(np.float32)
    tmean = np.array([0.1, -0.2, 0.3], np.float32)
    tstd = np.array([2.0, 0.5, 1.5], np.float32)
    norm = np.concatenate([mean, std, tmean, tstd])
    net2 = P.Mlp(params, norm)
    raw = X * std + mean
    Y_raw = net2.forward(torch.as_tensor(raw).cuda(), raw=True).cpu().numpy()
    Y_std = net2.forward(Xd, raw=False).cpu().numpy()
    assert np.allclose(Y_raw, Y_std * tstd + tmean, rtol=1e-3, atol=1e-3)


def test_gradient_parity(P, orc):
    net, params, norm, X, T, Xd, Td = setup(P, B=4000)
    g, loss = net.grad(Xd, Td)
    lo, go = orc.mlp_loss_grad(params.astype(np.float64), X.astype(np.float64),
                               T.astype(np.float64))
    g = g.cpu().numpy()
    assert loss == pytest.approx(lo, rel=1e-4)
    assert np.abs(g - go).max() / np.abs(go).max() < 2e-3
    assert np.linalg.norm(g - go) / np.linalg.norm(go) < 1e-3
    # padding rows and columns get exactly zero gradient
    d = orc.mlp_unpack(g)
    assert np.all(d["W3"][3:] == 0) and np.all(d["b3"][3:] == 0) and np.all(d["W1"][:, 12:] == 0)


def test_adam_step_parity(P, orc):
    net, params, norm, X, T, Xd, Td = setup(P, B=512)
    _, go = orc.mlp_loss_grad(params.astype(np.float64), X.astype(np.float64),
                              T.astype(np.float64))
    net.train_step(Xd, Td, lr=1e-3)
    got, _ = net.get()
    ref = params.astype(np.float64).copy()
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    orc.mlp_adam(ref, m, v, go, 1, lr=1e-3)
    # the first Adam step moves each weight by lr * g / (|g| + eps) ~ lr sign(g);
    # compare where the gradient is clearly away from zero (its sign is robust)
    moved = np.abs(go) > 1e-3 * np.abs(go).max()
    assert moved.sum() > 3000
    assert np.abs(got - ref)[moved].max() < 2e-5
    assert np.array_equal(got[6275:], params[6275:])      # padding outputs untouched


def test_training_reduces_loss(P):
    """A smooth synthetic regression is learned (loss drops by 10x)."""
    import torch

    rng = np.random.default_rng(11)
    B = 8192
    X = np.zeros((B, 16), np.float32)
    X[:, :12] = rng.normal(size=(B, 12))
    A = rng.normal(size=(12, 3)) / 4
    T = (np.tanh(X[:, :12] @ A) * 2).astype(np.float32)
    T = (T - T.mean(0)) / T.std(0)
    norm = np.concatenate([np.zeros(16), np.ones(16), np.zeros(3), np.ones(3)]).astype(np.float32)
    net = P.Mlp(P.Mlp.init_params(1), norm)
    Xd, Td = torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()
    first = net.train_step(Xd, Td, lr=3e-3)
    for _ in range(300):
        last = net.train_step(Xd, Td, lr=3e-3, want_loss=False)
    last = net.train_step(Xd, Td, lr=3e-3)
    assert last < first / 10


def dyadic_setup(P, orc, seed=3, B=4096):
    import torch

    params, X = mlp_cases.dyadic_network(seed, B=B)
    Y = orc.mlp_forward(params, X)
    T = mlp_cases.dyadic_targets(seed, Y)
    norm = np.concatenate([np.zeros(16), np.ones(16), np.zeros(3), np.ones(3)]).astype(np.float32)
    p32 = params.astype(np.float32)
    assert np.array_equal(p32.astype(np.float64), params)     # exact in FP32
    net = P.Mlp(p32, norm)
    Xd = torch.as_tensor(X.astype(np.float32)).cuda()
    Td = torch.as_tensor(T.astype(np.float32)).cuda()
    assert np.array_equal(T.astype(np.float32).astype(np.float64), T)
    return net, params, X, T, Y, Xd, Td


def test_dyadic_forward_parity(P, orc):
    net, params, X, T, Y, Xd, Td = dyadic_setup(P, orc)
    got = net.forward(Xd, raw=False).cpu().numpy().astype(np.float64)
    assert np.abs(got - Y[:, :3]).max() <= 1e-5 * np.abs(Y[:, :3]).max()


def test_dyadic_gradient_parity(P, orc):
    net, params, X, T, Y, Xd, Td = dyadic_setup(P, orc)
    g, loss = net.grad(Xd, Td)
    lo, go = orc.mlp_loss_grad(params, X, T)
    g = g.cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(lo, rel=1e-5)
    assert np.abs(g - go).max() <= 1e-5 * np.abs(go).max()
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)
    # the forward-only loss agrees with the backward pass's
    assert net.loss(Xd, Td) == pytest.approx(lo, rel=1e-5)


def test_dyadic_adam_parity(P, orc):
    """Adam's arithmetic on the same gradient: the device's step from its
    gradient against the oracle's step from that gradient (a gradient entry
    that cancels to ~1e-8 over the batch differs between FP32 and FP64
    accumulation by a relative 1e-4, which Adam's g / (|g| + eps) would
    magnify; the gradient itself is compared above)."""
    net, params, X, T, Y, Xd, Td = dyadic_setup(P, orc)
    ref = params.copy()
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    lr = 1e-3
    g, _ = net.grad(Xd, Td)
    net.adam(g, lr=lr)                       # explicit gradient
    orc.mlp_adam(ref, m, v, g.cpu().numpy().astype(np.float64), 1, lr=lr)
    got, _ = net.get()
    # within 1e-5 of the step, plus the FP32 rounding of the stored weight
    # (the biases of 8 and 12 have an FP32 spacing near 1e-6)
    room = 1e-5 * lr + 0.5 * np.spacing(np.abs(params).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got - ref) <= room)
    # a step from the kept gradient of the latest backward equals the step
    # from that gradient passed explicitly (bitwise), on a second network
    twin = P.Mlp(params.astype(np.float32), np.concatenate(
        [np.zeros(16), np.ones(16), np.zeros(3), np.ones(3)]).astype(np.float32))
    g2, _ = twin.grad(Xd, Td)
    twin.adam(g2, lr=lr)
    net2 = P.Mlp(params.astype(np.float32), np.concatenate(
        [np.zeros(16), np.ones(16), np.zeros(3), np.ones(3)]).astype(np.float32))
    net2.grad(Xd, Td)
    net2.adam(lr=lr)
    assert np.array_equal(net2.get()[0], twin.get()[0])


def test_gradient_parity_large_batch(P, orc):
    """Random weights, batch 65,536: BF16 ties may round differently on a few
    activations, but over the batch the gradient agrees within 1e-5 in norm."""
    net, params, norm, X, T, Xd, Td = setup(P, seed=8, B=65536)
    g, loss = net.grad(Xd, Td)
    lo, go = orc.mlp_loss_grad(params.astype(np.float64), X.astype(np.float64),
                               T.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(lo, rel=1e-5)
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)
    assert np.abs(g - go).max() <= 1e-4 * np.abs(go).max()


def test_statistics_and_standardisation(P):
    import torch

    rng = np.random.default_rng(21)
    m = 100003
    X = np.zeros((m, 16), np.float32)
    X[:, :12] = rng.normal(size=(m, 12)) * rng.uniform(0.1, 5, 12) + rng.normal(size=12)
    X[:, 7] = 2.5                                          # a constant feature
    T = (rng.normal(size=(m, 3)) * [0.01, 1.0, 30.0] + [1.0, -2.0, 0.5]).astype(np.float32)
    Xd, Td = torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()
    norm = P.Mlp.fit_norm(Xd, Td)
    X64, T64 = X.astype(np.float64), T.astype(np.float64)
    mean, std = X64.mean(0), X64.std(0, ddof=1)
    mean[12:], std[12:] = 0.0, 1.0
    std[7] = 1.0
    ref = np.concatenate([mean, std, T64.mean(0), T64.std(0, ddof=1)])
    assert np.allclose(norm, ref, rtol=2e-7, atol=1e-12)
    net = P.Mlp(P.Mlp.init_params(0), norm)
    Xs, Ts = net.standardize(Xd, Td)
    n64 = norm.astype(np.float64)
    assert np.allclose(Xs.cpu().numpy(), (X64 - n64[:16]) / n64[16:32], rtol=1e-6, atol=1e-6)
    assert np.allclose(Ts.cpu().numpy(), (T64 - n64[32:35]) / n64[35:38], rtol=1e-6, atol=1e-6)
