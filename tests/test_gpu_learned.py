"""The learned warm start in the step, through the C ABI.

- Training samples (features and plain-forcing targets) against the oracle.
- The fused network pass: with a network whose output does not depend on its
  inputs (zero weights, bias only) both sides form the same F0 (to an FP64
  rounding), so the learned step must match the oracle step started from
  that F0 to the usual parity bounds (FP64 1e-11, FP32 1e-5).
- With a realistic network the BF16 roundings of the device (FP32
  accumulation) and of the oracle (FP64 accumulation) can fall on different
  sides of a tie for a few activations; the initial force then agrees per
  sphere to the forward pass's bound, not to 1e-11.
- The rejection rule (first slip >= 1, or growing slip) against the oracle's
  run of the same rule.
- Gain: a network trained on the GPU on one set of beds lowers the first
  relative slip and the number of iterations to a tolerance on held-out
  beds."""
import numpy as np
import pytest

from helpers import fields_for, oracle_params, prs_params, rel_err
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}
TINY = W.small("tiny", 40, 10, (4.0, 6.0, 4.0), seed=11, bed_u_std=0.1)


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


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def gpu_fields(fields64, precision):
    import torch

    dt = torch.float64 if precision == 1 else torch.float32
    return [a.to(device="cuda", dtype=dt).contiguous() for a in fields64]


def host64(fields):
    return [np.ascontiguousarray(a.detach().cpu().double().numpy()) for a in fields]


def unit_norm(tmean=(0.0, 0.0, 0.0), tstd=(1.0, 1.0, 1.0)):
    return np.concatenate([np.zeros(16), np.ones(16), tmean, tstd]).astype(np.float32)


def bias_only(b):
    p = np.zeros(6288, np.float32)
    p[6272:6275] = b
    return p


@pytest.mark.parametrize("precision", [1, 0])
def test_forcing_samples_parity(P, orc, precision):
    import torch

    w = TINY
    bed = W.make_bed(w)
    f64 = fields_for(w, bed)
    g = gpu_fields(f64, precision)
    n_iter = 5
    with P.Context(prs_params(P, w, precision)) as ctx:
        f = [torch.empty_like(a) for a in g]
        feat, target, st = ctx.forcing_samples(g, f, dev(bed.x), dev(bed.u), dev(bed.om), n_iter)
        feat, target, fg = feat.cpu().numpy(), target.cpu().numpy(), host64(f)
    p = oracle_params(orc, w, n_iter=n_iter)
    uh = host64(g)
    ref_feat = orc.learned_features(p, uh, bed.x, bed.u, bed.om)
    fo = [np.zeros_like(a) for a in uh]
    out = orc.ib_forcing(p, uh, fo, bed.x, bed.u, bed.om, want_marker_force=True)
    ref_target = p.dt_f * p.alpha * out["Fmark"]
    # features are stored in FP32: equal to FP32 rounding (FP64 path) or to
    # the FP32 interpolation error (FP32 path)
    ftol = 1e-6 if precision == 1 else 1e-5
    for a, b in ((0, 3), (3, 6), (6, 9), (9, 12)):
        assert rel_err(feat[..., a:b], ref_feat[..., a:b]) < ftol
    assert np.all(feat[..., 12:] == 0)
    # targets: n_iter FP32 additions of alpha dt dF
    assert rel_err(target, ref_target) < (1e-6 if precision == 1 else 2e-5)
    assert st["iterations"] == n_iter
    assert np.allclose(st["rel_slip"], out["slip"], rtol=10 * TOL[precision])
    for c in range(3):
        assert rel_err(fg[c], fo[c]) < TOL[precision]


def run_learned(P, w, precision, params, norm, **kw):
    import torch

    bed = W.make_bed(w)
    f64 = fields_for(w, bed)
    g = gpu_fields(f64, precision)
    x, u, om = dev(bed.x), dev(bed.u), dev(bed.om)
    net = P.Mlp(params, norm)
    with P.Context(prs_params(P, w, precision, **kw)) as ctx:
        ctx.set_learned(net)
        H = P.History.zeros(w.n)
        f = [torch.zeros_like(a) for a in g]
        Fh, Th, st = ctx.step(g, f, x, u, om, H, zero_f=True)
        gpu = dict(x=x.cpu().numpy(), u=u.cpu().numpy(), om=om.cpu().numpy(),
                   Fh=Fh.cpu().numpy(), Th=Th.cpu().numpy(), f=host64(f), st=st)
    return bed, host64(g), gpu


def oracle_step(orc, w, bed, uh, F0, **kw):
    p = oracle_params(orc, w, **kw)
    xo, uo, oo = bed.x.copy(), bed.u.copy(), bed.om.copy()
    fo = [np.zeros_like(a) for a in uh]
    rc, out = orc.step(p, uh, fo, xo, uo, oo, orc.History(w.n), F0=F0)
    assert rc == 0
    return dict(x=xo, u=uo, om=oo, Fh=out["Fh"], Th=out["Th"], f=fo, slip=out["slip"],
                iters=out["iters"])


def compare(gpu, ref, tol):
    assert rel_err(gpu["Fh"], ref["Fh"]) < tol
    assert rel_err(gpu["Th"], ref["Th"]) < tol
    for c in range(3):
        assert rel_err(gpu["f"][c], ref["f"][c]) < tol
    assert np.abs(gpu["x"] - ref["x"]).max() < tol
    assert rel_err(gpu["u"], ref["u"]) < tol
    assert rel_err(gpu["om"], ref["om"]) < tol


def constant_start(orc, w, uh, bed, scale):
    """A bias-only network: F0 = b / (alpha dt) on every marker, with b a
    fraction of the mean slip (from the oracle)."""
    p = oracle_params(orc, w)
    feat = orc.learned_features(p, uh, bed.x, bed.u, bed.om)
    b = (scale * feat[..., 0:3].reshape(-1, 3).mean(0)).astype(np.float32)
    norm = unit_norm()
    F0 = orc.learned_initial_force(bias_only(b).astype(np.float64), norm, feat, p.dt_f * p.alpha)
    return b, norm, F0


@pytest.mark.parametrize("precision", [1, 0])
def test_learned_start_parity(P, orc, precision):
    w = TINY
    bed = W.make_bed(w)
    uh = [np.ascontiguousarray(a.numpy()) for a in fields_for(w, bed)]
    if precision == 0:   # the oracle sees the FP32-rounded field the device sees
        uh = [a.astype(np.float32).astype(np.float64) for a in uh]
    b, norm, F0 = constant_start(orc, w, uh, bed, 0.5)
    ref = oracle_step(orc, w, bed, uh, F0)
    assert not orc.reject_learned(ref["slip"]), "the test's start should be accepted"
    _, _, gpu = run_learned(P, w, precision, bias_only(b), norm)
    assert gpu["st"]["rejected_learned"] == 0
    assert gpu["st"]["iterations"] == ref["iters"]
    assert np.allclose(gpu["st"]["rel_slip"], ref["slip"], rtol=10 * TOL[precision])
    compare(gpu, ref, TOL[precision])


def test_learned_start_tolerance_mode(P, orc):
    w = TINY
    bed = W.make_bed(w)
    uh = [np.ascontiguousarray(a.numpy()) for a in fields_for(w, bed)]
    b, norm, F0 = constant_start(orc, w, uh, bed, 0.5)
    kw = dict(tol_mode=1, tol=0.2, max_iter=12)
    ref = oracle_step(orc, w, bed, uh, F0, **kw)
    assert not orc.reject_learned(ref["slip"])
    _, _, gpu = run_learned(P, w, 1, bias_only(b), norm, **kw)
    assert gpu["st"]["rejected_learned"] == 0
    assert gpu["st"]["iterations"] == ref["iters"]
    assert len(gpu["st"]["rel_slip"]) == len(ref["slip"])
    compare(gpu, ref, 1e-11)


@pytest.mark.parametrize("precision", [1, 0])
def test_learned_rejection_falls_back_to_plain(P, orc, precision):
    """A start far off the forcing (huge constant force) is rejected; the step
    then equals the plain step."""
    w = TINY
    bed = W.make_bed(w)
    uh = [np.ascontiguousarray(a.numpy()) for a in fields_for(w, bed)]
    if precision == 0:
        uh = [a.astype(np.float32).astype(np.float64) for a in uh]
    b, norm, F0 = constant_start(orc, w, uh, bed, 400.0)
    bad = oracle_step(orc, w, bed, uh, F0)
    assert orc.reject_learned(bad["slip"])
    ref = oracle_step(orc, w, bed, uh, None)
    _, _, gpu = run_learned(P, w, precision, bias_only(b), norm)
    assert gpu["st"]["rejected_learned"] == 1
    assert gpu["st"]["iterations"] == ref["iters"]
    assert np.allclose(gpu["st"]["rel_slip"], ref["slip"], rtol=10 * TOL[precision])
    compare(gpu, ref, TOL[precision])


def test_learned_needs_cleared_field(P):
    import torch

    w = TINY
    bed = W.make_bed(w)
    g = gpu_fields(fields_for(w, bed), 1)
    net = P.Mlp(bias_only(np.zeros(3)), unit_norm())
    with P.Context(prs_params(P, w, P.F64)) as ctx:
        ctx.set_learned(net)
        f = [torch.zeros_like(a) for a in g]
        with pytest.raises(P.PrsError) as e:
            ctx.step(g, f, dev(bed.x), dev(bed.u), dev(bed.om), P.History.zeros(w.n),
                     zero_f=False)
        assert e.value.code == P.PRS_EINVAL


@pytest.mark.parametrize("precision", [1, 0])
def test_fused_network_matches_oracle_prediction(P, orc, precision):
    """Realistic weights, no iteration (n_iter = 0): F_h is the sum of the
    network's initial force.  Agreement to the BF16 tie bound of the forward
    pass: median per-sphere error tiny, maximum below 1e-3 of the largest.
    The single-precision pass standardises FP32 features, so its oracle gets
    the FP32-rounded field the device sees."""
    rng = np.random.default_rng(5)
    w = TINY
    bed = W.make_bed(w)
    uh = [np.ascontiguousarray(a.numpy()) for a in fields_for(w, bed)]
    if precision == 0:
        uh = [a.astype(np.float32).astype(np.float64) for a in uh]
    p = oracle_params(orc, w, n_iter=0)
    feat = orc.learned_features(p, uh, bed.x, bed.u, bed.om)
    X = feat.reshape(-1, 16)
    mean, std = X.mean(0), X.std(0)
    mean[12:], std[12:] = 0.0, 1.0
    norm = np.concatenate([mean, std, [0.0, 0.0, 0.0], [0.05, 0.05, 0.05]]).astype(np.float32)
    import paper_2108_01814_amd as PP

    params = PP.Mlp.init_params(7)
    params[1024:1088] = rng.uniform(-0.2, 0.2, 64)
    F0 = orc.learned_initial_force(params.astype(np.float64), norm, feat, p.dt_f * p.alpha)
    ref = oracle_step(orc, w, bed, uh, F0, n_iter=0)
    _, _, gpu = run_learned(P, w, precision, params, norm, n_iter=0)
    assert gpu["st"]["iterations"] == 0
    err = np.linalg.norm(gpu["Fh"] - ref["Fh"], axis=1)
    scale = np.linalg.norm(ref["Fh"], axis=1).max()
    assert np.median(err) / scale < 1e-5
    assert err.max() / scale < 1e-3


def test_trained_network_gains_on_held_out_beds(P):
    """Train on the GPU with samples of the plain method from some beds; on
    beds it has not seen the learned start must (i) lower the first relative
    slip well below one and (ii) reach a slip tolerance in fewer iterations
    than the plain start, without being rejected."""
    import torch

    from paper_2108_01814_amd import learned as L

    w = W.C1
    train_snaps = [(100 + k, k) for k in range(6)]
    S = L.collect(w, train_snaps, n_iter=30, keep=0.1, seed=0)
    net, norm, losses = L.train(S, iters=400, batch=16384, lr=2e-3, seed=0, log_every=100)
    assert losses[-1][1] < 0.5 * losses[0][1]
    held = L.collect(w, [(900, 3)], n_iter=30, keep=0.1, seed=1)
    assert L.validation_loss(net, held, norm) < 0.5
    # a step on a held-out bed, plain and learned, to the same tolerance
    bed = W.make_bed(w, seed=900)
    modes = W.flow_modes(w, bed.bed_top, seed=900)
    g = W.fluid_field(w, modes, step=3, device="cuda", dtype=torch.float32)
    res = {}
    for mode in ("plain", "learned"):
        with P.Context(L.params_for(w, P.F32, w.n, tol_mode=1, tol=0.05, max_iter=30)) as ctx:
            if mode == "learned":
                ctx.set_learned(net)
            f = [torch.zeros_like(a) for a in g]
            _, _, st = ctx.step(g, f, dev(bed.x), dev(bed.u), dev(bed.om), P.History.zeros(w.n),
                                zero_f=True)
            res[mode] = st
    assert res["learned"]["rejected_learned"] == 0
    assert res["learned"]["rel_slip"][0] < 0.5
    assert res["learned"]["iterations"] < res["plain"]["iterations"]
