"""Training of the learned warm start (not part of the paper's method).

Samples come from the plain multi-direct forcing itself: for a sphere bed and
a fluid field, prs_forcing_samples returns every marker's features and the
forcing the plain iteration reaches after n_iter passes (times alpha dt).  A
seeded random subset of the markers is kept; the library computes the
training set's mean and standard deviation (prs_mlp_fit_norm), standardises
the samples (prs_mlp_standardize) and fits the network by Adam on the device
(prs_mlp_train_step: its own forward and backward kernels).  The random
batch indices are drawn here and the batches gathered by index (data
movement); all arithmetic on the samples runs in the library."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Iterable, Optional, Sequence

import numpy as np

from . import Context, Mlp, make_params
from . import workloads as W

N_FEAT = 12


def params_for(w: W.Workload, precision: int, n: int, **kw):
    """Library parameters of a workload (physical constants of workloads.PHYS)."""
    P = W.PHYS
    nx, ny, nz = w.grid
    d = dict(nx=nx, ny=ny, nz=nz, h=w.h, radius=0.5 * P["D"], rho_p=P["rho_p"],
             rho_f=P["rho_f"], gravity=P["g"], n_markers=w.n_markers, dt_f=P["dt_f"],
             alpha=P["alpha"], n_iter=w.n_iter, n_sub=P["n_sub"], k_n=P["k_n"], e_n=P["e_n"],
             mu=P["mu"], kt_ratio=P["kt_ratio"], dt_ratio=P["dt_ratio"], precision=precision,
             max_particles=n)
    d.update(kw)
    return make_params(**d)


@dataclass
class Samples:
    X: "object"      # torch float32 [m, 16] raw features (last 4 zero)
    T: "object"      # torch float32 [m, 3] targets (alpha dt F)
    slips: list      # relative slip histories of the plain runs


def collect(w: W.Workload, snapshots: Sequence[tuple], n_iter: int = 30, keep: float = 0.02,
            seed: int = 0, precision: int = 0, progress=None) -> Samples:
    """Samples from plain forcing on (bed seed, flow step) snapshots of w.

    keep: fraction of the markers kept per snapshot (seeded, without
    replacement)."""
    import torch

    dev = torch.device("cuda")
    dt = torch.float32 if precision == 0 else torch.float64
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    xs, ts, slips = [], [], []
    ctx = Context(params_for(w, precision, w.n))
    try:
        uhat = f = feat = target = None
        bed_seed_cur, bed, modes = None, None, None
        for k, (bed_seed, flow_step) in enumerate(snapshots):
            if bed_seed != bed_seed_cur:
                bed = W.make_bed(w, seed=bed_seed)
                modes = W.flow_modes(w, bed.bed_top, seed=bed_seed)
                bed_seed_cur = bed_seed
            uhat = W.fluid_field(w, modes, step=flow_step, device=dev, dtype=dt, out=uhat)
            if f is None:
                f = [torch.empty_like(a) for a in uhat]
            x = torch.as_tensor(bed.x, device=dev)
            u = torch.as_tensor(bed.u, device=dev)
            om = torch.as_tensor(bed.om, device=dev)
            if feat is None or feat.shape[0] != x.shape[0]:
                feat = target = None
            feat, target, st = ctx.forcing_samples(uhat, f, x, u, om, n_iter, feat, target)
            slips.append(st["rel_slip"])
            M = feat.shape[0] * feat.shape[1]
            m = max(1, int(round(keep * M)))
            idx = torch.randperm(M, generator=gen, device=dev)[:m]
            xs.append(feat.reshape(M, 16).index_select(0, idx))
            ts.append(target.reshape(M, 3).index_select(0, idx))
            if progress:
                progress(k, st)
    finally:
        ctx.close()
    return Samples(torch.cat(xs), torch.cat(ts), slips)


def fit_norm(S: Samples) -> np.ndarray:
    """Normalisation vector: feature mean/std (padding: 0/1), target mean/std,
    computed by the library (prs_mlp_fit_norm)."""
    return Mlp.fit_norm(S.X, S.T)


def train(S: Samples, iters: int = 2000, batch: int = 65536, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0, progress=None):
    """Fit a network to the samples; returns (Mlp, norm, loss history)."""
    import torch

    norm = fit_norm(S)
    net = Mlp(Mlp.init_params(seed), norm)
    Xs, Ts = net.standardize(S.X, S.T)
    gen = torch.Generator(device=Xs.device)
    gen.manual_seed(seed + 1)
    m = Xs.shape[0]
    b = min(batch, m)
    losses = []
    for it in range(iters):
        idx = torch.randint(0, m, (b,), generator=gen, device=Xs.device)
        Xb = Xs.index_select(0, idx)
        Tb = Ts.index_select(0, idx)
        want = log_every > 0 and (it % log_every == 0 or it == iters - 1)
        loss = net.train_step(Xb, Tb, lr=lr, want_loss=want)
        if want:
            losses.append((it, loss))
            if progress:
                progress(it, loss)
    return net, norm, losses


def validation_loss(net: Mlp, S: Samples, norm: np.ndarray, batch: int = 1 << 20) -> float:
    """Mean square error of the standardised prediction on held-out samples
    (the library's standardisation and loss; norm must be the network's)."""
    tot, cnt = 0.0, 0
    for a in range(0, S.X.shape[0], batch):
        Xs, Ts = net.standardize(S.X[a:a + batch].contiguous(), S.T[a:a + batch].contiguous())
        B = Xs.shape[0]
        tot += net.loss(Xs, Ts) * B
        cnt += B
    return tot / max(cnt, 1)
