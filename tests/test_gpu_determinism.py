"""Bitwise reproducibility of the single-precision step: the spreading adds
in 32-bit fixed point (integer sums do not depend on the order of the LDS
atomics), the interpolation and every per-sphere reduction use a fixed
order, and the contact gather is atomic-free -- so two runs of the same step
from the same state agree bit for bit in every output.  (Double-precision
fields accumulate with floating-point LDS atomics, whose order varies; they
are compared with the oracle instead.)"""
import numpy as np
import pytest

from helpers import fields_for, prs_params
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    import paper_2108_01814_amd as P

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    P.lib()
    return P


def one_step(P, ctx, w, bed, g, n_steps):
    import torch

    x, u, om = (torch.as_tensor(a).cuda() for a in (bed.x, bed.u, bed.om))
    H = P.History.zeros(w.n)
    f = [torch.full_like(a, float("nan")) for a in g]
    outs = []
    for _ in range(n_steps):
        Fh, Th, st = ctx.step(g, f, x, u, om, H, zero_f=True)
    torch.cuda.synchronize()
    for a in [Fh, Th, x, u, om, H.partner, H.delta_t, H.u_in, H.count, *f]:
        outs.append(a.cpu().numpy().copy())
    return outs, st


@pytest.mark.parametrize("w", [W.C1, W.small("det4k", 3000, 600, (24.0, 12.0, 24.0), seed=31,
                                             bed_u_std=0.2)], ids=["c1", "bed3600"])
def test_fp32_step_is_bitwise_reproducible(P, w):
    import torch

    bed = W.make_bed(w)
    g = [a.to(device="cuda", dtype=torch.float32).contiguous() for a in fields_for(w, bed)]
    print(f"{w.name}: {w.n} spheres, two runs of 3 steps each", flush=True)
    with P.Context(prs_params(P, w, P.F32)) as ctx:
        a, sa = one_step(P, ctx, w, bed, g, 3)
        b, sb = one_step(P, ctx, w, bed, g, 3)
    assert sa["contacts"] > 0 and sa["rel_slip"] == sb["rel_slip"]
    for k, (x, y) in enumerate(zip(a, b)):
        assert x.tobytes() == y.tobytes(), k
