"""The phase timer through the C ABI: a step on the 512-sphere bed counts one
record pass of the spreading tiles, as many spreading passes as forcing
iterations, one interpolation per iteration, n_sub substeps, and positive
times; a second step adds to them and reset clears them."""
import pytest

from helpers import fields_for, prs_params
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_phase_counts(precision):
    import torch

    import paper_2108_01814_amd as P

    assert torch.cuda.is_available()
    w = W.C1
    bed = W.make_bed(w)
    dt = torch.float32 if precision == 0 else torch.float64
    g = [a.to(device="cuda", dtype=dt).contiguous() for a in fields_for(w, bed)]
    with P.Context(prs_params(P, w, precision)) as ctx:
        x = torch.as_tensor(bed.x, device="cuda")
        u = torch.as_tensor(bed.u, device="cuda")
        om = torch.as_tensor(bed.om, device="cuda")
        H = P.History.zeros(w.n)
        f = [torch.zeros_like(a) for a in g]
        ctx.timing(True)
        ctx.read_timing(reset=True)
        _, _, st = ctx.step(g, f, x, u, om, H, zero_f=True)
        t = ctx.read_timing(reset=False)
        it = st["iterations"]
        assert it == w.n_iter
        assert t["steps"] == 1 and t["n_record"] == 1 and t["n_spread"] == it
        assert t["n_interp"] == it and t["n_substep"] == W.PHYS["n_sub"]
        for k in ("ms_record", "ms_spread", "ms_interp", "ms_substep"):
            assert t[k] > 0, k
        ctx.step(g, f, x, u, om, H, zero_f=True)
        t2 = ctx.read_timing(reset=True)
        assert t2["steps"] == 2 and t2["n_record"] == 2 and t2["n_spread"] == 2 * it
        assert ctx.read_timing(reset=True)["n_spread"] == 0
