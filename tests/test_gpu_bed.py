"""Bed / flying detection (sec. 4.3.1, step (1)) through the C ABI against
the oracle's detection iteration: bit-exact flags and counts on hand-built
configurations, the 512-sphere bed, and the whole 1,048,576-sphere bed."""
import numpy as np
import pytest

from helpers import prs_params
from paper_2108_01814_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def both(P, orc, w, x):
    import torch

    nx, ny, nz = w.grid
    with P.Context(prs_params(P, w, P.F64, n=max(len(x), 1))) as ctx:
        flags, nb = ctx.bed_flags(torch.as_tensor(np.ascontiguousarray(x)).cuda())
        flags = flags.cpu().numpy().astype(np.int32)
    po = orc.make_params(nx=nx, ny=ny, nz=nz, h=w.h, R=0.5 * W.PHYS["D"], nl=w.n_markers,
                         use_cells=1)
    rc, ref, nref = orc.bed_flags(po, x)
    assert rc == 0
    return flags, nb, ref, nref


SMALL = W.small("bedbox", 1, 0, (6.0, 8.0, 6.0))


@pytest.mark.parametrize("x,expect", [
    ([[3.0, 0.6 + 0.98 * k, 3.0] for k in range(6)], [1] * 6),
    ([[1.0, 0.55, 1.0], [4.0, 4.0, 4.0], [4.0, 4.95, 4.0], [4.9, 4.5, 4.0]], [1, 0, 0, 0]),
    ([[1.0, 0.999, 1.0], [3.0, 1.0, 3.0], [5.0, 1.3, 5.0], [1.0, 7.6, 5.0]], [1, 0, 0, 0]),
    ([[0.2, 0.55, 3.0], [5.4, 1.1, 3.0], [5.1, 1.95, 3.0], [5.1, 3.5, 3.0]], [1, 1, 1, 0]),
], ids=["chain", "detached", "one_diameter", "seam"])
def test_hand_built(P, orc, x, expect):
    x = np.array(x, dtype=float)
    flags, nb, ref, nref = both(P, orc, SMALL, x)
    assert flags.tolist() == expect == ref.tolist()
    assert nb == nref == sum(expect)


@pytest.mark.parametrize("w", [W.C1, W.C3], ids=["c1", "c3"])
def test_bed_flags_bit_exact(P, orc, w):
    bed = W.make_bed(w)
    print(f"{w.name}: {w.n} spheres", flush=True)
    flags, nb, ref, nref = both(P, orc, w, bed.x)
    print(f"bed spheres: device {nb}, oracle {nref}", flush=True)
    assert np.array_equal(flags, ref)
    assert nb == nref
    assert 0 < nb < w.n


def test_empty(P):
    import torch

    with P.Context(prs_params(P, SMALL, P.F64, n=4)) as ctx:
        flags, nb = ctx.bed_flags(torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    assert nb == 0 and flags.numel() == 0
