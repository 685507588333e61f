"""The C-ABI library on the host (no GPU): it loads, exports every symbol the
header declares, and rejects bad arguments before any device work."""
import ctypes as C
import os
import re

import pytest

import paper_2108_01814_amd as P
from paper_2108_01814_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "prs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(prs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for need in ("prs_step_particles", "prs_interpolate", "prs_spread", "prs_contacts",
                 "prs_create", "prs_destroy", "prs_template", "prs_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(P.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(declared_symbols()) == set(P.EXPORTS)


def test_params_struct_matches_header_size():
    """The ctypes mirror has the field order of prs_params (checked by offsets
    of a few fields against a layout computed from the header's order)."""
    p = P.make_params(nx=8, ny=9, nz=10)
    assert (p.nx, p.ny, p.nz) == (8, 9, 10)
    assert P.Params.h.offset == 16 and P.Params.radius.offset == 24
    assert P.Params.max_particles.offset > P.Params.precision.offset
    assert P.Params.contact_model.offset > P.Params.max_particles.offset
    assert P.Params.e_t.offset == P.Params.t_c.offset + 8


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(h=0.0), dict(radius=-1.0), dict(n_markers=0), dict(n_markers=2000),
    dict(e_n=0.0), dict(e_n=1.5), dict(kt_ratio=0.0), dict(precision=3), dict(max_iter=64),
    dict(tol_mode=2), dict(skin=-0.1), dict(nx=2),   # periodic box shorter than three cells
    dict(mu=-1.0), dict(dt_f=0.0), dict(gravity=(0.0, float("nan"), 0.0)),
    dict(contact_model=2), dict(contact_model=1, t_c=0.0), dict(contact_model=1, e_t=0.0),
    dict(contact_model=1, e_t=1.5), dict(nx=30),    # too narrow for a spreading tile's image
])
def test_create_rejects_bad_parameters(bad):
    kw = dict(nx=80, ny=100, nz=80, max_particles=10)
    kw.update(bad)
    p = P.make_params(**kw)
    h = C.c_void_p()
    rc = P.lib().prs_create(C.byref(p), C.byref(h))
    assert rc == P.PRS_EINVAL
    assert not h.value


def test_null_context_is_rejected():
    L = P.lib()
    assert L.prs_last_error(None) == b"null context"
    assert L.prs_template(None, None, None) == P.PRS_EINVAL
    assert L.prs_interpolate(None, None, None, None, None, None, None, None, 0, None, None) == P.PRS_EINVAL
    assert L.prs_spread(None, None, None, 0, None, None, None, None, 0) == P.PRS_EINVAL
    n = C.c_int64()
    assert L.prs_contacts(None, None, None, 0, None, 0, C.byref(n)) == P.PRS_EINVAL


def test_history_capacity_is_linear_in_particles():
    """The fixed-capacity history of sec. 3.4: 14 slots per sphere (12 spheres
    + 2 walls), not a table over all pairs."""
    n = W.C3.n
    per_sphere = P.SLOTS * (4 + 3 * 8 + 8) + 1     # partner, delta_t, u_in, count
    assert P.SLOTS == P.MAX_PP + 2 == 14
    assert per_sphere == 505
    assert n * per_sphere < 0.6e9                    # ~0.53 GB for a million spheres
    naive = n * n * (3 * 8 + 8)                      # delta_t and u_in for every pair
    assert naive / (n * per_sphere) > 1e4
