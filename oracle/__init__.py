"""ctypes binding of the plain FP64 CPU oracle (``prs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  The oracle
shares no code with the HIP path; see ``prs_oracle.c`` for what each function
computes and which passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "prs_oracle.c"), os.path.join(_HERE, "mlp_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

SLOTS = 14
OK, EINVAL, ECAPACITY, EDOMAIN, ENONFINITE = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
        ("wi0", C.c_int32), ("wnx", C.c_int32), ("wk0", C.c_int32), ("wnz", C.c_int32),
        ("R", C.c_double), ("rho_p", C.c_double), ("rho_f", C.c_double), ("g", C.c_double * 3),
        ("nl", C.c_int32),
        ("dt_f", C.c_double), ("alpha", C.c_double),
        ("n_iter", C.c_int32), ("tol_mode", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
        ("n_sub", C.c_int32), ("k_n", C.c_double), ("e_n", C.c_double), ("mu", C.c_double),
        ("kt_ratio", C.c_double), ("dt_ratio", C.c_double),
        ("use_cells", C.c_int32),
        ("contact_model", C.c_int32), ("t_c", C.c_double), ("e_t", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER(Params)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.or_template.argtypes = [C.c_int32, C.c_double, C.c_double, dp, dp]
        L.or_phi.argtypes = [C.c_double]
        L.or_phi.restype = C.c_double
        L.or_interpolate.argtypes = [P, dp, dp, dp, C.c_int32, dp, dp, dp, dp, dp]
        L.or_spread.argtypes = [P, C.c_int32, dp, dp, dp, dp, dp]
        L.or_ib_forcing.argtypes = [P, dp, dp, dp, dp, dp, dp, C.c_int32, dp, dp, dp, dp, dp, dp,
                                    dp, ip, dp, dp, dp, dp]
        L.or_contacts.argtypes = [P, C.c_int32, dp, ip, C.c_int64, C.POINTER(C.c_int64)]
        L.or_bed_flags.argtypes = [P, C.c_int32, dp, ip, C.POINTER(C.c_int64)]
        L.or_inner_fluid.argtypes = [P, dp, dp, dp, C.c_int32, dp, dp]
        L.or_step_ex.argtypes = [P, C.c_double, C.c_int, dp, dp, dp, dp, dp, dp, C.c_int32, dp,
                                 dp, dp, dp, ip, dp, dp, ip, dp, dp, dp, ip, dp, dp]
        L.or_history_match.argtypes = [C.c_int32, ip, C.c_int32, ip, ip]
        L.or_history_match.restype = None
        L.or_dem.argtypes = [P, C.c_int32, dp, dp, dp, dp, dp, ip, dp, dp, ip, dp, dp]
        L.or_step.argtypes = [P, dp, dp, dp, dp, dp, dp, C.c_int32, dp, dp, dp, dp, ip, dp, dp, ip,
                              dp, dp, dp, ip]
        L.or_mlp_nparam.restype = C.c_int
        L.or_bf16.argtypes = [C.c_double]
        L.or_bf16.restype = C.c_double
        L.or_mlp_forward.argtypes = [dp, C.c_int32, dp, dp, C.c_int32]
        L.or_mlp_forward.restype = None
        L.or_mlp_loss_grad.argtypes = [dp, C.c_int32, dp, dp, dp, C.c_int32]
        L.or_mlp_loss_grad.restype = C.c_double
        L.or_mlp_adam.argtypes = [dp, dp, dp, dp, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                  C.c_double, C.c_double]
        L.or_mlp_adam.restype = None
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def make_params(**kw) -> Params:
    """Oracle parameters; keyword names follow the ``Params`` fields."""
    p = Params()
    defaults = dict(h=0.1, R=0.5, rho_p=2.65, rho_f=1.0, g=(0.0, -1.0, 0.0), nl=314,
                    dt_f=8.27944e-4, alpha=1.0, n_iter=3, tol_mode=0, tol=1e-6, max_iter=10,
                    n_sub=20, k_n=1e5, e_n=0.9, mu=0.5, kt_ratio=2.0 / 7.0, dt_ratio=2.0 / 7.0,
                    use_cells=0, contact_model=0, t_c=10 * 8.27944e-4, e_t=0.39)
    defaults.update(kw)
    for k, v in defaults.items():
        if k == "g":
            p.g = (C.c_double * 3)(*v)
        else:
            setattr(p, k, v)
    if "wnx" not in kw:
        p.wi0, p.wnx = 0, p.nx
    if "wnz" not in kw:
        p.wk0, p.wnz = 0, p.nz
    return p


def grid_shapes(p: Params):
    """Shapes of the stored u, v, w arrays for parameters p."""
    return ((p.wnz, p.ny, p.wnx), (p.wnz, p.ny + 1, p.wnx), (p.wnz, p.ny, p.wnx))


def template(nl: int, R: float, h: float):
    t = np.zeros((nl, 3))
    dV = C.c_double()
    lib().or_template(nl, R, h, _d(t), C.byref(dV))
    return t, dV.value


def phi(r: float) -> float:
    return lib().or_phi(float(r))


def interpolate(p: Params, grids, x, up, om):
    x, up, om = _f64(x), _f64(up), _f64(om)
    g = [_f64(a) for a in grids]
    n = x.shape[0]
    U = np.zeros((n, p.nl, 3))
    Ud = np.zeros((n, p.nl, 3))
    lib().or_interpolate(C.byref(p), _d(g[0]), _d(g[1]), _d(g[2]), n, _d(x), _d(up), _d(om),
                         _d(U), _d(Ud))
    return U, Ud


def spread(p: Params, x, F, fields):
    """Accumulate the spread of marker vectors F [n, nl, 3] into fields (modified in place)."""
    x, F = _f64(x), _f64(F)
    for a in fields:
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().or_spread(C.byref(p), x.shape[0], _d(x), _d(F), _d(fields[0]), _d(fields[1]),
                    _d(fields[2]))


def ib_forcing(p: Params, uhat, f, x, up, om, F0=None, want_marker_force=False,
               want_ustar=False):
    """Multi-direct forcing; f (3 float64 arrays) is updated in place.

    Returns dict(Fh, Th, slip, iters, [Fmark], [ustar])."""
    x, up, om, F0 = _f64(x), _f64(up), _f64(om), _f64(F0)
    uh = [_f64(a) for a in uhat]
    for a in f:
        assert a.dtype == np.float64 and a.flags.c_contiguous
    n = x.shape[0]
    Fh = np.zeros((n, 3))
    Th = np.zeros((n, 3))
    slip = np.zeros(max(p.n_iter, p.max_iter + 1, 1) + 1)
    iters = C.c_int32()
    Fm = np.zeros((n, p.nl, 3)) if want_marker_force else None
    us = [np.zeros_like(a) for a in uh] if want_ustar else [None, None, None]
    rc = lib().or_ib_forcing(C.byref(p), _d(uh[0]), _d(uh[1]), _d(uh[2]), _d(f[0]), _d(f[1]),
                             _d(f[2]), n, _d(x), _d(up), _d(om), _d(F0), _d(Fh), _d(Th), _d(slip),
                             C.byref(iters), _d(Fm), _d(us[0]), _d(us[1]), _d(us[2]))
    if rc:
        raise RuntimeError(f"oracle ib_forcing failed with code {rc}")
    it = iters.value
    n_slip = it + 1 if p.tol_mode else max(it, 1)
    out = dict(Fh=Fh, Th=Th, slip=slip[:n_slip].copy(), iters=it)
    if want_marker_force:
        out["Fmark"] = Fm
    if want_ustar:
        out["ustar"] = us
    return out


def contacts(p: Params, x, cap=None):
    """Canonical contact list (rows (i, j); j = -1 bottom wall, -2 top wall)."""
    x = _f64(x)
    n = x.shape[0]
    if cap is None:
        cap = 16 * max(n, 1)
    pairs = np.zeros((cap, 2), dtype=np.int32)
    n_out = C.c_int64()
    rc = lib().or_contacts(C.byref(p), n, _d(x), _i(pairs), cap, C.byref(n_out))
    return rc, pairs[: min(n_out.value, cap)].copy(), n_out.value


def bed_flags(p: Params, x):
    """Bed (1) / flying (0) flag of every sphere and the bed count, by the
    detection iteration of sec. 4.3.1 step (1); returns (rc, flags, n_bed)."""
    x = _f64(x)
    n = x.shape[0]
    flags = np.zeros(n, dtype=np.int32)
    nb = C.c_int64()
    rc = lib().or_bed_flags(C.byref(p), n, _d(x), _i(flags), C.byref(nb))
    return rc, flags, nb.value


def inner_fluid(p: Params, fields, x):
    """Fluid velocity and its moment integrated over each sphere's volume by
    the staggered nodes inside it, [n, 6] (int u dV, int r x u dV)."""
    x = _f64(x)
    g = [_f64(a) for a in fields]
    out = np.zeros((x.shape[0], 6))
    rc = lib().or_inner_fluid(C.byref(p), _d(g[0]), _d(g[1]), _d(g[2]), x.shape[0], _d(x),
                              _d(out))
    if rc:
        raise RuntimeError(f"oracle inner_fluid failed with code {rc}")
    return out


def step_ex(p: Params, alpha, advance, uhat, f, x, u, om, hist: "History", F0=None,
            inner_prev=None, want_inner=False):
    """One step with a per-call forcing coefficient alpha, optionally the
    inner-fluid term (inner_prev [n, 6]) and without the particle substeps
    (advance = False); x, u, om, hist, f updated in place."""
    for a in (x, u, om):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    uh = [_f64(a) for a in uhat]
    F0, ip_ = _f64(F0), _f64(inner_prev)
    n = x.shape[0]
    Fh = np.zeros((n, 3))
    Th = np.zeros((n, 3))
    slip = np.zeros(max(p.n_iter, p.max_iter + 1, 1) + 1)
    iters = C.c_int32()
    inner = np.zeros((n, 6)) if want_inner else None
    rc = lib().or_step_ex(C.byref(p), float(alpha), int(bool(advance)), _d(uh[0]), _d(uh[1]),
                          _d(uh[2]), _d(f[0]), _d(f[1]), _d(f[2]), n, _d(x), _d(u), _d(om),
                          _d(F0), _i(hist.partner), _d(hist.dt), _d(hist.uin), _i(hist.cnt),
                          _d(Fh), _d(Th), _d(slip), C.byref(iters), _d(ip_), _d(inner))
    it = iters.value
    n_slip = it + 1 if p.tol_mode else max(it, 1)
    return rc, dict(Fh=Fh, Th=Th, slip=slip[:n_slip].copy(), iters=it, inner=inner)


def history_match(old_ids, new_ids):
    old = np.ascontiguousarray(old_ids, dtype=np.int32)
    new = np.ascontiguousarray(new_ids, dtype=np.int32)
    src = np.zeros(len(new), dtype=np.int32)
    lib().or_history_match(len(old), _i(old), len(new), _i(new), _i(src))
    return src


class History:
    """Contact history M_p in the oracle's layout."""

    def __init__(self, n: int):
        self.partner = np.zeros((n, SLOTS), dtype=np.int32)
        self.dt = np.zeros((n, SLOTS, 3))
        self.uin = np.zeros((n, SLOTS))
        self.cnt = np.zeros(n, dtype=np.int32)

    def copy(self):
        h = History(0)
        h.partner, h.dt, h.uin, h.cnt = (self.partner.copy(), self.dt.copy(), self.uin.copy(),
                                         self.cnt.copy())
        return h


def dem(p: Params, x, u, om, Fh, Th, hist: History):
    """n_sub contact/integration substeps; x, u, om, hist updated in place.

    Returns (rc, Fc, Tc) with the contact force/torque of the last substep."""
    for a in (x, u, om):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    Fh, Th = _f64(Fh), _f64(Th)
    n = x.shape[0]
    Fc = np.zeros((n, 3))
    Tc = np.zeros((n, 3))
    rc = lib().or_dem(C.byref(p), n, _d(x), _d(u), _d(om), _d(Fh), _d(Th), _i(hist.partner),
                      _d(hist.dt), _d(hist.uin), _i(hist.cnt), _d(Fc), _d(Tc))
    return rc, Fc, Tc


def step(p: Params, uhat, f, x, u, om, hist: History, F0=None):
    """One particle step (IB forcing, then n_sub DEM substeps), in place."""
    for a in (x, u, om):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    uh = [_f64(a) for a in uhat]
    F0 = _f64(F0)
    n = x.shape[0]
    Fh = np.zeros((n, 3))
    Th = np.zeros((n, 3))
    slip = np.zeros(max(p.n_iter, p.max_iter + 1, 1) + 1)
    iters = C.c_int32()
    rc = lib().or_step(C.byref(p), _d(uh[0]), _d(uh[1]), _d(uh[2]), _d(f[0]), _d(f[1]), _d(f[2]),
                       n, _d(x), _d(u), _d(om), _d(F0), _i(hist.partner), _d(hist.dt),
                       _d(hist.uin), _i(hist.cnt), _d(Fh), _d(Th), _d(slip), C.byref(iters))
    it = iters.value
    n_slip = it + 1 if p.tol_mode else max(it, 1)
    return rc, dict(Fh=Fh, Th=Th, slip=slip[:n_slip].copy(), iters=it)


# --------------------------------------------------------------------------
# learned warm start (mlp_oracle.c)
# --------------------------------------------------------------------------
MLP_SHAPES = (("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (16, 64)), ("b3", (16,)))


def mlp_nparam() -> int:
    return lib().or_mlp_nparam()


def mlp_pack(d) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([np.asarray(d[k], dtype=np.float64).ravel()
                                                for k, _ in MLP_SHAPES]))


def mlp_unpack(flat):
    out, o = {}, 0
    for k, s in MLP_SHAPES:
        n = int(np.prod(s))
        out[k] = np.asarray(flat[o:o + n]).reshape(s).copy()
        o += n
    return out


def bf16(x: float) -> float:
    return lib().or_bf16(float(x))


def mlp_forward(params, X, emulate_bf16=True):
    P = _f64(params)
    X = _f64(X)
    Y = np.zeros((X.shape[0], 16))
    lib().or_mlp_forward(_d(P), X.shape[0], _d(X), _d(Y), int(emulate_bf16))
    return Y


def mlp_loss_grad(params, X, T, emulate_bf16=True):
    P, X, T = _f64(params), _f64(X), _f64(T)
    g = np.zeros(mlp_nparam())
    loss = lib().or_mlp_loss_grad(_d(P), X.shape[0], _d(X), _d(T), _d(g), int(emulate_bf16))
    return loss, g


def mlp_adam(params, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of params, m, v (float64 arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().or_mlp_adam(_d(params), _d(m), _d(v), _d(g), params.size, int(t), lr, beta1, beta2, eps)


def learned_features(p: Params, uhat, x, up, om):
    """Features of the learned warm start for every marker, [n, nl, 16] FP64
    (not part of the paper; the network's input as the library defines it):
    slip U_d - I[u-hat] with U_d the rigid-body velocity of the marker and
    I the interpolation of sec. 3.3, the template normal t_l, the sphere
    velocity u_p and R omega_p; the last four entries zero."""
    x, up, om = _f64(x), _f64(up), _f64(om)
    U, Ud = interpolate(p, uhat, x, up, om)
    t, _ = template(p.nl, p.R, p.h)
    n = x.shape[0]
    F = np.zeros((n, p.nl, 16))
    F[:, :, 0:3] = Ud - U
    F[:, :, 3:6] = t[None, :, :]
    F[:, :, 6:9] = up[:, None, :]
    F[:, :, 9:12] = p.R * om[:, None, :]
    return F


def learned_initial_force(params, norm, feat, adt):
    """Initial marker force of the learned start, [..., 3]: the network on the
    standardised features (BF16-emulating forward), de-standardised, divided
    by alpha dt."""
    norm = np.asarray(norm, dtype=np.float64)
    shape = feat.shape[:-1]
    X = (np.asarray(feat, dtype=np.float64).reshape(-1, 16) - norm[:16]) / norm[16:32]
    Y = mlp_forward(params, X)[:, :3]
    return ((Y * norm[35:38] + norm[32:35]) / adt).reshape(*shape, 3)


def reject_learned(rel_slip) -> bool:
    """The fallback rule of the learned start: reject when the first relative
    slip is not below one or the slip grows from one pass to the next."""
    s = list(rel_slip)
    if not s:
        return False
    if not s[0] < 1.0:
        return True
    return any(b > a for a, b in zip(s, s[1:]))
