"""Particle-phase step of the particle-resolved sediment-transport method
(Zhu et al., arXiv 2108.01814) on AMD MI355X.

Thin ctypes binding of ``libprs.so`` (declared in ``include/prs.h``): it only
checks shapes, dtypes and devices of the torch tensors it is given and passes
their device pointers and the current HIP stream to the library.  Every step
of the computation runs in the library's HIP kernels; there is no fallback,
and importing the binding without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprs.so")

PRS_OK, PRS_EINVAL, PRS_ECAPACITY, PRS_EDOMAIN, PRS_ENONFINITE, PRS_EHIP, PRS_ESKIN = range(7)
F32, F64 = 0, 1
CONTACT_FIXED, CONTACT_COLLISION_TIME = 0, 1
SLOTS = 14
MAX_PP = 12
WALL_BOTTOM, WALL_TOP = -1, -2
MAX_SLIP = 64
_NAMES = {1: "EINVAL", 2: "ECAPACITY", 3: "EDOMAIN", 4: "ENONFINITE", 5: "EHIP", 6: "ESKIN"}

EXPORTS = ("prs_create", "prs_destroy", "prs_last_error", "prs_template", "prs_interpolate",
           "prs_spread", "prs_contacts", "prs_bed_flags", "prs_step_particles",
           "prs_step_particles_ex", "prs_inner_fluid",
           "prs_timing_enable",
           "prs_timing_read", "prs_mlp_create", "prs_mlp_destroy", "prs_mlp_last_error",
           "prs_mlp_get", "prs_mlp_forward", "prs_mlp_backward", "prs_mlp_adam",
           "prs_mlp_train_step", "prs_mlp_loss", "prs_mlp_standardize", "prs_mlp_fit_norm",
           "prs_mlp_fit_norm_noalloc",
           "prs_set_learned", "prs_forcing_samples")
MLP_PARAMS = 6288
MLP_NORM = 38


class PrsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
        ("radius", C.c_double), ("rho_p", C.c_double), ("rho_f", C.c_double),
        ("gravity", C.c_double * 3),
        ("n_markers", C.c_int32),
        ("dt_f", C.c_double), ("alpha", C.c_double),
        ("n_iter", C.c_int32), ("tol_mode", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
        ("n_sub", C.c_int32),
        ("k_n", C.c_double), ("e_n", C.c_double), ("mu", C.c_double), ("kt_ratio", C.c_double),
        ("dt_ratio", C.c_double),
        ("skin", C.c_double),
        ("precision", C.c_int32),
        ("max_particles", C.c_int32),
        ("contact_model", C.c_int32), ("t_c", C.c_double), ("e_t", C.c_double),
    ]


class _History(C.Structure):
    _fields_ = [("partner", C.c_void_p), ("delta_t", C.c_void_p), ("u_in", C.c_void_p),
                ("count", C.c_void_p)]


class StepArgs(C.Structure):
    _fields_ = [("uhat", C.POINTER(C.c_void_p)), ("f", C.POINTER(C.c_void_p)),
                ("zero_f", C.c_int32), ("x", C.c_void_p), ("u", C.c_void_p), ("om", C.c_void_p),
                ("n", C.c_int32), ("hist", C.POINTER(_History)), ("Fh", C.c_void_p),
                ("Th", C.c_void_p), ("F0", C.c_void_p), ("alpha", C.c_double),
                ("advance", C.c_int32), ("inner_prev", C.c_void_p), ("inner_out", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32), ("n_slip", C.c_int32),
        ("rel_slip", C.c_double * MAX_SLIP),
        ("contacts", C.c_int64), ("pairs_last", C.c_int64), ("wall_last", C.c_int64),
        ("flags", C.c_uint32), ("rejected_learned", C.c_int32),
    ]

    def as_dict(self):
        return dict(iterations=self.iterations, rel_slip=list(self.rel_slip[: self.n_slip]),
                    contacts=self.contacts, pairs_last=self.pairs_last,
                    wall_last=self.wall_last, flags=self.flags,
                    rejected_learned=self.rejected_learned)


class Timing(C.Structure):
    _fields_ = [("steps", C.c_int64), ("ms_zero_f", C.c_double), ("ms_sort", C.c_double),
                ("ms_interp", C.c_double), ("ms_spread", C.c_double), ("ms_search", C.c_double),
                ("ms_substep", C.c_double), ("ms_writeback", C.c_double),
                ("n_interp", C.c_int64), ("n_spread", C.c_int64), ("n_substep", C.c_int64),
                ("ms_learned", C.c_double), ("n_learned", C.c_int64),
                ("ms_record", C.c_double), ("n_record", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libprs.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2108_01814_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.prs_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.prs_destroy.argtypes = [vp]
        L.prs_destroy.restype = None
        L.prs_last_error.argtypes = [vp]
        L.prs_last_error.restype = C.c_char_p
        L.prs_template.argtypes = [vp, vp, C.POINTER(C.c_double)]
        L.prs_interpolate.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_int32, vp, vp]
        L.prs_spread.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp, vp, C.c_int]
        L.prs_contacts.argtypes = [vp, vp, vp, C.c_int32, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.prs_bed_flags.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_int64)]
        L.prs_step_particles.argtypes = [vp, vp, C.POINTER(vp), C.POINTER(vp), C.c_int, vp, vp,
                                         vp, C.c_int32, C.POINTER(_History), vp, vp, vp,
                                         C.POINTER(Stats)]
        L.prs_step_particles_ex.argtypes = [vp, vp, C.POINTER(StepArgs), C.POINTER(Stats)]
        L.prs_inner_fluid.argtypes = [vp, vp, C.POINTER(vp), vp, C.c_int32, vp]
        L.prs_timing_enable.argtypes = [vp, C.c_int]
        L.prs_timing_read.argtypes = [vp, C.POINTER(Timing), C.c_int]
        L.prs_set_learned.argtypes = [vp, vp]
        L.prs_forcing_samples.argtypes = [vp, vp, C.POINTER(vp), C.POINTER(vp), vp, vp, vp,
                                          C.c_int32, C.c_int32, vp, vp, C.POINTER(Stats)]
        L.prs_mlp_create.argtypes = [vp, vp, C.POINTER(vp)]
        L.prs_mlp_destroy.argtypes = [vp]
        L.prs_mlp_destroy.restype = None
        L.prs_mlp_last_error.argtypes = [vp]
        L.prs_mlp_last_error.restype = C.c_char_p
        L.prs_mlp_get.argtypes = [vp, vp, vp]
        L.prs_mlp_forward.argtypes = [vp, vp, vp, C.c_int32, C.c_int, vp]
        L.prs_mlp_backward.argtypes = [vp, vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double)]
        L.prs_mlp_adam.argtypes = [vp, vp, vp, C.c_float]
        L.prs_mlp_loss.argtypes = [vp, vp, vp, vp, C.c_int32, C.POINTER(C.c_double)]
        L.prs_mlp_standardize.argtypes = [vp, vp, vp, vp, C.c_int64, vp, vp]
        L.prs_mlp_fit_norm.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.prs_mlp_fit_norm_noalloc.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.prs_mlp_train_step.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float,
                                         C.POINTER(C.c_double)]
        _lib = L
    return _lib


def make_params(**kw) -> Params:
    p = Params()
    d = dict(h=0.1, radius=0.5, rho_p=2.65, rho_f=1.0, gravity=(0.0, -1.0, 0.0), n_markers=314,
             dt_f=8.27944e-4, alpha=1.0, n_iter=3, tol_mode=0, tol=1e-6, max_iter=10, n_sub=20,
             k_n=1e5, e_n=0.9, mu=0.5, kt_ratio=2.0 / 7.0, dt_ratio=2.0 / 7.0, skin=0.1,
             precision=F64, max_particles=1, contact_model=CONTACT_FIXED, t_c=10 * 8.27944e-4,
             e_t=0.39)
    d.update(kw)
    for k, v in d.items():
        if k == "gravity":
            p.gravity = (C.c_double * 3)(*v)
        else:
            setattr(p, k, v)
    return p


def _stream_ptr():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


@dataclass
class History:
    """Contact history M_p (sec. 3.4) as device tensors."""
    partner: "object"
    delta_t: "object"
    u_in: "object"
    count: "object"

    @classmethod
    def zeros(cls, n: int, device="cuda"):
        import torch

        return cls(torch.zeros((n, SLOTS), dtype=torch.int32, device=device),
                   torch.zeros((n, SLOTS, 3), dtype=torch.float64, device=device),
                   torch.zeros((n, SLOTS), dtype=torch.float64, device=device),
                   torch.zeros((n,), dtype=torch.int8, device=device))

    @classmethod
    def from_host(cls, h: dict, device="cuda"):
        """Device copy of a history given as host arrays (partner, delta_t,
        u_in, count in the layout of prs_history)."""
        import torch

        return cls(torch.as_tensor(h["partner"], dtype=torch.int32).to(device),
                   torch.as_tensor(h["delta_t"], dtype=torch.float64).to(device),
                   torch.as_tensor(h["u_in"], dtype=torch.float64).to(device),
                   torch.as_tensor(h["count"], dtype=torch.int8).to(device))

    def clone(self):
        return History(self.partner.clone(), self.delta_t.clone(), self.u_in.clone(),
                       self.count.clone())

    def _c(self):
        return _History(self.partner.data_ptr(), self.delta_t.data_ptr(), self.u_in.data_ptr(),
                        self.count.data_ptr())


class Context:
    """One library context (scratch for up to max_particles spheres)."""

    def __init__(self, params: Params):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the particle step needs a ROCm GPU")
        self.p = params
        self._h = C.c_void_p()
        rc = lib().prs_create(C.byref(params), C.byref(self._h))
        if rc != PRS_OK:
            raise PrsError(rc, "prs_create rejected the parameters or could not allocate")
        self.dtype = torch.float64 if params.precision == F64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if self._h:
            lib().prs_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def timing(self, enable: bool = True):
        """Switch per-phase event timing of step() on or off."""
        self._err(lib().prs_timing_enable(self._h, int(bool(enable))))

    def read_timing(self, reset: bool = True) -> dict:
        t = Timing()
        self._err(lib().prs_timing_read(self._h, C.byref(t), int(bool(reset))))
        return t.as_dict()

    # -- argument checks (the library cannot see tensor sizes) --------------
    def _err(self, rc):
        if rc != PRS_OK:
            raise PrsError(rc, lib().prs_last_error(self._h).decode())

    def _chk(self, t, shape, dtype, name):
        if t is None:
            raise ValueError(f"{name} is required")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
        if t.dtype != dtype:
            raise ValueError(f"{name}: dtype {t.dtype} != {dtype}")
        if t.device != self.device:
            raise ValueError(f"{name}: on {t.device}, expected {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def grid_shapes(self):
        p = self.p
        return ((p.nz, p.ny, p.nx), (p.nz, p.ny + 1, p.nx), (p.nz, p.ny, p.nx))

    def _chk_fields(self, fields: Sequence, name):
        if len(fields) != 3:
            raise ValueError(f"{name}: three components expected")
        for c, (t, s) in enumerate(zip(fields, self.grid_shapes())):
            self._chk(t, s, self.dtype, f"{name}[{c}]")

    def _chk_particles(self, n, **arrays):
        import torch

        for k, t in arrays.items():
            self._chk(t, (n, 3), torch.float64, k)

    # -- calls ---------------------------------------------------------------
    def template(self):
        import numpy as np

        t = np.zeros((self.p.n_markers, 3))
        dV = C.c_double()
        self._err(lib().prs_template(self._h, C.c_void_p(t.ctypes.data), C.byref(dV)))
        return t, dV.value

    def interpolate(self, fields, x, up=None, om=None, want_ud=False):
        import torch

        n = x.shape[0]
        self._chk_fields(fields, "fields")
        self._chk_particles(n, x=x)
        if want_ud:
            self._chk_particles(n, up=up, om=om)
        U = torch.empty((n, self.p.n_markers, 3), dtype=self.dtype, device=self.device)
        Ud = torch.empty_like(U) if want_ud else None
        self._err(lib().prs_interpolate(self._h, _stream_ptr(), _ptr(fields[0]), _ptr(fields[1]),
                                        _ptr(fields[2]), _ptr(x), _ptr(up if want_ud else None),
                                        _ptr(om if want_ud else None), n, _ptr(U), _ptr(Ud)))
        return (U, Ud) if want_ud else U

    def spread(self, x, F, fields, accumulate=True):
        n = x.shape[0]
        self._chk_particles(n, x=x)
        self._chk(F, (n, self.p.n_markers, 3), self.dtype, "F")
        self._chk_fields(fields, "fields")
        self._err(lib().prs_spread(self._h, _stream_ptr(), _ptr(x), n, _ptr(F), _ptr(fields[0]),
                                   _ptr(fields[1]), _ptr(fields[2]), int(bool(accumulate))))

    def contacts(self, x, cap: Optional[int] = None):
        """Canonical contact list as an int32 [n_contacts, 2] device tensor."""
        import torch

        n = x.shape[0]
        self._chk_particles(n, x=x)
        if cap is None:
            cap = 8 * max(n, 1)
        pairs = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.device)
        n_out = C.c_int64()
        rc = lib().prs_contacts(self._h, _stream_ptr(), _ptr(x), n, _ptr(pairs), cap,
                                C.byref(n_out))
        if rc == PRS_ECAPACITY and n_out.value > cap:
            return self.contacts(x, cap=int(n_out.value))
        self._err(rc)
        return pairs[: n_out.value]

    def bed_flags(self, x):
        """Bed (1) / flying (0) flag of every sphere (int8 device tensor, caller
        order) and the number of bed spheres (prs_bed_flags)."""
        import torch

        n = x.shape[0]
        self._chk_particles(n, x=x)
        flags = torch.empty(n, dtype=torch.int8, device=x.device)
        nb = C.c_int64()
        self._err(lib().prs_bed_flags(self._h, _stream_ptr(), _ptr(x), n, _ptr(flags),
                                      C.byref(nb)))
        return flags, nb.value

    def step(self, uhat, f, x, u, om, hist: History, Fh=None, Th=None, F0=None, zero_f=False,
             alpha: float = 0.0, advance: bool = True, inner_prev=None, inner_out=None):
        """One particle step in place (x, u, om, hist, f); returns (Fh, Th, stats).

        alpha > 0: this call's forcing coefficient (a Runge-Kutta substep's
        alpha_k); advance = False: the forcing only; inner_prev / inner_out
        ([n, 6] float64): the inner-fluid term (prs_step_particles_ex)."""
        import torch

        n = x.shape[0]
        self._chk_fields(uhat, "uhat")
        self._chk_fields(f, "f")
        self._chk_particles(n, x=x, u=u, om=om)
        self._chk(hist.partner, (n, SLOTS), torch.int32, "hist.partner")
        self._chk(hist.delta_t, (n, SLOTS, 3), torch.float64, "hist.delta_t")
        self._chk(hist.u_in, (n, SLOTS), torch.float64, "hist.u_in")
        self._chk(hist.count, (n,), torch.int8, "hist.count")
        if Fh is None:
            Fh = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if Th is None:
            Th = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        self._chk_particles(n, Fh=Fh, Th=Th)
        if F0 is not None:
            self._chk(F0, (n, self.p.n_markers, 3), self.dtype, "F0")
        for name, t in (("inner_prev", inner_prev), ("inner_out", inner_out)):
            if t is not None:
                self._chk(t, (n, 6), torch.float64, name)
        uh = (C.c_void_p * 3)(*[t.data_ptr() for t in uhat])
        ff = (C.c_void_p * 3)(*[t.data_ptr() for t in f])
        H = hist._c()
        A = StepArgs()
        A.uhat = C.cast(uh, C.POINTER(C.c_void_p))
        A.f = C.cast(ff, C.POINTER(C.c_void_p))
        A.zero_f = int(bool(zero_f))
        A.x, A.u, A.om = _ptr(x), _ptr(u), _ptr(om)
        A.n = n
        A.hist = C.pointer(H)
        A.Fh, A.Th, A.F0 = _ptr(Fh), _ptr(Th), _ptr(F0)
        A.alpha = float(alpha)
        A.advance = int(bool(advance))
        A.inner_prev, A.inner_out = _ptr(inner_prev), _ptr(inner_out)
        st = Stats()
        rc = lib().prs_step_particles_ex(self._h, _stream_ptr(), C.byref(A), C.byref(st))
        self._err(rc)
        return Fh, Th, st.as_dict()

    def inner_fluid(self, fields, x):
        """Fluid velocity and its moment integrated over each sphere's volume,
        [n, 6] float64 (prs_inner_fluid)."""
        import torch

        n = x.shape[0]
        self._chk_fields(fields, "fields")
        self._chk_particles(n, x=x)
        out = torch.empty((n, 6), dtype=torch.float64, device=x.device)
        g = (C.c_void_p * 3)(*[t.data_ptr() for t in fields])
        self._err(lib().prs_inner_fluid(self._h, _stream_ptr(), g, _ptr(x), n, _ptr(out)))
        return out


    def set_learned(self, mlp: Optional["Mlp"]):
        """Start every following step from the network's prediction (None:
        plain start).  The context keeps a reference to the network."""
        self._err(lib().prs_set_learned(self._h, mlp._h if mlp is not None else None))
        self._mlp = mlp

    def forcing_samples(self, uhat, f, x, u, om, n_iter: int, feat=None, target=None):
        """Features [n, n_markers, 16] and targets [n, n_markers, 3] (float32,
        caller order) from n_iter plain forcing iterations; f is overwritten
        with the resulting force field.  Returns (feat, target, stats)."""
        import torch

        n = x.shape[0]
        nl = self.p.n_markers
        self._chk_fields(uhat, "uhat")
        self._chk_fields(f, "f")
        self._chk_particles(n, x=x, u=u, om=om)
        if feat is None:
            feat = torch.empty((n, nl, 16), dtype=torch.float32, device=self.device)
        if target is None:
            target = torch.empty((n, nl, 3), dtype=torch.float32, device=self.device)
        self._chk(feat, (n, nl, 16), torch.float32, "feat")
        self._chk(target, (n, nl, 3), torch.float32, "target")
        uh = (C.c_void_p * 3)(*[t.data_ptr() for t in uhat])
        ff = (C.c_void_p * 3)(*[t.data_ptr() for t in f])
        st = Stats()
        self._err(lib().prs_forcing_samples(self._h, _stream_ptr(), uh, ff, _ptr(x), _ptr(u),
                                            _ptr(om), n, int(n_iter), _ptr(feat), _ptr(target),
                                            C.byref(st)))
        return feat, target, st.as_dict()


class Mlp:
    """The learned warm-start network (device weights, Adam state,
    normalisation), wrapping the prs_mlp_* entry points."""

    def __init__(self, params, norm):
        import numpy as np

        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        nv = np.ascontiguousarray(norm, dtype=np.float32).ravel()
        if p.size != MLP_PARAMS or nv.size != MLP_NORM:
            raise ValueError("parameter / normalisation vectors of the wrong size")
        self._h = C.c_void_p()
        rc = lib().prs_mlp_create(C.c_void_p(p.ctypes.data), C.c_void_p(nv.ctypes.data),
                                  C.byref(self._h))
        if rc != PRS_OK:
            raise PrsError(rc, "prs_mlp_create failed")

    @staticmethod
    def init_params(seed: int = 0):
        """Seeded U(+-1/sqrt(fan_in)) weights, zero biases, padding rows and
        columns zero (flat vector in the library's order)."""
        import numpy as np

        rng = np.random.default_rng(seed)
        W1 = rng.uniform(-1, 1, (64, 16)) / np.sqrt(12.0)
        W1[:, 12:] = 0.0
        W2 = rng.uniform(-1, 1, (64, 64)) / 8.0
        W3 = rng.uniform(-1, 1, (16, 64)) / 8.0
        W3[3:] = 0.0
        return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(),
                               np.zeros(16)]).astype(np.float32)

    def close(self):
        if self._h:
            lib().prs_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        if rc != PRS_OK:
            raise PrsError(rc, lib().prs_mlp_last_error(self._h).decode())

    @staticmethod
    def _chk(t, shape, name):
        import torch

        if tuple(t.shape) != tuple(shape) or t.dtype != torch.float32 or not t.is_cuda \
                or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous float32 CUDA tensor of shape {shape}")

    def get(self):
        import numpy as np

        p = np.zeros(MLP_PARAMS, np.float32)
        nv = np.zeros(MLP_NORM, np.float32)
        self._err(lib().prs_mlp_get(self._h, C.c_void_p(p.ctypes.data),
                                    C.c_void_p(nv.ctypes.data)))
        return p, nv

    def forward(self, X, raw: bool = True):
        import torch

        B = X.shape[0]
        self._chk(X, (B, 16), "X")
        Y = torch.empty((B, 3), dtype=torch.float32, device=X.device)
        self._err(lib().prs_mlp_forward(self._h, _stream_ptr(), _ptr(X), B, int(raw), _ptr(Y)))
        return Y

    def grad(self, X, T):
        """Gradient of the loss and the loss (prs_mlp_backward)."""
        import torch

        B = X.shape[0]
        self._chk(X, (B, 16), "X")
        self._chk(T, (B, 3), "T")
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = C.c_double()
        self._err(lib().prs_mlp_backward(self._h, _stream_ptr(), _ptr(X), _ptr(T), B, _ptr(g),
                                         C.byref(loss)))
        return g, loss.value

    def adam(self, grad=None, lr: float = 1e-3):
        """One Adam step from grad (device FP32) or the latest backward's."""
        if grad is not None:
            self._chk(grad, (MLP_PARAMS,), "grad")
        self._err(lib().prs_mlp_adam(self._h, _stream_ptr(), _ptr(grad), float(lr)))

    def train_step(self, X, T, lr: float = 1e-3, want_loss: bool = True):
        B = X.shape[0]
        self._chk(X, (B, 16), "X")
        self._chk(T, (B, 3), "T")
        loss = C.c_double()
        self._err(lib().prs_mlp_train_step(self._h, _stream_ptr(), _ptr(X), _ptr(T), B,
                                           float(lr), C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def loss(self, X, T) -> float:
        """Mean square error of the standardised prediction (forward only)."""
        B = X.shape[0]
        self._chk(X, (B, 16), "X")
        self._chk(T, (B, 3), "T")
        loss = C.c_double()
        self._err(lib().prs_mlp_loss(self._h, _stream_ptr(), _ptr(X), _ptr(T), B,
                                     C.byref(loss)))
        return loss.value

    def standardize(self, X, T=None):
        """(X - mean) / std and (T - target mean) / target std with the
        network's statistics, as new device tensors."""
        import torch

        m = X.shape[0]
        self._chk(X, (m, 16), "X")
        if T is not None:
            self._chk(T, (m, 3), "T")
        Xs = torch.empty_like(X)
        Ts = torch.empty_like(T) if T is not None else None
        self._err(lib().prs_mlp_standardize(self._h, _stream_ptr(), _ptr(X), _ptr(T), m,
                                            _ptr(Xs), _ptr(Ts)))
        return Xs, Ts

    @staticmethod
    def fit_norm(X, T, noalloc: bool = False):
        """Normalisation vector (feature mean/std, target mean/std) of raw
        samples X [m, 16], T [m, 3] on the device (prs_mlp_fit_norm, or its
        allocation-free variant prs_mlp_fit_norm_noalloc)."""
        import numpy as np

        m = X.shape[0]
        Mlp._chk(X, (m, 16), "X")
        Mlp._chk(T, (m, 3), "T")
        nv = np.zeros(MLP_NORM, np.float32)
        fn = lib().prs_mlp_fit_norm_noalloc if noalloc else lib().prs_mlp_fit_norm
        rc = fn(_stream_ptr(), _ptr(X), _ptr(T), m, C.c_void_p(nv.ctypes.data))
        if rc != PRS_OK:
            raise PrsError(rc, "prs_mlp_fit_norm%s failed" % ("_noalloc" if noalloc else ""))
        return nv
