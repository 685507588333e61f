"""Network inputs shared by the CPU pins of the oracle's network and the GPU
parity tests (seeded construction only; no arithmetic of the method).

`dyadic_network` builds a 16-64-64-16 network and a batch on which every
value the network rounds to BF16 is computed exactly in single precision on
any accumulation order: inputs and weights are small dyadic rationals, and
the biases put every hidden pre-activation at z >= 6, where GELU(z) and its
derivative equal z and 1 in single precision (every unit is active: an
inactive unit's gradient would be a GELU tail of 1e-10, which Adam's
normalisation by |g| + eps magnifies).  Targets are placed
at y - 3 d with d a multiple of 1/8, so the output error 2 (y - T) / (3 B) is
again exact for a power-of-two batch B.  BF16 rounding decisions therefore
cannot differ between an FP32 device and the FP64 oracle."""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT, N_FEAT = 16, 64, 16, 12
SHAPES = (("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
          ("W3", (16, 64)), ("b3", (16,)))


def pack(d):
    return np.concatenate([np.asarray(d[k], dtype=np.float64).ravel() for k, _ in SHAPES])


def dyadic_network(seed: int, B: int = 4096):
    """(params float64 [6288], X float64 [B, 16]); targets come from
    dyadic_targets once the network output is known."""
    rng = np.random.default_rng(seed)
    d = {}
    d["W1"] = np.zeros((N_HID, N_IN))
    d["W1"][:, :N_FEAT] = rng.integers(-1, 2, size=(N_HID, N_FEAT)) / 16.0
    d["b1"] = np.full(N_HID, 8.0)
    d["W2"] = rng.integers(-1, 2, size=(N_HID, N_HID)) / 128.0
    d["b2"] = np.full(N_HID, 12.0)
    d["W3"] = np.zeros((N_OUT, N_HID))
    d["W3"][:3] = rng.integers(-4, 5, size=(3, N_HID)) / 64.0
    d["b3"] = np.zeros(N_OUT)
    d["b3"][:3] = rng.integers(-8, 9, size=3) / 4.0
    X = np.zeros((B, N_IN))
    X[:, :N_FEAT] = rng.integers(-8, 9, size=(B, N_FEAT)) / 4.0
    return pack(d), X


def dyadic_targets(seed: int, Y):
    """T = Y - 3 d, d uniform on the multiples of 1/8 in [-1, 1]."""
    rng = np.random.default_rng(seed + 1)
    d = rng.integers(-8, 9, size=(Y.shape[0], 3)) / 8.0
    return Y[:, :3] - 3.0 * d
