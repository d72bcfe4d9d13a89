"""Oracle of the learned-proposal form (not in the paper): the pair-scoring
network, its loss gradient, the Adam update and the pair features.

TEST INFRASTRUCTURE ONLY: used by the tests and nothing else; it shares no
code with the HIP library.  The network (``mlp_oracle.c``) is evaluated in
FP64.  Parameter vector layout (4545 values, also the library's):
W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.

Features of the pair flip (i, j), i < j, of a state x with local fields
F = h + J s: (s_i F_i, s_j F_j, sqrt(N) J_ij, s_i s_j).  The sign-adjusted
fields make the exact energy change -2 f_i - 2 f_j + 4 J_ij s_i s_j a function
of the features; sqrt(N) puts couplings drawn with standard deviation
1/sqrt(N) on the scale of the fields.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlp_oracle.so")
SRC_PATH = os.path.join(_HERE, "mlp_oracle.c")
H = 64
NPARAM = 4 * H + H + H * H + H + H + 1   # 4545
OFF_W1, OFF_B1 = 0, 4 * H
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H

_dp = ctypes.POINTER(ctypes.c_double)
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", SRC_PATH, "-o", LIB_PATH, "-lm"])
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        L.mo_nparam.restype = ctypes.c_int
        L.mo_forward.restype = None
        L.mo_forward.argtypes = [_dp, _dp, ctypes.c_int, _dp]
        L.mo_loss_grad.restype = ctypes.c_double
        L.mo_loss_grad.argtypes = [_dp, _dp, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_double, _dp]
        assert L.mo_nparam() == NPARAM
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def forward(params, X) -> np.ndarray:
    """Logits of the samples X (n, 4)."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 4)
    z = np.zeros(X.shape[0])
    if X.shape[0]:
        lib().mo_forward(_d(P), _d(X), X.shape[0], _d(z))
    return z


def loss_grad(params, X, y, pos_weight=1.0):
    """Class-weighted binary cross-entropy with logits, averaged over the
    samples, and its gradient.  Returns (loss, grad (4545,))."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 4)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    G = np.zeros(NPARAM)
    L = lib().mo_loss_grad(_d(P), _d(X), y.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), X.shape[0],
                           float(pos_weight), _d(G))
    return L, G


def adam_step(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) in FP64; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def spins(x, N) -> np.ndarray:
    """s_i = 1 - 2 sigma_i of one state (W words)."""
    x = np.asarray(x, np.uint64).reshape(-1)
    bits = np.array([(int(x[i >> 6]) >> (i & 63)) & 1 for i in range(N)], dtype=np.int64)
    return (1 - 2 * bits).astype(np.float64)


def pair_features(J, h, x, pairs=None):
    """Features of the pair flips of x: rows (s_i F_i, s_j F_j, sqrt(N) J_ij, s_i s_j)
    for the codes in ``pairs`` (i | j << 16), or for all i < j in row order."""
    J = np.asarray(J, np.float64)
    N = len(h)
    s = spins(x, N)
    F = np.asarray(h, np.float64) + J @ s
    f = s * F
    if pairs is None:
        ii, jj = np.triu_indices(N, 1)
    else:
        pairs = np.asarray(pairs, np.uint32)
        ii = (pairs & 0xFFFF).astype(np.int64)
        jj = (pairs >> 16).astype(np.int64)
    return np.stack([f[ii], f[jj], np.sqrt(N) * J[ii, jj], s[ii] * s[jj]], axis=1), ii, jj
