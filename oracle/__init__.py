"""Python access to the plain FP64 CPU oracle (``qi_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package.  The HIP library never imports, links or
calls it, and it imports nothing from the HIP library.

Functions mirror the C entry points; states are numpy uint64 arrays of shape
(n, W) with W = ceil(N/64) (bit i of word i>>6 is sigma_i, Eq. 15).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqi_oracle.so")
SRC_PATH = os.path.join(_HERE, "qi_oracle.c")

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_ip = ctypes.POINTER(ctypes.c_int)

_lib = None


def build(force: bool = True, src: str = SRC_PATH, out: str = LIB_PATH, extra=()) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", *extra,
               src, "-o", out, "-lm"]
        subprocess.check_call(cmd)
    return out


def load(path: str):
    """Load a compiled oracle library and declare its signatures."""
    L = ctypes.CDLL(path)
    L.qo_energy.restype = ctypes.c_double
    L.qo_energy.argtypes = [ctypes.c_int, _dp, _dp, _u64p]
    L.qo_flip_change.restype = ctypes.c_double
    L.qo_flip_change.argtypes = [ctypes.c_int, _dp, _dp, _u64p, ctypes.c_int, _ip]
    L.qo_step.restype = ctypes.c_int
    L.qo_step.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, _u64p, _dp, _u8p, _u64p, _dp, _u8p, _ip]
    L.qo_search.restype = ctypes.c_int
    L.qo_search.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            _u64p, _u64p, _dp, _ip, _ip]
    L.qo_merge.restype = ctypes.c_int
    L.qo_merge.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _u64p, _dp,
                           _u64p, _dp, _ip]
    L.qo_brute_lowest.restype = ctypes.c_int
    L.qo_brute_lowest.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _u64p, _dp, _ip]
    L.qo_step_proposed.restype = ctypes.c_int
    L.qo_step_proposed.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, _u64p, _dp,
                                   ctypes.c_int, _ip, _ip, ctypes.POINTER(ctypes.c_uint32),
                                   _u64p, _dp, _u8p, _ip]
    L.qo_field_change.restype = ctypes.c_double
    L.qo_field_change.argtypes = [ctypes.c_int, _dp, _dp, _u64p, ctypes.c_int, _ip]
    L.qo_step_fields.restype = ctypes.c_int
    L.qo_step_fields.argtypes = L.qo_step.argtypes
    L.qo_step_proposed_fields.restype = ctypes.c_int
    L.qo_step_proposed_fields.argtypes = L.qo_step_proposed.argtypes
    L.qo_step_h1.restype = ctypes.c_int
    L.qo_step_h1.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, _u64p, _dp, _u8p, _u64p, _dp, _u8p, _ip]
    L.qo_search_h1.restype = ctypes.c_int
    L.qo_search_h1.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, _u64p, _u64p, _dp, _ip, _ip]
    L.qo_bf_search.restype = ctypes.c_int
    L.qo_bf_search.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64p,
                               _u64p, _dp, _u8p, _ip, _ip, _ip]
    L.qo_bf_multi.restype = ctypes.c_int
    L.qo_bf_multi.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              _u64p, _u64p, _dp, _ip, _ip]
    L.qo_num_threads.restype = ctypes.c_int
    L.qo_num_threads.argtypes = []
    return L


_override = None


def use_library(L) -> None:
    """Route the module functions to another loaded build (None restores the default)."""
    global _override
    _override = L


def lib():
    global _lib
    if _override is not None:
        return _override
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build(force=True)
        _lib = load(LIB_PATH)
    return _lib


def _W(N: int) -> int:
    return (N + 63) // 64


def _d(a):
    return a.ctypes.data_as(_dp)


def _u64(a):
    return a.ctypes.data_as(_u64p)


def _prep(J, h):
    J = np.ascontiguousarray(J, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    return J, h


def energy(J, h, x) -> float:
    """Eq. 1 for one state x (W uint64 words)."""
    J, h = _prep(J, h)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    return lib().qo_energy(len(h), _d(J), _d(h), _u64(x))


def flip_change(J, h, x, sites) -> float:
    J, h = _prep(J, h)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    s = np.ascontiguousarray(sites, dtype=np.int32)
    return lib().qo_flip_change(len(h), _d(J), _d(h), _u64(x), len(s), s.ctypes.data_as(_ip))


def field_change(J, h, x, sites) -> float:
    """The energy change of flipping one or two sites, from the local fields of x."""
    J, h = _prep(J, h)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    s = np.ascontiguousarray(sites, dtype=np.int32)
    return lib().qo_field_change(len(h), _d(J), _d(h), _u64(x), len(s), s.ctypes.data_as(_ip))


H1_FLIPS, H1_SINGLES, H1_EXCHANGE = 0, 1, 2


def step(J, h, M, bits, E=None, front=None, literal=False, fields=False, h1=H1_FLIPS):
    """One synchronous step.  Returns (bits, E, front, n_new).  fields=True takes
    every energy change from the parent's local fields (O(1) per flip instead of
    O(N)); the result is the same.  h1 selects the neighbourhood: single and
    pair flips (0), single flips only (1), exchanges of unequal spins (2)."""
    J, h = _prep(J, h)
    N = len(h)
    W = _W(N)
    bits = np.ascontiguousarray(bits, dtype=np.uint64).reshape(-1, W)
    n = bits.shape[0]
    if front is None:
        front = np.ones(n, dtype=np.uint8)
    front = np.ascontiguousarray(front, dtype=np.uint8)
    Ep = None
    if E is not None:
        E = np.ascontiguousarray(E, dtype=np.float64)
        Ep = _d(E)
    ob = np.zeros((M, W), dtype=np.uint64)
    oE = np.zeros(M, dtype=np.float64)
    of = np.zeros(M, dtype=np.uint8)
    nn = ctypes.c_int(0)
    if h1 == H1_FLIPS:
        fn = lib().qo_step_fields if fields else lib().qo_step
        r = fn(N, _d(J), _d(h), M, 1 if literal else 0, n, _u64(bits), Ep,
               front.ctypes.data_as(_u8p), _u64(ob), _d(oE), of.ctypes.data_as(_u8p), ctypes.byref(nn))
    else:
        r = lib().qo_step_h1(N, _d(J), _d(h), M, 1 if literal else 0, 1 if fields else 0, int(h1), n,
                             _u64(bits), Ep, front.ctypes.data_as(_u8p), _u64(ob), _d(oE),
                             of.ctypes.data_as(_u8p), ctypes.byref(nn))
    if r < 0:
        raise MemoryError("qo_step failed")
    k = nn.value
    return ob[:k], oE[:k], of[:k], r


def step_proposed(J, h, M, bits, E, parents, pair_lists, fields=False):
    """One learned-form step: S_t plus, for each parent index, its N single
    flips and only the listed pair flips (codes i | j << 16).  Returns
    (bits, E, front, n_new).  fields=True as in step()."""
    J, h = _prep(J, h)
    N = len(h)
    W = _W(N)
    bits = np.ascontiguousarray(bits, dtype=np.uint64).reshape(-1, W)
    E = np.ascontiguousarray(E, dtype=np.float64)
    par = np.ascontiguousarray(parents, dtype=np.int32)
    npairs = np.ascontiguousarray([len(p) for p in pair_lists], dtype=np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(p, np.uint32) for p in pair_lists])
                                if len(pair_lists) else np.zeros(0, np.uint32), dtype=np.uint32)
    if flat.size == 0:
        flat = np.zeros(1, np.uint32)
    ob = np.zeros((M, W), dtype=np.uint64)
    oE = np.zeros(M, dtype=np.float64)
    of = np.zeros(M, dtype=np.uint8)
    nn = ctypes.c_int(0)
    fn = lib().qo_step_proposed_fields if fields else lib().qo_step_proposed
    r = fn(N, _d(J), _d(h), M, bits.shape[0], _u64(bits), _d(E), len(par),
                               par.ctypes.data_as(_ip), npairs.ctypes.data_as(_ip),
                               flat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                               _u64(ob), _d(oE), of.ctypes.data_as(_u8p), ctypes.byref(nn))
    if r < 0:
        raise ValueError("qo_step_proposed failed (allocation or a malformed pair)")
    k = nn.value
    return ob[:k], oE[:k], of[:k], r


def search(J, h, M, x0, max_iters=1 << 30, literal=False, fields=False, h1=H1_FLIPS):
    """One search from x0.  Returns (bits, E, iters, stable)."""
    J, h = _prep(J, h)
    N = len(h)
    W = _W(N)
    x0 = np.ascontiguousarray(x0, dtype=np.uint64).reshape(W)
    ob = np.zeros((M, W), dtype=np.uint64)
    oE = np.zeros(M, dtype=np.float64)
    nn = ctypes.c_int(0)
    it = ctypes.c_int(0)
    if h1 == H1_FLIPS and not fields:
        r = lib().qo_search(N, _d(J), _d(h), M, int(max_iters), 1 if literal else 0, _u64(x0),
                            _u64(ob), _d(oE), ctypes.byref(nn), ctypes.byref(it))
    else:
        r = lib().qo_search_h1(N, _d(J), _d(h), M, int(max_iters), 1 if literal else 0, 1 if fields else 0,
                               int(h1), _u64(x0), _u64(ob), _d(oE), ctypes.byref(nn), ctypes.byref(it))
    if r < 0:
        raise MemoryError("qo_search failed")
    k = nn.value
    return ob[:k], oE[:k], it.value, bool(r)


def merge(N, M, lists):
    """Alg. 4 merge.  lists: sequence of (bits (n,W), E (n,)) pairs."""
    W = _W(N)
    counts = np.array([len(e) for _, e in lists], dtype=np.int32)
    if counts.sum() == 0:
        return np.zeros((0, W), np.uint64), np.zeros(0)
    bits = np.ascontiguousarray(np.concatenate([np.asarray(b, np.uint64).reshape(-1, W) for b, _ in lists]))
    E = np.ascontiguousarray(np.concatenate([np.asarray(e, np.float64) for _, e in lists]))
    ob = np.zeros((M, W), dtype=np.uint64)
    oE = np.zeros(M, dtype=np.float64)
    nn = ctypes.c_int(0)
    r = lib().qo_merge(N, M, len(lists), counts.ctypes.data_as(_ip), _u64(bits), _d(E),
                       _u64(ob), _d(oE), ctypes.byref(nn))
    if r < 0:
        raise MemoryError("qo_merge failed")
    k = nn.value
    return ob[:k], oE[:k]


def brute_lowest(J, h, K):
    """The K lowest states over all 2^N (N <= 40), sorted by (E, psi)."""
    J, h = _prep(J, h)
    N = len(h)
    W = _W(N)
    ob = np.zeros((K, W), dtype=np.uint64)
    oE = np.zeros(K, dtype=np.float64)
    nn = ctypes.c_int(0)
    r = lib().qo_brute_lowest(N, _d(J), _d(h), K, _u64(ob), _d(oE), ctypes.byref(nn))
    if r < 0:
        raise ValueError("qo_brute_lowest failed")
    k = nn.value
    return ob[:k], oE[:k]


def num_threads() -> int:
    return lib().qo_num_threads()


def bf_search(J, h, K, I, x0, h1=H1_FLIPS):
    """Alg. 3 (with Alg. 2's list update) from x0, a list of K + 1 entries and I
    iterations.  Returns (bits (n, W), E (n,), used (n,), born (n,), expanded):
    the real entries in list order and the number of iterations that expanded
    a state."""
    J, h = _prep(J, h)
    N = len(h)
    W = _W(N)
    x0 = np.ascontiguousarray(x0, dtype=np.uint64).reshape(W)
    cap = K + 1
    ob = np.zeros((cap, W), dtype=np.uint64)
    oE = np.zeros(cap, dtype=np.float64)
    ou = np.zeros(cap, dtype=np.uint8)
    obn = np.zeros(cap, dtype=np.int32)
    nn = ctypes.c_int(0)
    ex = ctypes.c_int(0)
    r = lib().qo_bf_search(N, _d(J), _d(h), int(h1), int(K), int(I), _u64(x0), _u64(ob), _d(oE),
                           ou.ctypes.data_as(_u8p), obn.ctypes.data_as(_ip), ctypes.byref(nn), ctypes.byref(ex))
    if r < 0:
        raise MemoryError("qo_bf_search failed")
    k = nn.value
    return ob[:k], oE[:k], ou[:k], obn[:k], ex.value


def bf_multi(J, h, K, I, x0s, h1=H1_FLIPS):
    """Alg. 4: len(x0s) searches merged.  Returns (bits, E, expanded per search)."""
    J, h = _prep(J, h)
    N = len(h)
    W = _W(N)
    x0s = np.ascontiguousarray(x0s, dtype=np.uint64).reshape(-1, W)
    L = x0s.shape[0]
    cap = K + 1
    ob = np.zeros((cap, W), dtype=np.uint64)
    oE = np.zeros(cap, dtype=np.float64)
    ex = np.zeros(L, dtype=np.int32)
    nn = ctypes.c_int(0)
    r = lib().qo_bf_multi(N, _d(J), _d(h), int(h1), int(K), int(I), L, _u64(x0s), _u64(ob), _d(oE),
                          ctypes.byref(nn), ex.ctypes.data_as(_ip))
    if r < 0:
        raise MemoryError("qo_bf_multi failed")
    k = nn.value
    return ob[:k], oE[:k], ex
