"""ctypes binding of the C ABI in include/ising_search.h.

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  The names follow the C entry points.  Importing this module does not
need a GPU; creating a search does, and fails loudly when the library or the
device is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libising_search.so")

ISING_OK = 0
ISING_NOT_CONVERGED = 1
ISING_ERR_INVALID_ARG = -1
ISING_ERR_NO_DEVICE = -2
ISING_ERR_OUT_OF_MEMORY = -3
ISING_ERR_HIP = -4
ISING_ERR_BAD_STATE = -5
ISING_ERR_CAPACITY = -6

FORM_PLAIN = 0
FORM_SPLIT_BF16 = 1
FORM_LEARNED = 2

EXPORTED = (
    "ising_search_init",
    "ising_search_reset",
    "ising_search_step",
    "ising_search_run",
    "ising_search_get_states",
    "ising_search_get_search",
    "ising_search_set_search",
    "ising_search_get_stats",
    "ising_search_autotune",
    "ising_search_get_tuning",
    "ising_search_destroy",
    "ising_search_last_error",
)


class IsingConfig(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
        ("form", ctypes.c_int32),
        ("states_per_item", ctypes.c_int32),
        ("topk_factor", ctypes.c_int32),
        ("persistent", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class IsingStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_uint64),
        ("pair_evals", ctypes.c_uint64),
        ("single_evals", ctypes.c_uint64),
        ("frontier_states", ctypes.c_uint64),
        ("survivors", ctypes.c_uint64),
        ("retries", ctypes.c_uint64),
        ("fallbacks", ctypes.c_uint64),
        ("scan_launches", ctypes.c_uint64),
        ("scan_ms", ctypes.c_double),
        ("merge_ms", ctypes.c_double),
        ("frontier_ms", ctypes.c_double),
        ("prep_ms", ctypes.c_double),
        ("init_ms", ctypes.c_double),
        ("step_ms", ctypes.c_double),
        ("split_field_err", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class IsingError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.ising_search_init.restype = ctypes.c_int
    L.ising_search_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(IsingConfig), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.c_int32, ctypes.POINTER(vp), vp]
    L.ising_search_reset.restype = ctypes.c_int
    L.ising_search_reset.argtypes = [vp]
    L.ising_search_step.restype = ctypes.c_int
    L.ising_search_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.ising_search_run.restype = ctypes.c_int
    L.ising_search_run.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.ising_search_get_states.restype = ctypes.c_int
    L.ising_search_get_states.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.POINTER(ctypes.c_int32)]
    L.ising_search_get_search.restype = ctypes.c_int
    L.ising_search_get_search.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.POINTER(ctypes.c_int32)]
    L.ising_search_set_search.restype = ctypes.c_int
    L.ising_search_set_search.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32]
    L.ising_search_get_stats.restype = ctypes.c_int
    L.ising_search_get_stats.argtypes = [vp, ctypes.POINTER(IsingStats)]
    L.ising_search_autotune.restype = ctypes.c_int
    L.ising_search_autotune.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.ising_search_get_tuning.restype = ctypes.c_int
    L.ising_search_get_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.ising_search_destroy.restype = None
    L.ising_search_destroy.argtypes = [vp]
    L.ising_search_last_error.restype = ctypes.c_char_p
    L.ising_search_last_error.argtypes = []
    _lib = L
    return L


def last_error() -> str:
    return load().ising_search_last_error().decode()


def _check(rc: int, allow=(ISING_OK,)) -> int:
    if rc in allow:
        return rc
    raise IsingError(rc, last_error())


def current_stream_handle() -> Optional[int]:
    """The HIP stream torch is using on the current device, if torch has a GPU."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _words(N: int) -> int:
    return (N + 63) // 64


class IsingSearch:
    """One handle: B instances x L searches, kept-set size M."""

    def __init__(self, Ns: Sequence[int], Js, hs, init_bits, M: int, form: int = FORM_PLAIN,
                 max_iters: int = 0, states_per_item: int = 0, topk_factor: int = 8,
                 persistent: int = 0, timing: int = 0, stream: Optional[int] = None):
        L = load()
        self.Ns = [int(n) for n in Ns]
        self.B = len(self.Ns)
        self.M = int(M)
        self._keep = []
        Jp = (ctypes.c_void_p * self.B)()
        hp = (ctypes.c_void_p * self.B)()
        xp = (ctypes.c_void_p * self.B)()
        nL = None
        for b in range(self.B):
            Jb = np.ascontiguousarray(Js[b], dtype=np.float64)
            hb = np.ascontiguousarray(hs[b], dtype=np.float64)
            xb = np.ascontiguousarray(init_bits[b], dtype=np.uint64)
            W = _words(self.Ns[b])
            xb = xb.reshape(-1, W)
            if nL is None:
                nL = xb.shape[0]
            elif xb.shape[0] != nL:
                raise ValueError("every instance needs the same number of initial states")
            self._keep += [Jb, hb, xb]
            Jp[b] = Jb.ctypes.data
            hp[b] = hb.ctypes.data
            xp[b] = xb.ctypes.data
        self.L = int(nL)
        Narr = (ctypes.c_int32 * self.B)(*self.Ns)
        cfg = IsingConfig(M=self.M, max_iters=int(max_iters), form=int(form),
                          states_per_item=int(states_per_item), topk_factor=int(topk_factor),
                          persistent=int(persistent), timing=int(timing))
        if stream is None:
            stream = current_stream_handle()
        h = ctypes.c_void_p()
        _check(L.ising_search_init(ctypes.byref(h), ctypes.byref(cfg), self.B, Narr, Jp, hp, self.L, xp,
                                   ctypes.c_void_p(stream) if stream else None))
        self._h = h
        self._keep = []

    @classmethod
    def from_workload(cls, w, **kw):
        return cls([i.N for i in w.instances], [i.J for i in w.instances], [i.h for i in w.instances],
                   [i.init_bits for i in w.instances], w.M, **kw)

    @property
    def handle(self):
        return self._h

    def reset(self):
        _check(load().ising_search_reset(self._h))

    def step(self) -> int:
        n = ctypes.c_int32(0)
        _check(load().ising_search_step(self._h, ctypes.byref(n)))
        return n.value

    def run(self, max_iters: int = 0):
        it = ctypes.c_int32(0)
        rc = _check(load().ising_search_run(self._h, int(max_iters), ctypes.byref(it)),
                    allow=(ISING_OK, ISING_NOT_CONVERGED))
        return it.value, rc == ISING_OK

    def get_states(self, instance: int):
        W = _words(self.Ns[instance])
        bits = np.zeros((self.M, W), dtype=np.uint64)
        E = np.zeros(self.M, dtype=np.float64)
        n = ctypes.c_int32(0)
        _check(load().ising_search_get_states(self._h, int(instance), bits.ctypes.data, E.ctypes.data,
                                              ctypes.byref(n)))
        return bits[:n.value], E[:n.value]

    def get_search(self, search: int):
        W = _words(self.Ns[search // self.L])
        bits = np.zeros((self.M, W), dtype=np.uint64)
        E = np.zeros(self.M, dtype=np.float64)
        fr = np.zeros(self.M, dtype=np.uint8)
        n = ctypes.c_int32(0)
        _check(load().ising_search_get_search(self._h, int(search), bits.ctypes.data, E.ctypes.data,
                                              fr.ctypes.data, ctypes.byref(n)))
        k = n.value
        return bits[:k], E[:k], fr[:k]

    def set_search(self, search: int, bits, front=None):
        W = _words(self.Ns[search // self.L])
        bits = np.ascontiguousarray(bits, dtype=np.uint64).reshape(-1, W)
        fp = None
        if front is not None:
            front = np.ascontiguousarray(front, dtype=np.uint8)
            fp = front.ctypes.data
        _check(load().ising_search_set_search(self._h, int(search), bits.ctypes.data, fp, bits.shape[0]))

    def autotune(self) -> int:
        n = ctypes.c_int32(0)
        _check(load().ising_search_autotune(self._h, ctypes.byref(n)))
        return n.value

    def tuning(self):
        out = (ctypes.c_int32 * self.B)()
        _check(load().ising_search_get_tuning(self._h, out))
        return list(out)

    def stats(self) -> dict:
        st = IsingStats()
        _check(load().ising_search_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ising_search_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
