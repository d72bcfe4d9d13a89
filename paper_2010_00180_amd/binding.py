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
FLAG_RECORD_PROPOSALS = 1
FLAG_SITE_BOUND = 2
FLAG_FP16_SCAN = 4
FLAG_SINGLE_FLIPS = 8
FLAG_EXCHANGE = 16
SCORER_NETWORK = 0
SCORER_FIELDS = 1
SCORER_UNIFORM = 2
MLP_NPARAM = 4545

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
    "ising_search_set_scorer",
    "ising_search_set_trace",
    "ising_search_get_trace_count",
    "ising_search_get_proposals",
    "ising_search_topk",
    "ising_mlp_num_params",
    "ising_mlp_workspace_bytes",
    "ising_mlp_forward",
    "ising_mlp_loss_grad",
    "ising_mlp_adam",
    "ising_mlp_train",
    "ising_mlp_loss_grad_noalloc",
    "ising_brute_lowest",
    "ising_bestfirst",
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
        ("flags", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32),
        ("surv_capacity", ctypes.c_int32),
        ("tile_cache", ctypes.c_char_p),
        ("mlp_weights", ctypes.c_char_p),
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
        ("scored_pairs", ctypes.c_uint64),
        ("ranked_states", ctypes.c_uint64),
        ("trace_samples", ctypes.c_uint64),
        ("learn_ms", ctypes.c_double),
        ("bounded_states", ctypes.c_uint64),
        ("surv_capacity", ctypes.c_uint64),
        ("bound_ms", ctypes.c_double),
        ("field_bytes", ctypes.c_uint64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def save_mlp_weights(path: str, params) -> None:
    """Write the network's parameter vector as the file cfg.mlp_weights reads:
    MLP_NPARAM little-endian FP32 values."""
    params = np.ascontiguousarray(params, dtype="<f4").reshape(-1)
    if params.size != MLP_NPARAM:
        raise ValueError(f"the network has {MLP_NPARAM} parameters, got {params.size}")
    with open(path, "wb") as f:
        f.write(params.tobytes())


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
    i32, i64, u64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
    L.ising_search_set_scorer.restype = ctypes.c_int
    L.ising_search_set_scorer.argtypes = [vp, i32, vp, u64]
    L.ising_search_set_trace.restype = ctypes.c_int
    L.ising_search_set_trace.argtypes = [vp, vp, vp, i64, i32, f32, u64]
    L.ising_search_get_trace_count.restype = ctypes.c_int
    L.ising_search_get_trace_count.argtypes = [vp, ctypes.POINTER(i64)]
    L.ising_search_get_proposals.restype = ctypes.c_int
    L.ising_search_get_proposals.argtypes = [vp, i32, vp, vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ising_search_topk.restype = i32
    L.ising_search_topk.argtypes = [vp]
    L.ising_mlp_num_params.restype = i32
    L.ising_mlp_num_params.argtypes = []
    L.ising_mlp_workspace_bytes.restype = i64
    L.ising_mlp_workspace_bytes.argtypes = []
    L.ising_mlp_forward.restype = ctypes.c_int
    L.ising_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    L.ising_mlp_loss_grad.restype = ctypes.c_int
    L.ising_mlp_loss_grad.argtypes = [vp, vp, vp, i64, f32, vp, vp, vp, i64, vp]
    L.ising_bestfirst.restype = ctypes.c_int
    L.ising_bestfirst.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(vp), i32,
                                  ctypes.POINTER(vp), i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.ising_brute_lowest.restype = ctypes.c_int
    L.ising_brute_lowest.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, vp,
                                     ctypes.POINTER(i32), vp]
    L.ising_mlp_loss_grad_noalloc.restype = ctypes.c_int
    L.ising_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, i64, f32, vp, vp, vp]
    L.ising_mlp_adam.restype = ctypes.c_int
    L.ising_mlp_adam.argtypes = [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]
    L.ising_mlp_train.restype = ctypes.c_int
    L.ising_mlp_train.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i32, f32, f32, u64, vp, vp, i64, vp]
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


def brute_lowest(Js, hs, K: int, stream: Optional[int] = None):
    """The K lowest states of every instance over all 2^N states (N <= 40),
    sorted by (E, psi), enumerated on the GPU.  Returns a list of
    (bits (k, 1) uint64, E (k,)) per instance."""
    L = load()
    B = len(hs)
    keep = []
    Jp = (ctypes.c_void_p * B)()
    hp = (ctypes.c_void_p * B)()
    Ns = []
    for b in range(B):
        Jb = np.ascontiguousarray(Js[b], dtype=np.float64)
        hb = np.ascontiguousarray(hs[b], dtype=np.float64)
        keep += [Jb, hb]
        Jp[b] = Jb.ctypes.data
        hp[b] = hb.ctypes.data
        Ns.append(len(hb))
    Narr = (ctypes.c_int32 * B)(*Ns)
    bits = np.zeros((B, int(K)), np.uint64)
    E = np.zeros((B, int(K)), np.float64)
    cnt = (ctypes.c_int32 * B)()
    if stream is None:
        stream = current_stream_handle()
    _check(L.ising_brute_lowest(B, Narr, Jp, hp, int(K), bits.ctypes.data, E.ctypes.data, cnt,
                                ctypes.c_void_p(stream) if stream else None))
    return [(bits[b, :cnt[b]].reshape(-1, 1).copy(), E[b, :cnt[b]].copy()) for b in range(B)]


def bestfirst(Js, hs, init_bits, K: int, I: int, flags: int = 0, searches: bool = False,
              stream: Optional[int] = None):
    """Alg. 3 / Alg. 4 on the GPU.  init_bits[b]: L initial states (one word
    each, N <= 64).  Returns a dict: 'merged' = [(bits (n, 1), E (n,))] per
    instance, 'expanded' (B, L), 'kernel_ms'; with searches=True also
    'searches' = [[(bits, E, used, born)] * L] per instance."""
    L = load()
    B = len(hs)
    keep = []
    Jp = (ctypes.c_void_p * B)()
    hp = (ctypes.c_void_p * B)()
    xp = (ctypes.c_void_p * B)()
    Ns = []
    nL = None
    for b in range(B):
        Jb = np.ascontiguousarray(Js[b], dtype=np.float64)
        hb = np.ascontiguousarray(hs[b], dtype=np.float64)
        xb = np.ascontiguousarray(np.asarray(init_bits[b], dtype=np.uint64).reshape(-1))
        if nL is None:
            nL = len(xb)
        elif len(xb) != nL:
            raise ValueError("every instance needs the same number of initial states")
        keep += [Jb, hb, xb]
        Jp[b], hp[b], xp[b] = Jb.ctypes.data, hb.ctypes.data, xb.ctypes.data
        Ns.append(len(hb))
    K1 = int(K) + 1
    mb = np.zeros((B, K1), np.uint64)
    mE = np.zeros((B, K1), np.float64)
    mc = np.zeros(B, np.int32)
    ex = np.zeros((B, nL), np.int32)
    ms = ctypes.c_float(0.0)
    if searches:
        sb = np.zeros((B, nL, K1), np.uint64)
        sE = np.zeros((B, nL, K1), np.float64)
        su = np.zeros((B, nL, K1), np.uint8)
        sn = np.zeros((B, nL, K1), np.int32)
        sc = np.zeros((B, nL), np.int32)
        sptr = [sb.ctypes.data, sE.ctypes.data, su.ctypes.data, sn.ctypes.data, sc.ctypes.data]
    else:
        sptr = [None] * 5
    if stream is None:
        stream = current_stream_handle()
    _check(L.ising_bestfirst(B, (ctypes.c_int32 * B)(*Ns), Jp, hp, int(nL), xp, int(K), int(I), int(flags),
                             mb.ctypes.data, mE.ctypes.data, mc.ctypes.data, *sptr, ex.ctypes.data,
                             ctypes.byref(ms), ctypes.c_void_p(stream) if stream else None))
    out = {"merged": [(mb[b, :mc[b]].reshape(-1, 1).copy(), mE[b, :mc[b]].copy()) for b in range(B)],
           "expanded": ex, "kernel_ms": ms.value}
    if searches:
        out["searches"] = [[(sb[b, l, :sc[b, l]].reshape(-1, 1).copy(), sE[b, l, :sc[b, l]].copy(),
                             su[b, l, :sc[b, l]].copy(), sn[b, l, :sc[b, l]].copy()) for l in range(nL)]
                           for b in range(B)]
    return out


class IsingSearch:
    """One handle: B instances x L searches, kept-set size M."""

    def __init__(self, Ns: Sequence[int], Js, hs, init_bits, M: int, form: int = FORM_PLAIN,
                 max_iters: int = 0, states_per_item: int = 0, topk_factor: int = 8,
                 persistent: int = 0, timing: int = 0, stream: Optional[int] = None, flags: int = 0,
                 graph_steps: int = 0, surv_capacity: int = 0, tile_cache: Optional[str] = None,
                 mlp_weights: Optional[str] = None):
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
                          persistent=int(persistent), timing=int(timing), flags=int(flags),
                          graph_steps=int(graph_steps), surv_capacity=int(surv_capacity),
                          tile_cache=os.fsencode(tile_cache) if tile_cache else None,
                          mlp_weights=os.fsencode(mlp_weights) if mlp_weights else None)
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

    # learned-proposal form
    def set_scorer(self, scorer: int, params=None, seed: int = 0):
        pp = None
        if params is not None:
            params = np.ascontiguousarray(params, dtype=np.float32)
            if params.size != MLP_NPARAM:
                raise ValueError(f"the network has {MLP_NPARAM} parameters, got {params.size}")
            pp = params.ctypes.data
        _check(load().ising_search_set_scorer(self._h, int(scorer), pp, ctypes.c_uint64(seed)))

    def set_trace(self, feat_ptr: int, label_ptr: int, capacity: int, pairs_per_state: int = 8,
                  rate: float = 1.0, seed: int = 0):
        """Device buffers (pointers, e.g. torch tensors' data_ptr()) of capacity x 4 FP32 and capacity bytes."""
        _check(load().ising_search_set_trace(self._h, ctypes.c_void_p(feat_ptr or None),
                                             ctypes.c_void_p(label_ptr or None), int(capacity),
                                             int(pairs_per_state), float(rate), ctypes.c_uint64(seed)))

    def trace_count(self) -> int:
        c = ctypes.c_int64(0)
        _check(load().ising_search_get_trace_count(self._h, ctypes.byref(c)))
        return c.value

    def topk(self) -> int:
        return int(load().ising_search_topk(self._h))

    def get_proposals(self, search: int, max_parents: Optional[int] = None):
        """Returns (mode, [(parent_bits (W,), pair codes (n,))]) of the last step of one search."""
        W = _words(self.Ns[search // self.L])
        K = self.topk()
        mp = self.M if max_parents is None else int(max_parents)
        pb = np.zeros((mp, W), dtype=np.uint64)
        pr = np.zeros((mp, K), dtype=np.uint32)
        npr = np.zeros(mp, dtype=np.int32)
        n = ctypes.c_int32(0)
        md = ctypes.c_int32(0)
        _check(load().ising_search_get_proposals(self._h, int(search), pb.ctypes.data, pr.ctypes.data,
                                                 npr.ctypes.data, mp, ctypes.byref(n), ctypes.byref(md)))
        return md.value, [(pb[k].copy(), pr[k, :npr[k]].copy()) for k in range(n.value)]

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ising_search_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------- training of the scoring network
# Thin wrappers over the device entry points: every argument is a device
# pointer (an integer such as torch's data_ptr()), work goes on `stream`.

def mlp_workspace_bytes() -> int:
    return int(load().ising_mlp_workspace_bytes())


def _vp(p):
    return ctypes.c_void_p(int(p)) if p else None


def mlp_forward(params, feat, n, logits, stream=None):
    _check(load().ising_mlp_forward(_vp(params), _vp(feat), int(n), _vp(logits), _vp(stream)))


def mlp_loss_grad(params, feat, label, n, pos_weight, grad, loss, workspace, workspace_bytes, stream=None):
    _check(load().ising_mlp_loss_grad(_vp(params), _vp(feat), _vp(label), int(n), float(pos_weight), _vp(grad),
                                      _vp(loss), _vp(workspace), int(workspace_bytes), _vp(stream)))


def mlp_loss_grad_noalloc(params, feat, label, n, pos_weight, grad, loss, stream=None):
    _check(load().ising_mlp_loss_grad_noalloc(_vp(params), _vp(feat), _vp(label), int(n), float(pos_weight),
                                              _vp(grad), _vp(loss), _vp(stream)))


def mlp_adam(params, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().ising_mlp_adam(_vp(params), _vp(m), _vp(v), _vp(grad), int(t), float(lr), float(beta1),
                                 float(beta2), float(eps), _vp(stream)))


def mlp_train(params, m, v, feat, label, n, batch, steps, t0, lr, pos_weight, seed, loss, workspace,
              workspace_bytes, stream=None):
    _check(load().ising_mlp_train(_vp(params), _vp(m), _vp(v), _vp(feat), _vp(label), int(n), int(batch),
                                  int(steps), int(t0), float(lr), float(pos_weight), ctypes.c_uint64(seed), _vp(loss),
                                  _vp(workspace), int(workspace_bytes), _vp(stream)))
