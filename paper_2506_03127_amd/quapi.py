"""ctypes binding of libquapi.so (include/quapi.h), argument marshalling only.

Every function here forwards to the C ABI of the same name; every step of the
propagation runs in the library's HIP kernels.  If the library is not built
the import fails: there is no fallback.  PyTorch, when used, only supplies the
stream (``stream=torch.cuda.current_stream().cuda_stream``).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libquapi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "quapi.h")

QUAPI_OK = 0
QUAPI_EINVAL = -1
QUAPI_ENOMEM = -2
QUAPI_EDEVICE = -3
QUAPI_ESTATE = -4
QUAPI_EUNSUPPORTED = -5
QUAPI_PRE = 0
QUAPI_POST = 1
QUAPI_FP64 = 0
QUAPI_FP32_LOG = 1
QUAPI_MERGE_AUTO = 0
QUAPI_MERGE_DIRECT = 1
QUAPI_MERGE_BUCKETED = 2
QUAPI_MERGE_HASH = 3
QUAPI_MERGE_PARTITION = 4


class c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class quapi_params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("H", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("dt", ctypes.c_double), ("dk_max", ctypes.c_int), ("eta", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("n_mask", ctypes.c_int), ("theta", ctypes.c_double),
                ("rho0", ctypes.c_void_p), ("mode", ctypes.c_int), ("qbits", ctypes.c_int),
                ("max_groups", ctypes.c_longlong), ("max_steps", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("precision", ctypes.c_int), ("merge", ctypes.c_int)]


class quapi_stepstat_t(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int), ("n_groups", ctypes.c_longlong),
                ("n_children", ctypes.c_longlong), ("n_survivors", ctypes.c_longlong),
                ("n_stored", ctypes.c_longlong), ("dropped_abs", ctypes.c_double)]


class quapi_info_t(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("P", ctypes.c_int), ("K", ctypes.c_int), ("L", ctypes.c_int),
                ("bits_per_point", ctypes.c_int), ("record_bytes", ctypes.c_int),
                ("capacity", ctypes.c_longlong), ("device_bytes", ctypes.c_size_t),
                ("precision", ctypes.c_int), ("hash_merge", ctypes.c_int), ("n_instances", ctypes.c_int),
                ("store", ctypes.c_int)]


class quapi_bath(ctypes.Structure):
    _fields_ = [("ohmic_alpha", ctypes.c_double), ("ohmic_wc", ctypes.c_double),
                ("n_peaks", ctypes.c_int), ("peaks", ctypes.c_void_p)]


class QuapiError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_2506_03127_amd/_build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, ci, cd, cll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        L.quapi_create.argtypes = [ctypes.POINTER(quapi_params), ctypes.POINTER(vp)]
        L.quapi_step.argtypes = [vp, ci]
        L.quapi_step_graph.argtypes = [vp, ci]
        L.quapi_sync.argtypes = [vp]
        L.quapi_time.argtypes = [vp, ctypes.POINTER(ci)]
        L.quapi_rho.argtypes = [vp, ci, vp]
        L.quapi_rho_history.argtypes = [vp, ci, ci, vp]
        L.quapi_step_stats.argtypes = [vp, ci, ci, vp]
        L.quapi_groups.argtypes = [vp, cll, vp, vp, ctypes.POINTER(cll)]
        L.quapi_create_batch.argtypes = [ctypes.POINTER(quapi_params), ci, vp, vp, ctypes.POINTER(vp)]
        L.quapi_batch_rho_history.argtypes = [vp, ci, ci, ci, vp]
        L.quapi_batch_step_stats.argtypes = [vp, ci, ci, ci, vp]
        L.quapi_batch_groups.argtypes = [vp, ci, cll, vp, vp, ctypes.POINTER(cll)]
        L.quapi_batch_rho_all.argtypes = [vp, ci, ci, vp]
        L.quapi_set_chunk_run.argtypes = [vp, ci]
        L.quapi_autotune.argtypes = [vp, ci, ctypes.POINTER(ci)]
        L.quapi_mlp_create.argtypes = [ci, ci, ci, ci, ci, ctypes.c_ulonglong, vp, ctypes.POINTER(vp)]
        L.quapi_mlp_n_params.argtypes = [vp, ctypes.POINTER(cll)]
        L.quapi_mlp_set_params.argtypes = [vp, vp, cll]
        L.quapi_mlp_get_params.argtypes = [vp, vp, cll]
        L.quapi_mlp_get_grads.argtypes = [vp, vp, cll]
        L.quapi_mlp_forward.argtypes = [vp, vp, ci, vp]
        L.quapi_mlp_backward.argtypes = [vp, vp, vp, ci, vp]
        L.quapi_mlp_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        L.quapi_mlp_sync.argtypes = [vp]
        L.quapi_mlp_destroy.restype = None
        L.quapi_mlp_destroy.argtypes = [vp]
        L.quapi_reset.argtypes = [vp]
        L.quapi_info.argtypes = [vp, ctypes.POINTER(quapi_info_t)]
        L.quapi_stream.restype = vp
        L.quapi_stream.argtypes = [vp]
        L.quapi_strerror.restype = ctypes.c_char_p
        L.quapi_strerror.argtypes = [ci]
        L.quapi_destroy.restype = None
        L.quapi_destroy.argtypes = [vp]
        L.quapi_eta.argtypes = [ctypes.POINTER(quapi_bath), cd, cd, ci, vp]
        L.quapi_propagator.argtypes = [ci, vp, cd, vp]
        L.quapi_profile_begin.argtypes = [vp, ci]
        L.quapi_profile_end.argtypes = [vp, ci, vp, vp, ctypes.POINTER(ci)]
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/quapi.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(quapi_\w+)\s*\(", src)))


def strerror(code: int) -> str:
    return lib().quapi_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc != QUAPI_OK:
        raise QuapiError(rc, where)


def _c128(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a if shape is None else a.reshape(shape)


# ------------------------------------------------------------------ C ABI, one to one
def _params(H, q, dt, dk_max, eta, rho0, mask, theta, mode, qbits, max_groups, max_steps, stream,
            precision, merge=QUAPI_MERGE_AUTO):
    """quapi_params and the arrays its pointers refer to (kept alive by the caller)."""
    H = _c128(H)
    M = H.shape[0]
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    eta = None if eta is None else _c128(eta, (3, int(dk_max) + 1))
    rho0 = _c128(rho0, (M, M))
    m = None if mask is None else np.ascontiguousarray(np.asarray(mask, dtype=np.int32))
    p = quapi_params()
    p.M = M
    p.H = H.ctypes.data
    p.q = q.ctypes.data
    p.dt = float(dt)
    p.dk_max = int(dk_max)
    p.eta = None if eta is None else eta.ctypes.data
    p.mask = None if m is None else m.ctypes.data
    p.n_mask = 0 if m is None else len(m)
    p.theta = float(theta)
    p.rho0 = rho0.ctypes.data
    p.mode = int(mode)
    p.qbits = int(qbits)
    p.max_groups = int(max_groups)
    p.max_steps = int(max_steps)
    p.stream = None if stream is None else int(stream)
    p.precision = int(precision)
    p.merge = int(merge)
    return p, (H, q, eta, rho0, m)


def quapi_create(H, q, dt, dk_max, eta, rho0, mask=None, theta=0.0, mode=QUAPI_PRE, qbits=-1,
                 max_groups=0, max_steps=0, stream=None, precision=QUAPI_FP64, merge=QUAPI_MERGE_AUTO) -> int:
    p, keep = _params(H, q, dt, dk_max, eta, rho0, mask, theta, mode, qbits, max_groups, max_steps,
                      stream, precision, merge)
    h = ctypes.c_void_p()
    _check(lib().quapi_create(ctypes.byref(p), ctypes.byref(h)), "quapi_create")
    return h.value


def quapi_create_batch(H, q, dt, dk_max, etas, rho0, mask=None, theta=0.0, mode=QUAPI_PRE, qbits=-1,
                       max_groups=0, max_steps=0, stream=None, H_batch=None, merge=QUAPI_MERGE_AUTO) -> int:
    """etas: (n_inst, 3, dk_max + 1) complex, one eta table per instance; H_batch:
    (n_inst, M, M) complex, one Hamiltonian per instance, or None (H for all)."""
    etas = _c128(etas)
    etas = etas.reshape(-1, 3, int(dk_max) + 1)
    p, keep = _params(H, q, dt, dk_max, None, rho0, mask, theta, mode, qbits, max_groups, max_steps,
                      stream, QUAPI_FP64, merge)
    hb = None if H_batch is None else _c128(H_batch).reshape(etas.shape[0], p.M, p.M)
    h = ctypes.c_void_p()
    _check(lib().quapi_create_batch(ctypes.byref(p), int(etas.shape[0]), etas.ctypes.data,
                                    None if hb is None else hb.ctypes.data, ctypes.byref(h)),
           "quapi_create_batch")
    return h.value


def quapi_run_static(H, q, dt, dk_max, eta, rho0, n_steps: int, rho_out_ptr: int, mask=None, theta=0.0,
                     mode=QUAPI_PRE, qbits=-1, stream=None):
    """The propagation with no device allocation (see include/quapi.h): rho(0..n_steps)
    into the device buffer at rho_out_ptr ((n_steps+1) * M * M complex128), enqueued on
    stream; returns without waiting."""
    p, keep = _params(H, q, dt, dk_max, eta, rho0, mask, theta, mode, qbits, 0, 0, stream, QUAPI_FP64)
    _check(lib().quapi_run_static(ctypes.byref(p), int(n_steps), ctypes.c_void_p(int(rho_out_ptr))),
           "quapi_run_static")


def quapi_step(ctx, n_steps: int):
    _check(lib().quapi_step(ctx, int(n_steps)), "quapi_step")


def quapi_step_graph(ctx, n_steps: int):
    _check(lib().quapi_step_graph(ctx, int(n_steps)), "quapi_step_graph")


def quapi_sync(ctx):
    _check(lib().quapi_sync(ctx), "quapi_sync")


def quapi_time(ctx) -> int:
    t = ctypes.c_int()
    _check(lib().quapi_time(ctx, ctypes.byref(t)), "quapi_time")
    return t.value


def quapi_rho(ctx, t: int, M: int) -> np.ndarray:
    out = np.zeros((M, M), dtype=np.complex128)
    _check(lib().quapi_rho(ctx, int(t), out.ctypes.data), "quapi_rho")
    return out


def quapi_rho_history(ctx, t0: int, n: int, M: int) -> np.ndarray:
    out = np.zeros((n, M, M), dtype=np.complex128)
    _check(lib().quapi_rho_history(ctx, int(t0), int(n), out.ctypes.data), "quapi_rho_history")
    return out


def quapi_step_stats(ctx, t0: int, n: int) -> list:
    arr = (quapi_stepstat_t * max(n, 1))()
    _check(lib().quapi_step_stats(ctx, int(t0), int(n), arr), "quapi_step_stats")
    return [{k: getattr(arr[i], k) for k, _ in quapi_stepstat_t._fields_} for i in range(n)]


def quapi_groups(ctx, K: int):
    n = ctypes.c_longlong()
    _check(lib().quapi_groups(ctx, 0, None, None, ctypes.byref(n)), "quapi_groups")
    hist = np.zeros((max(n.value, 1), K), dtype=np.uint8)
    w = np.zeros(max(n.value, 1), dtype=np.complex128)
    _check(lib().quapi_groups(ctx, n.value, hist.ctypes.data, w.ctypes.data, ctypes.byref(n)),
           "quapi_groups")
    return hist[:n.value], w[:n.value]


def quapi_batch_rho_history(ctx, inst: int, t0: int, n: int, M: int) -> np.ndarray:
    out = np.zeros((n, M, M), dtype=np.complex128)
    _check(lib().quapi_batch_rho_history(ctx, int(inst), int(t0), int(n), out.ctypes.data),
           "quapi_batch_rho_history")
    return out


def quapi_batch_rho_all(ctx, t0: int, n: int, n_inst: int, M: int) -> np.ndarray:
    out = np.zeros((n, n_inst, M, M), dtype=np.complex128)
    _check(lib().quapi_batch_rho_all(ctx, int(t0), int(n), out.ctypes.data), "quapi_batch_rho_all")
    return out


def quapi_set_chunk_run(ctx, run: int):
    _check(lib().quapi_set_chunk_run(ctx, int(run)), "quapi_set_chunk_run")


def quapi_autotune(ctx, n_steps: int) -> int:
    r = ctypes.c_int()
    _check(lib().quapi_autotune(ctx, int(n_steps), ctypes.byref(r)), "quapi_autotune")
    return r.value


def quapi_batch_step_stats(ctx, inst: int, t0: int, n: int) -> list:
    arr = (quapi_stepstat_t * max(n, 1))()
    _check(lib().quapi_batch_step_stats(ctx, int(inst), int(t0), int(n), arr), "quapi_batch_step_stats")
    return [{k: getattr(arr[i], k) for k, _ in quapi_stepstat_t._fields_} for i in range(n)]


def quapi_batch_groups(ctx, inst: int, K: int):
    n = ctypes.c_longlong()
    _check(lib().quapi_batch_groups(ctx, int(inst), 0, None, None, ctypes.byref(n)), "quapi_batch_groups")
    hist = np.zeros((max(n.value, 1), K), dtype=np.uint8)
    w = np.zeros(max(n.value, 1), dtype=np.complex128)
    _check(lib().quapi_batch_groups(ctx, int(inst), n.value, hist.ctypes.data, w.ctypes.data, ctypes.byref(n)),
           "quapi_batch_groups")
    return hist[:n.value], w[:n.value]


def quapi_reset(ctx):
    _check(lib().quapi_reset(ctx), "quapi_reset")


def quapi_info(ctx) -> dict:
    i = quapi_info_t()
    _check(lib().quapi_info(ctx, ctypes.byref(i)), "quapi_info")
    return {k: getattr(i, k) for k, _ in quapi_info_t._fields_}


def quapi_stream(ctx) -> int:
    return lib().quapi_stream(ctx) or 0


def quapi_destroy(ctx):
    if ctx:
        lib().quapi_destroy(ctx)


def quapi_profile_begin(ctx, max_launches: int):
    _check(lib().quapi_profile_begin(ctx, int(max_launches)), "quapi_profile_begin")


def quapi_profile_end(ctx, cap: int):
    """(step_ms, plan_ms): per recorded step, the step kernel's and the planner's duration."""
    step = np.zeros(max(int(cap), 1))
    plan = np.zeros(max(int(cap), 1))
    n = ctypes.c_int(0)
    _check(lib().quapi_profile_end(ctx, int(cap), step.ctypes.data, plan.ctypes.data, ctypes.byref(n)),
           "quapi_profile_end")
    k = min(n.value, int(cap))
    return step[:k], plan[:k]


def quapi_eta(ohmic_alpha, ohmic_wc, peaks, beta, dt, dk_max) -> np.ndarray:
    pk = np.ascontiguousarray(np.asarray(peaks if peaks else [], dtype=np.float64).reshape(-1))
    b = quapi_bath()
    b.ohmic_alpha = float(ohmic_alpha)
    b.ohmic_wc = float(ohmic_wc)
    b.n_peaks = len(pk) // 3
    b.peaks = pk.ctypes.data if len(pk) else None
    out = np.zeros((3, int(dk_max) + 1), dtype=np.complex128)
    _check(lib().quapi_eta(ctypes.byref(b), float(beta), float(dt), int(dk_max), out.ctypes.data),
           "quapi_eta")
    return out


def quapi_propagator(H, dt) -> np.ndarray:
    H = _c128(H)
    U = np.zeros_like(H)
    _check(lib().quapi_propagator(H.shape[0], H.ctypes.data, float(dt), U.ctypes.data),
           "quapi_propagator")
    return U


# ------------------------------------------------------------------ convenience
class Propagator:
    """Owns one context; thin object wrapper over the functions above."""

    def __init__(self, H, q, dt, dk_max, eta, rho0, **kw):
        self.M = np.asarray(H).shape[0]
        self.K = int(dk_max)
        self.ctx = quapi_create(H, q, dt, dk_max, eta, rho0, **kw)

    def step(self, n=1):
        quapi_step(self.ctx, n)

    def step_graph(self, n):
        """n steps as one HIP graph, replayed when a later call starts at the
        same step (see quapi_step_graph)."""
        quapi_step_graph(self.ctx, n)

    def sync(self):
        quapi_sync(self.ctx)

    @property
    def t(self) -> int:
        return quapi_time(self.ctx)

    def rho(self, t):
        return quapi_rho(self.ctx, t, self.M)

    def rho_history(self, t0=0, n=None):
        if n is None:
            n = self.t + 1 - t0
        return quapi_rho_history(self.ctx, t0, n, self.M)

    def stats(self, t0=1, n=None):
        if n is None:
            n = self.t - t0 + 1
        return quapi_step_stats(self.ctx, t0, n)

    def groups(self):
        return quapi_groups(self.ctx, self.K)

    def reset(self):
        quapi_reset(self.ctx)

    def info(self):
        return quapi_info(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            quapi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPropagator:
    """Owns one batched context: n_inst instances with their own eta tables."""

    def __init__(self, H, q, dt, dk_max, etas, rho0, **kw):
        self.M = np.asarray(H).shape[0]
        self.K = int(dk_max)
        self.n_inst = int(np.asarray(etas).reshape(-1, 3, self.K + 1).shape[0])
        self.ctx = quapi_create_batch(H, q, dt, dk_max, etas, rho0, **kw)

    def step(self, n=1):
        quapi_step(self.ctx, n)

    def step_graph(self, n):
        """n steps as one HIP graph, replayed when a later call starts at the
        same step (see quapi_step_graph)."""
        quapi_step_graph(self.ctx, n)

    def sync(self):
        quapi_sync(self.ctx)

    @property
    def t(self) -> int:
        return quapi_time(self.ctx)

    def rho_history(self, inst, t0=0, n=None):
        n = quapi_time(self.ctx) + 1 - t0 if n is None else n
        return quapi_batch_rho_history(self.ctx, inst, t0, n, self.M)

    def stats(self, inst, t0=1, n=None):
        n = quapi_time(self.ctx) + 1 - t0 if n is None else n
        return quapi_batch_step_stats(self.ctx, inst, t0, n)

    def groups(self, inst):
        return quapi_batch_groups(self.ctx, inst, self.K)

    def rho_all(self, t0=0, n=None):
        """rho(t) of every instance: (n, n_inst, M, M)."""
        n = quapi_time(self.ctx) + 1 - t0 if n is None else n
        return quapi_batch_rho_all(self.ctx, t0, n, self.n_inst, self.M)

    def set_chunk_run(self, run):
        quapi_set_chunk_run(self.ctx, run)

    def autotune(self, n_steps):
        """Fastest chunk run length over n_steps from t = 0; leaves the context at t = 0."""
        return quapi_autotune(self.ctx, n_steps)

    def reset(self):
        quapi_reset(self.ctx)

    def info(self):
        return quapi_info(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            quapi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ surrogate network
class MLP:
    """The library's multilayer perceptron (quapi_mlp_*).  Batches are torch
    float32 tensors on the GPU (memory only; the arithmetic is the library's)."""

    def __init__(self, n_in, width, depth, n_out, max_batch, seed=1, stream=None):
        self.n_in, self.width, self.depth, self.n_out = int(n_in), int(width), int(depth), int(n_out)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        _check(lib().quapi_mlp_create(self.n_in, self.width, self.depth, self.n_out, self.max_batch,
                                      ctypes.c_ulonglong(seed), None if stream is None else int(stream),
                                      ctypes.byref(h)), "quapi_mlp_create")
        self.h = h.value
        n = ctypes.c_longlong()
        _check(lib().quapi_mlp_n_params(self.h, ctypes.byref(n)), "quapi_mlp_n_params")
        self.n_params = n.value

    def layers(self):
        """(fan_in, fan_out) of each layer, in the flat parameter order."""
        dims = [self.n_in] + [self.width] * self.depth + [self.n_out]
        return list(zip(dims[:-1], dims[1:]))

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().quapi_mlp_get_params(self.h, out.ctypes.data, self.n_params), "quapi_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        _check(lib().quapi_mlp_set_params(self.h, p.ctypes.data, self.n_params), "quapi_mlp_set_params")

    def grads(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().quapi_mlp_get_grads(self.h, out.ctypes.data, self.n_params), "quapi_mlp_get_grads")
        return out

    def forward(self, x, y):
        """y[:B] = network(x[:B]) (device tensors, float32, contiguous)."""
        _check(lib().quapi_mlp_forward(self.h, x.data_ptr(), int(x.shape[0]), y.data_ptr()), "quapi_mlp_forward")

    def backward(self, x, target, loss=None):
        _check(lib().quapi_mlp_backward(self.h, x.data_ptr(), target.data_ptr(), int(x.shape[0]),
                                        None if loss is None else loss.data_ptr()), "quapi_mlp_backward")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().quapi_mlp_adam(self.h, lr, beta1, beta2, eps), "quapi_mlp_adam")

    def sync(self):
        _check(lib().quapi_mlp_sync(self.h), "quapi_mlp_sync")

    def close(self):
        if getattr(self, "h", None):
            lib().quapi_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
