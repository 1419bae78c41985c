"""CPU FP64 oracle for the MACGIC-iQUAPI path propagation.

TEST INFRASTRUCTURE ONLY: only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of bench.py may import this package.  It shares no code
with the HIP library (``paper_2506_03127_amd``) and never imports it.

* ``quapi_oracle.cpp`` -- the iterative propagation (pre- and post-merging),
  built into ``liboracle.so`` and driven through ctypes here;
* ``eta.py``           -- bath coefficients by quadrature of their definition;
* ``brute.py``         -- full enumeration of the truncated path sum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "quapi_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

PRE = 0
POST = 1
DEFAULT_QBITS = 32
DEFAULT_AMB_EPS = 1e-12


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("H", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("dt", ctypes.c_double), ("K", ctypes.c_int), ("eta", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("n_mask", ctypes.c_int), ("theta", ctypes.c_double),
                ("rho0", ctypes.c_void_p), ("mode", ctypes.c_int), ("qbits", ctypes.c_int),
                ("amb_eps", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_longlong), ("n_children", ctypes.c_longlong),
                ("n_survivors", ctypes.c_longlong), ("n_stored", ctypes.c_longlong),
                ("n_amb_rep", ctypes.c_longlong), ("n_amb_theta", ctypes.c_longlong),
                ("dropped_abs", ctypes.c_double), ("theta_margin", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        vp, ci, cd, cll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [ctypes.POINTER(_Params)]
        L.oracle_step.argtypes = [vp, ci]
        L.oracle_time.argtypes = [vp]
        L.oracle_rho.argtypes = [vp, ci, vp]
        L.oracle_stats_at.argtypes = [vp, ci, ctypes.POINTER(Stats)]
        L.oracle_groups.restype = cll
        L.oracle_groups.argtypes = [vp, vp, vp, cll]
        L.oracle_stored.restype = cll
        L.oracle_stored.argtypes = [vp, vp, vp, cll]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_propagator.argtypes = [ci, vp, cd, vp]
        L.oracle_merge_demo.argtypes = [vp, vp, ci, ci, vp, ci, ci, vp, vp]
        L.oracle_could_flip.argtypes = [vp, vp, ci, cd]
        L.oracle_flag_demo.argtypes = [vp, vp, ci, ci, vp, ci, ci, cd, vp, vp]
        _lib = L
    return _lib


def _c128(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One propagation run of the oracle.

    H (M x M complex), q (M), dt, K = dk_max, eta ((3, K+1) complex: eta_int,
    eta_half, eta_hh), mask (sorted lags with 0 and 1, or None for all K lags),
    theta, rho0 (M x M), mode PRE or POST.
    """

    def __init__(self, H, q, dt, K, eta, rho0, mask=None, theta=0.0, mode=PRE,
                 qbits=DEFAULT_QBITS, amb_eps=DEFAULT_AMB_EPS):
        self.H = _c128(H)
        self.M = self.H.shape[0]
        self.P = self.M * self.M
        self.q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
        self.K = int(K)
        self.eta = _c128(eta, (3, self.K + 1))
        self.rho0 = _c128(rho0, (self.M, self.M))
        self.mask = None if mask is None else np.ascontiguousarray(np.asarray(mask, dtype=np.int32))
        p = _Params()
        p.M = self.M
        p.H = self.H.ctypes.data
        p.q = self.q.ctypes.data
        p.dt = float(dt)
        p.K = self.K
        p.eta = self.eta.ctypes.data
        p.mask = None if self.mask is None else self.mask.ctypes.data
        p.n_mask = 0 if self.mask is None else len(self.mask)
        p.theta = float(theta)
        p.rho0 = self.rho0.ctypes.data
        p.mode = int(mode)
        p.qbits = int(qbits)
        p.amb_eps = float(amb_eps)
        self._h = lib().oracle_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle_create rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return lib().oracle_time(self._h)

    def step(self, n: int = 1):
        if lib().oracle_step(self._h, int(n)) != 0:
            raise RuntimeError("oracle_step failed")

    def rho(self, t: int) -> np.ndarray:
        out = np.zeros((self.M, self.M), dtype=np.complex128)
        if lib().oracle_rho(self._h, int(t), out.ctypes.data) != 0:
            raise IndexError(t)
        return out

    def rho_history(self) -> np.ndarray:
        return np.stack([self.rho(t) for t in range(self.t + 1)])

    def stats(self, t: int) -> dict:
        s = Stats()
        if lib().oracle_stats_at(self._h, int(t), ctypes.byref(s)) != 0:
            raise IndexError(t)
        return s.as_dict()

    def _dump(self, fn):
        n = fn(self._h, None, None, 0)
        hist = np.zeros((max(n, 1), self.K), dtype=np.uint8)
        w = np.zeros(max(n, 1), dtype=np.complex128)
        fn(self._h, hist.ctypes.data, w.ctypes.data, n)
        return hist[:n], w[:n]

    def groups(self):
        """Groups the next step expands: (hist (n, K) uint8, weights (n,) complex)."""
        return self._dump(lib().oracle_groups)

    def stored(self):
        return self._dump(lib().oracle_stored)


def propagator(H, dt) -> np.ndarray:
    H = _c128(H)
    M = H.shape[0]
    U = np.zeros((M, M), dtype=np.complex128)
    lib().oracle_propagator(M, H.ctypes.data, float(dt), U.ctypes.data)
    return U


def merge_demo(hist, w, positions, qbits=DEFAULT_QBITS):
    """Merge explicit paths on `positions`; returns (rep index per group, sums)."""
    hist = np.ascontiguousarray(np.asarray(hist, dtype=np.uint8))
    w = _c128(w)
    n, L = hist.shape
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32))
    rep = np.zeros(n, dtype=np.int32)
    sums = np.zeros(n, dtype=np.complex128)
    ng = lib().oracle_merge_demo(hist.ctypes.data, w.ctypes.data, n, L, pos.ctypes.data,
                                 len(pos), int(qbits), rep.ctypes.data, sums.ctypes.data)
    return rep[:ng], sums[:ng]


def could_flip(winner, other, qbits=DEFAULT_QBITS, eps=DEFAULT_AMB_EPS) -> bool:
    """Whether a relative perturbation eps of |winner|^2 and |other|^2 could
    change the representative choice between them (the oracle's decision log)."""
    a = np.array([complex(winner).real, complex(winner).imag])
    b = np.array([complex(other).real, complex(other).imag])
    return bool(lib().oracle_could_flip(a.ctypes.data, b.ctypes.data, int(qbits), float(eps)))


def flag_demo(hist, w, positions, qbits=DEFAULT_QBITS, eps=DEFAULT_AMB_EPS):
    """Merge explicit paths on `positions`; returns (rep index, ambiguous flag) per group."""
    hist = np.ascontiguousarray(np.asarray(hist, dtype=np.uint8))
    w = _c128(w)
    n, L = hist.shape
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32))
    rep = np.zeros(n, dtype=np.int32)
    amb = np.zeros(n, dtype=np.int32)
    ng = lib().oracle_flag_demo(hist.ctypes.data, w.ctypes.data, n, L, pos.ctypes.data, len(pos),
                                int(qbits), float(eps), rep.ctypes.data, amb.ctypes.data)
    return rep[:ng], amb[:ng].astype(bool)
