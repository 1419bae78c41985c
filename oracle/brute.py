"""Full enumeration of the memory-truncated QUAPI path sum (tiny sizes only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

rho(N)[x_N] = sum over all pair sequences x_0..x_N of
    rho0[x_0] * prod_{k=1..N} S(x_k, x_{k-1})
             * exp( - sum_{k=0..N} sum_{k'=max(0,k-K)..k} ds[x_k] (Re eta_kk' ds[x_k'] + i Im eta_kk' ss[x_k']) )
(eqs. quapi_red_rho, SysP0, SysP and inf_fun of Sec. 2, with the memory cut of
Sec. 2 dropping every pair of points more than K steps apart).  The
coefficient eta_kk' is taken by the type of the two windows:
    k = k' = 0 or k = k' = N       -> eta_half[0]    (half window, self)
    k = k' otherwise               -> eta_int[0]
    k' = 0 and k = N               -> eta_hh[N]      (initial x final point)
    k' = 0 or k = N (not both)     -> eta_half[k-k']
    otherwise                      -> eta_int[k-k']
U = exp(-i H dt) is taken from scipy.linalg.expm here (the iterative oracle
uses its own power series), S(x', x) = U[a'][a] conj(U[b'][b]).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def brute_rho(H, q, dt, K, eta, rho0, N):
    H = np.asarray(H, dtype=np.complex128)
    M = H.shape[0]
    P = M * M
    q = np.asarray(q, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.complex128).reshape(3, K + 1)
    rho0 = np.asarray(rho0, dtype=np.complex128).reshape(M, M)
    if N == 0:
        return rho0.copy()
    U = expm(-1j * dt * H)
    a_of = np.arange(P) // M
    b_of = np.arange(P) % M
    S = U[a_of[:, None], a_of[None, :]] * np.conj(U[b_of[:, None], b_of[None, :]])
    ds = q[a_of] - q[b_of]
    ss = q[a_of] + q[b_of]

    n_paths = P ** (N + 1)
    idx = np.arange(n_paths, dtype=np.int64)
    x = np.empty((N + 1, n_paths), dtype=np.int64)
    for k in range(N + 1):                 # x[k] = digit k of the path index
        x[k] = (idx // P ** k) % P

    w = rho0.reshape(-1)[x[0]].astype(np.complex128)
    for k in range(1, N + 1):
        w = w * S[x[k], x[k - 1]]

    def coeff(k, kp):
        d = k - kp
        if d == 0:
            return eta[1, 0] if (k == 0 or k == N) else eta[0, 0]
        if kp == 0 and k == N:
            return eta[2, d]
        if kp == 0 or k == N:
            return eta[1, d]
        return eta[0, d]

    expo = np.zeros(n_paths, dtype=np.complex128)
    for k in range(N + 1):
        for kp in range(max(0, k - K), k + 1):
            c = coeff(k, kp)
            expo += -ds[x[k]] * (c.real * ds[x[kp]] + 1j * c.imag * ss[x[kp]])
    w = w * np.exp(expo)
    rho = np.zeros(P, dtype=np.complex128)
    np.add.at(rho, x[N], w)
    return rho.reshape(M, M)
