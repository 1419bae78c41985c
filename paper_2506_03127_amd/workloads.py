"""Synthetic workloads: model parameters and seeded generators only.

This module is the one place both the library's tests/bench and the oracle
take their inputs from.  It holds no step of the method: no propagator, no
bath coefficient, no path arithmetic -- only the parameters of the model
Hamiltonians and baths (Sec. 2 eq. tot_ham, eq. SD; Sec. 4.2 and 4.3 for the
kind of systems the paper runs) and seeded random draws.

State labels for a two-level system: index 0 is sigma_z = +1, so the
coupling eigenvalues are q = (+1, -1) and
    H_S = (eps/2) sigma_z + (Delta/2) sigma_x.
For three levels q = (+1, 0, -1).  hbar = k_B = 1, energies in units of Delta.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


def tls_hamiltonian(eps: float, delta: float) -> np.ndarray:
    return np.array([[0.5 * eps, 0.5 * delta], [0.5 * delta, -0.5 * eps]], dtype=np.complex128)


def random_hermitian(M: int, sigma: float, seed: int) -> np.ndarray:
    """Hermitian matrix with entries ~ N(0, sigma): real diagonal, complex off-diagonal."""
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, sigma, (M, M)) + 1j * rng.normal(0.0, sigma, (M, M))
    H = np.triu(A, 1)
    H = H + H.conj().T + np.diag(rng.normal(0.0, sigma, M))
    return H.astype(np.complex128)


@dataclass(frozen=True)
class BathSpec:
    """J(w) = (pi/2) alpha w exp(-w/wc)  +  sum over peaks (w0, gamma, lam) of
    2 lam gamma w0^2 w / ((w0^2 - w^2)^2 + gamma^2 w^2)."""
    ohmic_alpha: float = 0.0
    ohmic_wc: float = 1.0
    peaks: Tuple[Tuple[float, float, float], ...] = field(default_factory=tuple)


@dataclass(frozen=True)
class Workload:
    name: str
    H: np.ndarray
    q: np.ndarray
    bath: BathSpec
    beta: float
    dt: float
    K: int
    mask: Optional[Tuple[int, ...]]      # None: every lag 0..K-1 is on the mask
    theta: float
    rho0: np.ndarray
    n_steps: int
    mode: str = "pre"                    # "pre" or "post"

    @property
    def M(self) -> int:
        return self.H.shape[0]


def ground_projector(M: int) -> np.ndarray:
    r = np.zeros((M, M), dtype=np.complex128)
    r[0, 0] = 1.0
    return r


def spin_boson_ohmic(mode: str = "post", n_steps: int = 100) -> Workload:
    """Unbiased spin-boson, Ohmic bath; full memory K = 8, no mask, no filter
    (4^8 = 65536 stored paths at steady state)."""
    return Workload(name="spin_boson_ohmic_K8", H=tls_hamiltonian(0.0, 1.0),
                    q=np.array([1.0, -1.0]), bath=BathSpec(0.1, 5.0), beta=5.0, dt=0.25,
                    K=8, mask=None, theta=0.0, rho0=ground_projector(2), n_steps=n_steps,
                    mode=mode)


def structured_bath(n_steps: int = 1000, K: int = 24, n_exact: int = 12,
                    theta: float = 1e-8, w0: float = 1.0, gamma: float = 0.05,
                    lam: float = 0.1) -> Workload:
    """Biased TLS in an Ohmic bath plus an underdamped Brownian-oscillator peak;
    memory K = 24, mask keeping the last `n_exact` lags exact, theta = 1e-8."""
    return Workload(name=f"structured_bath_K{K}_E{n_exact}", H=tls_hamiltonian(0.5, 1.0),
                    q=np.array([1.0, -1.0]),
                    bath=BathSpec(0.05, 5.0, ((w0, gamma, lam),)), beta=5.0, dt=0.2, K=K,
                    mask=tuple(range(n_exact)), theta=theta, rho0=ground_projector(2),
                    n_steps=n_steps, mode="pre")


def long_memory(n_steps: int = 1000) -> Workload:
    """The structured bath with memory K = 40 and theta = 1e-9; the mask keeps lags
    0..11 exact and lags 16, 24 and 32 of the tail (80-bit histories; the merge
    positions are not a contiguous run, so it takes the hash-table merge)."""
    w = structured_bath(n_steps=n_steps, K=40, theta=1e-9)
    return Workload(name="long_memory_K40_E12_16_24_32", H=w.H, q=w.q, bath=w.bath, beta=w.beta,
                    dt=w.dt, K=40, mask=tuple(range(12)) + (16, 24, 32), theta=1e-9, rho0=w.rho0,
                    n_steps=n_steps, mode="pre")


def batched_scan(n_inst: int = 64, seed: int = 11, n_steps: int = 1000, K: int = 24, n_exact: int = 12,
                 theta: float = 1e-8) -> Tuple[Workload, Tuple[BathSpec, ...]]:
    """The structured bath at n_inst bath parameter points: peak frequency w0
    uniform in [0.5, 2.0] and width gamma drawn from {0.02, 0.05, 0.1} (seeded);
    everything else as `structured_bath`.  Returns the shared workload (its bath
    is the first point's) and the points' baths."""
    rng = np.random.default_rng(seed)
    w0 = rng.uniform(0.5, 2.0, n_inst)
    gam = rng.choice(np.array([0.02, 0.05, 0.1]), n_inst)
    base = structured_bath(n_steps=n_steps, K=K, n_exact=n_exact, theta=theta)
    baths = tuple(BathSpec(base.bath.ohmic_alpha, base.bath.ohmic_wc, ((float(a), float(g), 0.1),))
                  for a, g in zip(w0, gam))
    wl = Workload(name=f"batched_scan_{n_inst}x_structured_bath_K{K}_E{n_exact}", H=base.H, q=base.q,
                  bath=baths[0], beta=base.beta, dt=base.dt, K=K, mask=base.mask, theta=theta,
                  rho0=base.rho0, n_steps=n_steps, mode="pre")
    return wl, baths


def four_level(seed: int = 11, K: int = 5, n_exact: int = 3, theta: float = 1e-7,
               n_steps: int = 40) -> Workload:
    """Four-level system (16 forward/backward pairs) with a seeded random Hermitian
    H_S (entries ~ N(0, 0.5)) and equally spaced coupling eigenvalues."""
    return Workload(name=f"four_level_K{K}", H=random_hermitian(4, 0.5, seed),
                    q=np.array([1.5, 0.5, -0.5, -1.5]),
                    bath=BathSpec(0.05, 5.0, ((1.0, 0.05, 0.1),)), beta=5.0, dt=0.2, K=K,
                    mask=tuple(range(n_exact)), theta=theta, rho0=ground_projector(4),
                    n_steps=n_steps, mode="pre")


def three_level(seed: int = 7, K: int = 16, n_exact: int = 6, theta: float = 1e-8,
                n_steps: int = 200) -> Workload:
    """Three-level system with a seeded random Hermitian H_S (entries ~ N(0, 0.5))."""
    return Workload(name=f"three_level_K{K}", H=random_hermitian(3, 0.5, seed),
                    q=np.array([1.0, 0.0, -1.0]),
                    bath=BathSpec(0.05, 5.0, ((1.0, 0.05, 0.1),)), beta=5.0, dt=0.2, K=K,
                    mask=tuple(range(n_exact)), theta=theta, rho0=ground_projector(3),
                    n_steps=n_steps, mode="pre")
