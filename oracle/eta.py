"""Bath coefficients eta for the oracle, by quadrature of their defining integrals.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module;
only tests/, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
bench.py may use it.

What is computed (Sec. 2, eqs. SD and inf_fun; the explicit eta formulas are
only cited there, so the window integrals below are the standard
Makri--Makarov construction written out from the influence functional):

* the bath response  alpha(t) = (1/pi) int_0^inf J(w) [coth(beta w/2) cos wt - i sin wt] dw,
  with J normalised as in eq. SD (J carries the factor pi/2 of the bath sum);
* its double time integral
      g(t) = int_0^t dt' int_0^t' dt'' alpha(t'')
           = (1/pi) int_0^inf J(w)/w^2 [coth(beta w/2)(1 - cos wt) + i (sin wt - wt)] dw,
  evaluated by adaptive quadrature (scipy.integrate.quad) of exactly this integrand;
* the eta coefficients as integrals of alpha over the Trotter windows of the two
  time points (interior points own a window of length dt centred on the point,
  the initial and the final point own the half window inside [0, t]):
      eta_int[0]  = g(dt)                                    (interior, self)
      eta_int[d]  = g((d+1)dt) - 2 g(d dt) + g((d-1)dt)      (interior x interior, lag d)
      eta_half[0] = g(dt/2)                                  (end point, self)
      eta_half[d] = g(d dt + h) - g(d dt) - g(d dt - h) + g((d-1)dt)   (end point x interior)
      eta_hh[d]   = g(d dt) - 2 g(d dt - h) + g((d-1)dt)     (initial x final point)
  with h = dt/2.  Each follows from  int_a^b dt' int_c^e dt'' alpha(t'-t'')
  = g(b-c) - g(a-c) - g(b-e) + g(a-e)  for disjoint windows [c,e] < [a,b].

Units: hbar = k_B = 1.  The spectral densities follow eq. SD; the
reorganisation energy used for the Brownian-oscillator peak is the
conventional  lambda = (1/pi) int J(w)/w dw  (eq. SD prints it without the
1/pi; with J carrying pi/2 the 1/pi is what makes lambda the energy shift).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import integrate


@dataclass(frozen=True)
class Bath:
    """Spectral density J = Ohmic part + Brownian-oscillator peaks.

    ohmic_alpha, ohmic_wc : J_O(w)  = (pi/2) alpha w exp(-w/wc)
    peaks                 : tuples (w0, gamma, lam) for
                            J_BO(w) = 2 lam gamma w0^2 w / ((w0^2 - w^2)^2 + gamma^2 w^2)
    The peak is the structured density of eq. sharpSD with Omega = w0 and
    2 pi kappa Omega = gamma.
    """
    ohmic_alpha: float = 0.0
    ohmic_wc: float = 1.0
    peaks: tuple = field(default_factory=tuple)

    def J(self, w):
        w = np.asarray(w, dtype=np.float64)
        out = np.zeros_like(w)
        if self.ohmic_alpha:
            out = out + 0.5 * math.pi * self.ohmic_alpha * w * np.exp(-w / self.ohmic_wc)
        for (w0, gam, lam) in self.peaks:
            out = out + 2.0 * lam * gam * w0 * w0 * w / ((w0 * w0 - w * w) ** 2 + (gam * w) ** 2)
        return out


def _breakpoints(bath: Bath, t: float):
    """Sub-interval ends for the quadrature: around each peak and the cutoff tail."""
    pts = [0.0]
    for (w0, gam, _lam) in bath.peaks:
        for k in (-40, -10, -3, -1, 0, 1, 3, 10, 40):
            x = w0 + k * gam
            if x > 0:
                pts.append(x)
    wc = bath.ohmic_wc if bath.ohmic_alpha else 0.0
    top = max([p for p in pts] + [1.0])
    if wc:
        top = max(top, 60.0 * wc)
    top = max(top, 20.0)
    # pieces of bounded length so that each holds a bounded number of periods of w t
    step = max(1.0, 2.0 * math.pi / max(t, 1e-3))
    n = int(math.ceil(top / step))
    pts += [k * top / n for k in range(1, n + 1)]
    pts = sorted(set(p for p in pts if 0.0 <= p <= top))
    return pts, top


def _integrand_re(w, bath: Bath, beta: float, t: float):
    # J/w^2 coth(beta w/2) (1 - cos wt), written with 1 - cos x = 2 sin^2(x/2)
    if w == 0.0:
        return 0.0
    j = float(bath.J(w))
    s = math.sin(0.5 * w * t)
    return j / (w * w) * (2.0 * s * s) / math.tanh(0.5 * beta * w)


def _integrand_im(w, bath: Bath, t: float):
    # J/w^2 (sin wt - wt); series for small wt where the difference cancels
    if w == 0.0:
        return 0.0
    x = w * t
    if abs(x) < 1e-3:
        x2 = x * x
        d = -x * x2 / 6.0 * (1.0 - x2 / 20.0 * (1.0 - x2 / 42.0))
    else:
        d = math.sin(x) - x
    return float(bath.J(w)) / (w * w) * d


def _tail(bath: Bath, beta: float, t: float, top: float) -> complex:
    """Contribution of [top, inf): the oscillating factors are integrated with
    Fourier-weighted quadrature (QAWF), the rest plainly."""
    jw2 = lambda w: float(bath.J(w)) / (w * w)
    jw2c = lambda w: jw2(w) / math.tanh(0.5 * beta * w)
    re = integrate.quad(jw2c, top, np.inf, epsabs=1e-18, epsrel=1e-12, limit=400)[0]
    re -= integrate.quad(jw2c, top, np.inf, weight='cos', wvar=t, epsabs=1e-18, limlst=200)[0]
    im = integrate.quad(jw2, top, np.inf, weight='sin', wvar=t, epsabs=1e-18, limlst=200)[0]
    im -= t * integrate.quad(lambda w: jw2(w) * w, top, np.inf, epsabs=1e-18,
                             epsrel=1e-12, limit=400)[0]
    return complex(re, im)


def g_of_t(bath: Bath, beta: float, t: float) -> complex:
    """g(t) = (1/pi) int_0^inf J/w^2 [coth(beta w/2)(1-cos wt) + i(sin wt - wt)] dw."""
    if t == 0.0:
        return 0.0j
    pts, top = _breakpoints(bath, t)
    re = 0.0
    im = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        r, _ = integrate.quad(_integrand_re, a, b, args=(bath, beta, t),
                              epsabs=1e-16, epsrel=1e-13, limit=400)
        i, _ = integrate.quad(_integrand_im, a, b, args=(bath, t),
                              epsabs=1e-16, epsrel=1e-13, limit=400)
        re += r
        im += i
    tail = _tail(bath, beta, t, top)
    return complex((re + tail.real) / math.pi, (im + tail.imag) / math.pi)


def eta_columns(bath: Bath, beta: float, dt: float, K: int) -> np.ndarray:
    """Return eta as a (3, K+1) complex array: rows eta_int, eta_half, eta_hh.

    eta_hh[0] is never used by the method (it would couple the initial and
    the final point at lag 0, i.e. a zero-length run); it is set to g(dt/2),
    the same as eta_half[0].
    """
    h = 0.5 * dt
    # g on the half-step grid: G[j] = g(j h), j = 0 .. 2K+2
    G = np.array([g_of_t(bath, beta, j * h) for j in range(2 * K + 3)], dtype=np.complex128)

    def g(n_half):
        return G[n_half]

    eta = np.zeros((3, K + 1), dtype=np.complex128)
    eta[0, 0] = g(2)
    eta[1, 0] = g(1)
    eta[2, 0] = g(1)
    for d in range(1, K + 1):
        eta[0, d] = g(2 * d + 2) - 2.0 * g(2 * d) + g(2 * d - 2)
        eta[1, d] = g(2 * d + 1) - g(2 * d) - g(2 * d - 1) + g(2 * d - 2)
        eta[2, d] = g(2 * d) - 2.0 * g(2 * d - 1) + g(2 * d - 2)
    return eta


def reorganisation_energy(bath: Bath) -> float:
    """lambda = (1/pi) int_0^inf J(w)/w dw, by quadrature."""
    pts, top = _breakpoints(bath, 1.0)
    tot = 0.0
    f = lambda w: float(bath.J(w)) / w if w > 0 else 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        tot += integrate.quad(f, a, b, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    tot += integrate.quad(f, top, np.inf, epsabs=1e-18, epsrel=1e-12, limit=400)[0]
    return tot / math.pi
