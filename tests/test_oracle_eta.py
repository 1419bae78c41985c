"""Pins of the oracle's bath coefficients (eq. SD, eq. inf_fun of Sec. 2).

g(t) is the oracle's quadrature of its defining integral; the pins below are
closed forms and independent window integrals, not re-evaluations of g.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import loggamma

from oracle.eta import Bath, eta_columns, g_of_t, reorganisation_energy


def ohmic_g_closed(alpha, wc, beta, t):
    """Closed form of g for J = (pi/2) alpha w exp(-w/wc):
    Im g = (alpha/2)(arctan(wc t) - wc t);
    Re g = (alpha/2)[ (1/2) ln(1 + wc^2 t^2) + ln( Gamma(1+u)^2 / |Gamma(1+u+i t/beta)|^2 ) ],
    u = 1/(beta wc)."""
    u = 1.0 / (beta * wc)
    re = 0.5 * alpha * (0.5 * math.log1p((wc * t) ** 2)
                        + 2.0 * loggamma(1.0 + u).real - 2.0 * loggamma(1.0 + u + 1j * t / beta).real)
    im = 0.5 * alpha * (math.atan(wc * t) - wc * t)
    return complex(re, im)


@pytest.mark.parametrize("alpha,wc,beta", [(0.1, 5.0, 5.0), (0.05, 5.0, 5.0), (0.3, 2.0, 0.7)])
@pytest.mark.parametrize("t", [0.05, 0.125, 0.25, 1.0, 3.3, 6.0])
def test_g_ohmic_closed_form(alpha, wc, beta, t):
    g = g_of_t(Bath(alpha, wc), beta, t)
    c = ohmic_g_closed(alpha, wc, beta, t)
    assert abs(g - c) < 2e-14 * max(1.0, abs(c))


def test_brownian_oscillator_reorganisation_energy():
    # (1/pi) int J_BO/w dw = lam, from  int_0^inf dw / ((w0^2-w^2)^2 + g^2 w^2) = pi/(2 g w0^2)
    for (w0, gam, lam) in [(1.0, 0.05, 0.1), (0.7, 0.3, 0.25), (2.0, 0.02, 0.1)]:
        assert abs(reorganisation_energy(Bath(peaks=((w0, gam, lam),))) - lam) < 1e-11 * lam
    # Ohmic: (1/pi) int (pi/2) alpha exp(-w/wc) dw = alpha wc / 2
    assert abs(reorganisation_energy(Bath(0.1, 5.0)) - 0.25) < 1e-13


def _window_coefficient(bath, beta, a, b, c, e):
    """eta of two disjoint windows [c,e] < [a,b]:  int_a^b dt' int_c^e dt'' alpha(t'-t''),
    evaluated in frequency space:  (1/pi) int J [coth(beta w/2) Re X - i Im X] dw with
    X = (e^{iwb} - e^{iwa}) (e^{-iwe} - e^{-iwc}) / w^2  (no use of g)."""
    def X(w):
        return (np.exp(1j * w * b) - np.exp(1j * w * a)) * (np.exp(-1j * w * e) - np.exp(-1j * w * c)) / (w * w)

    def fre(w):
        return float(bath.J(w)) / math.tanh(0.5 * beta * w) * X(w).real if w > 0 else 0.0

    def fim(w):
        return float(bath.J(w)) * X(w).imag if w > 0 else 0.0

    pts = [0.0]
    for (w0, gam, _l) in bath.peaks:
        pts += [max(1e-9, w0 - 10 * gam), w0, w0 + 10 * gam]
    top = 400.0
    pts += list(np.linspace(1.0, top, 200))
    pts = sorted(set(pts))
    re = sum(integrate.quad(fre, x, y, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
             for x, y in zip(pts[:-1], pts[1:]))
    im = sum(integrate.quad(fim, x, y, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
             for x, y in zip(pts[:-1], pts[1:]))
    return complex(re, -im) / math.pi


def test_eta_windows_direct_structured_bath():
    """Every eta column at lags d >= 1 equals the direct frequency-space window
    integral, for the structured bath (Ohmic + underdamped peak)."""
    bath = Bath(0.05, 5.0, ((1.0, 0.05, 0.1),))
    beta, dt, K = 5.0, 0.2, 6
    eta = eta_columns(bath, beta, dt, K)
    h = 0.5 * dt
    for d in range(1, K + 1):
        T = d * dt
        direct_int = _window_coefficient(bath, beta, T - h, T + h, -h, h)
        direct_half = _window_coefficient(bath, beta, T - h, T + h, 0.0, h)   # initial point x interior
        direct_half_f = _window_coefficient(bath, beta, T - h, T, -h, h)      # final point x interior
        direct_hh = _window_coefficient(bath, beta, T - h, T, 0.0, h)         # final x initial
        assert abs(eta[0, d] - direct_int) < 3e-12, d
        assert abs(eta[1, d] - direct_half) < 3e-12, d
        assert abs(eta[1, d] - direct_half_f) < 3e-12, d
        assert abs(eta[2, d] - direct_hh) < 3e-12, d


def test_eta_self_terms_and_tiling_sum_rule():
    """Self terms are g of the window length; the windows of N steps tile the
    ordered square, so the sum of all coefficient pairs is g(N dt)."""
    bath = Bath(0.1, 5.0)
    beta, dt, K = 5.0, 0.25, 6
    eta = eta_columns(bath, beta, dt, K)
    assert abs(eta[0, 0] - ohmic_g_closed(0.1, 5.0, 5.0, dt)) < 1e-14
    assert abs(eta[1, 0] - ohmic_g_closed(0.1, 5.0, 5.0, dt / 2)) < 1e-14
    for N in range(1, K + 1):
        tot = 2 * eta[1, 0] + (N - 1) * eta[0, 0]          # self terms of end points and interior points
        tot += eta[2, N]                                   # initial x final
        for d in range(1, N):
            tot += 2 * eta[1, d]                           # end point x interior, both ends
            tot += (N - 1 - d) * eta[0, d]                 # interior x interior
        assert abs(tot - ohmic_g_closed(0.1, 5.0, 5.0, N * dt)) < 1e-13, N
