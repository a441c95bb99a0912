"""Special functions for the oracle (test infrastructure only).

The fundamental solution of 2D elastodynamics (equation of the fundamental
solution, Section 3) is built from Hankel functions of the first kind at the
transverse and longitudinal wavenumbers.  Writing a = k_T r, b = k_L r and
beta = k_L / k_T, it takes the form

    G = (i / 4 mu) [ psi I + chi e e^T ],  e = (x - y)/r,
    psi = H0(a) - E,      E   = (a H1(a) - b H1(b)) / a^2,
    chi = H2(a) - beta^2 H2(b),

obtained by expanding the second derivatives in the definition of G.  Both E
and chi contain 1/a^2 singular pieces that cancel exactly, so their direct
evaluation loses about |log10(a^2)| digits.  Below ``SERIES_SWITCH`` the
oracle evaluates them from the ascending (Frobenius) series of H1 and H2 with
the cancelling terms removed analytically.

Hankel functions themselves are the library routine ``scipy.special.hankel1``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as _sp

EULER_GAMMA = 0.57721566490153286060651209008240243
SERIES_SWITCH = 1.0
_NTERMS = 14


def hankel0(z):
    """H_0^(1)(z) for real z > 0."""
    return _sp.hankel1(0, z)


def hankel1(z):
    """H_1^(1)(z) for real z > 0."""
    return _sp.hankel1(1, z)


def _digamma_int(m: int) -> float:
    """psi(m) for integer m >= 1: -gamma + sum_{j<m} 1/j."""
    return -EULER_GAMMA + sum(1.0 / j for j in range(1, m))


def e_series(a, beta):
    """E = (a H1(a) - b H1(b))/a^2 with b = beta a, from the ascending series.

    a H1(a) = -2i/pi + 2 sum_k (-1)^k (a^2/4)^(k+1)/(k!(k+1)!) c_k(a),
    c_k(z) = 1 + (2i/pi) log(z/2) - (i/pi)(psi(k+1) + psi(k+2)).
    The constant -2i/pi cancels in the difference.
    """
    a = np.asarray(a, dtype=np.float64)
    w = a * a / 4.0
    la = np.log(a / 2.0)
    lb = math.log(beta)
    out = np.zeros(a.shape, dtype=np.complex128)
    wk = np.ones_like(a)
    for k in range(_NTERMS):
        ck = 1.0 + 2j / math.pi * la - 1j / math.pi * (_digamma_int(k + 1) + _digamma_int(k + 2))
        b2 = beta ** (2 * k + 2)
        term = ((1.0 - b2) * ck - b2 * (2j / math.pi) * lb) / (2.0 * math.factorial(k) * math.factorial(k + 1))
        out += ((-1) ** k) * wk * term
        wk = wk * w
    return out


def chi_series(a, beta):
    """chi = H2(a) - beta^2 H2(beta a) from the ascending series.

    H2(z) = -(i/pi)(4/z^2 + 1) + sum_k (-1)^k (z/2)^(2k+2)/(k!(k+2)!) d_k(z),
    d_k(z) = 1 + (2i/pi) log(z/2) - (i/pi)(psi(k+1) + psi(k+3)).
    The 4/z^2 pieces cancel; the constants leave -(i/pi)(1 - beta^2).
    """
    a = np.asarray(a, dtype=np.float64)
    w = a * a / 4.0
    la = np.log(a / 2.0)
    lb = math.log(beta)
    out = np.full(a.shape, -1j / math.pi * (1.0 - beta * beta), dtype=np.complex128)
    wk = w.copy()
    for k in range(_NTERMS):
        dk = 1.0 + 2j / math.pi * la - 1j / math.pi * (_digamma_int(k + 1) + _digamma_int(k + 3))
        b4 = beta ** (2 * k + 4)
        term = ((1.0 - b4) * dk - b4 * (2j / math.pi) * lb) / (math.factorial(k) * math.factorial(k + 2))
        out += ((-1) ** k) * wk * term
        wk = wk * w
    return out


def e_direct(a, beta):
    b = beta * a
    return (a * hankel1(a) - b * hankel1(b)) / (a * a)


def chi_direct(a, beta):
    b = beta * a
    h2a = 2.0 * hankel1(a) / a - hankel0(a)
    h2b = 2.0 * hankel1(b) / b - hankel0(b)
    return h2a - beta * beta * h2b


def e_chi(a, beta):
    """(E, chi) with the series below SERIES_SWITCH and the direct form above."""
    a = np.asarray(a, dtype=np.float64)
    small = a < SERIES_SWITCH
    e = np.empty(a.shape, dtype=np.complex128)
    c = np.empty(a.shape, dtype=np.complex128)
    if np.any(small):
        e[small] = e_series(a[small], beta)
        c[small] = chi_series(a[small], beta)
    big = ~small
    if np.any(big):
        e[big] = e_direct(a[big], beta)
        c[big] = chi_direct(a[big], beta)
    return e, c
