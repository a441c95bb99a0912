"""Pins of the oracle's special functions against mpmath at 40 digits."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import special

mp.mp.dps = 40


def _mp_e_chi(a, beta):
    A = mp.mpf(a)
    B = A * mp.mpf(beta)
    h1 = lambda z: mp.hankel1(1, z)
    h2 = lambda z: mp.hankel1(2, z)
    E = (A * h1(A) - B * h1(B)) / A ** 2
    C = h2(A) - mp.mpf(beta) ** 2 * h2(B)
    return complex(E), complex(C)


@pytest.mark.parametrize("beta", [0.5, 1.0 / math.sqrt(3.0), 0.3])
@pytest.mark.parametrize("a", [1e-7, 3e-5, 1e-3, 0.05, 0.4, 0.99, 1.01, 3.0, 17.0])
def test_e_chi_against_mpmath(a, beta):
    E, C = special.e_chi(np.array([a]), beta)
    Er, Cr = _mp_e_chi(a, beta)
    assert abs(E[0] - Er) <= 2e-14 * abs(Er)
    assert abs(C[0] - Cr) <= 2e-14 * abs(Cr)


def test_direct_form_loses_digits_at_small_argument():
    # the reason for the series: the direct difference is wrong at 1e-5
    a, beta = 1e-5, 0.5
    Er, Cr = _mp_e_chi(a, beta)
    Cd = special.chi_direct(np.array([a]), beta)[0]
    assert abs(Cd - Cr) > 1e-9 * abs(Cr)
    Cs = special.chi_series(np.array([a]), beta)[0]
    assert abs(Cs - Cr) < 1e-15 * abs(Cr)


@pytest.mark.parametrize("z", [1e-4, 0.3, 2.0, 7.5, 40.0, 300.0])
def test_hankel_library(z):
    for n, f in ((0, special.hankel0), (1, special.hankel1)):
        ref = complex(mp.hankel1(n, z))
        assert abs(f(z) - ref) <= 1e-14 * abs(ref)
