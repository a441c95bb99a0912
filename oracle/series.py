"""Closed-form series for plane-wave scattering by a traction-free circular
cavity (oracle; test infrastructure only).  Not in the paper: it is the
textbook exact solution of the boundary value problem of Section 2 for a
circle, used to pin the whole discretisation.

Helmholtz potentials u = grad phi + curl(psi e_z), with
u_r = d_r phi + (1/r) d_theta psi,  u_theta = (1/r) d_theta phi - d_r psi.
Incident P-wave along +x_1: phi^I = exp(i k_L x_1)/(i k_L)
  = (1/(i k_L)) sum_n eps_n i^n J_n(k_L r) cos(n theta),  eps_0 = 1, eps_n = 2.
Scattered: phi^S = sum A_n H_n(k_L r) cos(n theta), psi^S = sum B_n H_n(k_T r) sin(n theta).
Per mode, sigma_rr = -lambda k_L^2 phi_n + 2 mu (phi_n'' + n psi_n'/r - n psi_n/r^2)
and sigma_rtheta = mu (-2 n phi_n'/r + 2 n phi_n/r^2 - psi_n'' + psi_n'/r - n^2 psi_n/r^2),
both zero at r = a.  Time factor exp(-i omega t), H = H^(1) (outgoing).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as sp

from .kernels import Material


def _z(kind, n, z, der):
    """Bessel J (kind 'j') or Hankel H^(1) (kind 'h') of order n, derivative der."""
    f = sp.jv if kind == "j" else sp.hankel1
    if der == 0:
        return f(n, z)
    if der == 1:
        return 0.5 * (f(n - 1, z) - f(n + 1, z))
    # Bessel equation: Z'' = -Z'/z - (1 - n^2/z^2) Z
    return -_z(kind, n, z, 1) / z - (1.0 - n * n / (z * z)) * f(n, z)


def _mode_stress(mat, n, r, phi, dphi, ddphi, psi, dpsi, ddpsi):
    lam, mu, kL = mat.lam, mat.mu, mat.kL
    srr = -lam * kL ** 2 * phi + 2 * mu * (ddphi + n * dpsi / r - n * psi / r ** 2)
    srt = mu * (-2 * n * dphi / r + 2 * n * phi / r ** 2 - ddpsi + dpsi / r - n * n * psi / r ** 2)
    return srr, srt


def coefficients(mat: Material, a: float = 1.0, nmax=None):
    """Scattering coefficients (A_n, B_n), n = 0..nmax, for a unit P-wave along +x_1."""
    kL, kT = mat.kL, mat.kT
    if nmax is None:
        nmax = int(kT * a + 30)
    A = np.zeros(nmax + 1, dtype=np.complex128)
    B = np.zeros(nmax + 1, dtype=np.complex128)
    for n in range(nmax + 1):
        eps = 1.0 if n == 0 else 2.0
        c = eps * (1j ** n) / (1j * kL)
        # incident potential phi_n = c J_n(kL r)
        inc = _mode_stress(mat, n, a, c * _z("j", n, kL * a, 0), c * kL * _z("j", n, kL * a, 1),
                           c * kL ** 2 * _z("j", n, kL * a, 2), 0, 0, 0)
        sa = _mode_stress(mat, n, a, _z("h", n, kL * a, 0), kL * _z("h", n, kL * a, 1),
                          kL ** 2 * _z("h", n, kL * a, 2), 0, 0, 0)
        sb = _mode_stress(mat, n, a, 0, 0, 0, _z("h", n, kT * a, 0), kT * _z("h", n, kT * a, 1),
                          kT ** 2 * _z("h", n, kT * a, 2))
        if n == 0:
            A[0] = -inc[0] / sa[0]
        else:
            M = np.array([[sa[0], sb[0]], [sa[1], sb[1]]])
            A[n], B[n] = np.linalg.solve(M, -np.array(inc))
    return A, B


def displacement(mat: Material, x, a: float = 1.0, nmax=None):
    """Total displacement (u_1, u_2) at points x (|x| >= a) for a unit plane
    P-wave along +x_1 scattered by the traction-free circle of radius a."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    A, B = coefficients(mat, a, nmax)
    kL, kT = mat.kL, mat.kT
    r = np.hypot(x[:, 0], x[:, 1])
    th = np.arctan2(x[:, 1], x[:, 0])
    ur = np.zeros(len(r), dtype=np.complex128)
    ut = np.zeros(len(r), dtype=np.complex128)
    for n in range(len(A)):
        eps = 1.0 if n == 0 else 2.0
        c = eps * (1j ** n) / (1j * kL)
        phi = c * _z("j", n, kL * r, 0) + A[n] * _z("h", n, kL * r, 0)
        dphi = c * kL * _z("j", n, kL * r, 1) + A[n] * kL * _z("h", n, kL * r, 1)
        psi = B[n] * _z("h", n, kT * r, 0)
        dpsi = B[n] * kT * _z("h", n, kT * r, 1)
        ur += (dphi + n * psi / r) * np.cos(n * th)
        ut += (-n * phi / r - dpsi) * np.sin(n * th)
    u1 = ur * np.cos(th) - ut * np.sin(th)
    u2 = ur * np.sin(th) + ut * np.cos(th)
    return np.stack([u1, u2], axis=1)
