"""Per-point integrands of the regularised Galerkin Burton-Miller form
(oracle; test infrastructure only).

Problem (Section 2): in-plane time-harmonic elasticity outside a traction-free
cavity, normal n pointing into the cavity.  The time factor is read as
exp(-i omega t) so that H0^(1) is outgoing (the paper writes exp(+i omega t);
the other reading only conjugates results).

Boundary integral equation (equation of the Burton-Miller BIE, Section 3):
(D + 1/2 + alpha N) u = u^I + alpha T u^I with the double-layer operator D
(principal value) and its traction N (finite part), built on the fundamental
solution G of the equation of the fundamental solution.

Galerkin entries (Section 5.2).  The paper regularises N following a
reference that is not reproduced in it.  The oracle uses the following
weakly singular form, obtained from the 2D identity for the traction operator

    T^n u = 2 mu d_s(J u) + (lambda + 2 mu) n div u + mu (curl u) t,   t = J n,

with J the rotation by +90 degrees and d_s the derivative along t, the facts
div_y G_i. = d_{y_i} Phi_L / (lambda + 2 mu) and curl_y G_i. = (J grad_y Phi_T)_i / mu
(Phi_k = (i/4) H0(k r)), and integration by parts along the closed polygons
(the hat functions are continuous, so no boundary terms appear).  With
Q = mu G - Phi_T I, dPhi = Phi_L - Phi_T, psi a test hat at x and phi a
trial hat at y (primes are d_s along t):

  D_st = int int [ psi phi' (Phi_T J - 2 Q J^T)
                   + psi phi ((d_{n_y} Phi_T) I + grad_y dPhi n_y^T) ]
  N_st = int int [ 4 mu psi' phi' J Q J^T
                   - 2 mu psi' phi ((d_{n_y} Phi_T) J + (J grad_y dPhi) n_y^T)
                   + 2 mu psi phi' ((d_{n_x} Phi_T) J - n_x (J grad_x dPhi)^T)
                   + rho omega^2 psi phi (n_x n_y^T Phi_L + t_x t_y^T Phi_T) ]

Every kernel above is at most logarithmically singular on coincident
elements, bounded there otherwise, and O(1/r) only at the shared corner of
two adjacent elements.  The oracle's tests check this form against the
direct kernels T_y G and T_x T_y G by finite differences on separated
elements, against the static rigid-body identities, and (through the full
solver) against the closed-form circular-cavity series.
"""
from __future__ import annotations

import math

import numpy as np

from . import special


class Material:
    """Lame constants, density and angular frequency (Section 2).

    c_L = sqrt((lambda + 2 mu)/rho), c_T = sqrt(mu/rho), k = omega / c.
    The Burton-Miller coupling alpha is not given in the paper; the default
    is alpha = i / (mu k_T).
    """

    def __init__(self, lam: float, mu: float, rho: float, omega: float, alpha=None):
        self.lam, self.mu, self.rho, self.omega = float(lam), float(mu), float(rho), float(omega)
        self.cL = math.sqrt((self.lam + 2.0 * self.mu) / self.rho)
        self.cT = math.sqrt(self.mu / self.rho)
        self.kL = self.omega / self.cL
        self.kT = self.omega / self.cT
        self.beta = self.kL / self.kT
        self.alpha = complex(1j / (self.mu * self.kT)) if alpha is None else complex(alpha)


_J = np.array([[0.0, -1.0], [1.0, 0.0]])


def rot(v):
    """J v for vectors stored in the last axis."""
    return np.stack([-v[..., 1], v[..., 0]], axis=-1)


def fundamental_solution(x, y, mat: Material):
    """G_ij(x - y) straight from the definition (i/4mu)[H0(k_T r) delta_ij +
    k_T^-2 d_i d_j (H0(k_T r) - H0(k_L r))], expanded with
    d_i d_j H0(k r) = k^2 H2(k r) e_i e_j - (k/r) H1(k r) delta_ij.
    Used only by the tests (no cancellation handling)."""
    d = np.asarray(x, float) - np.asarray(y, float)
    r = np.linalg.norm(d, axis=-1)
    e = d / r[..., None]
    kT, kL = mat.kT, mat.kL
    h0t, h1t = special.hankel0(kT * r), special.hankel1(kT * r)
    h0l, h1l = special.hankel0(kL * r), special.hankel1(kL * r)
    h2t = 2 * h1t / (kT * r) - h0t
    h2l = 2 * h1l / (kL * r) - h0l
    ee = e[..., :, None] * e[..., None, :]
    eye = np.eye(2)
    hess_t = kT ** 2 * h2t[..., None, None] * ee - (kT / r * h1t)[..., None, None] * eye
    hess_l = kL ** 2 * h2l[..., None, None] * ee - (kL / r * h1l)[..., None, None] * eye
    return 1j / (4 * mat.mu) * (h0t[..., None, None] * eye + (hess_t - hess_l) / kT ** 2)


def point_blocks(x, y, nx, ny, mat: Material):
    """The four 2x2 matrix kernels of A = D + alpha N at quadrature points
    (x and y may be given as the difference x - y and 0).

    Returns (M1, M2, M3, M4), each of shape (..., 2, 2), such that the
    element-pair contribution to the entry between test hat N_a and trial
    hat N_b is  sum_q w_q [N_a dN_b M1 + dN_a dN_b M2 + N_a N_b M3 + dN_a N_b M4],
    dN the (constant) tangential derivative of the hat on its element.
    """
    d = np.asarray(x) - np.asarray(y)
    r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    e = d / r[..., None]
    je = rot(e)
    a = mat.kT * r
    h0a = special.hankel0(a)
    h1a = special.hankel1(a)
    h0b = special.hankel0(mat.kL * r)
    E, chi = special.e_chi(a, mat.beta)
    phiT = 0.25j * h0a
    phiL = 0.25j * h0b
    tx = rot(nx)
    ty = rot(ny)
    dny = 0.25j * mat.kT * h1a * np.einsum("...k,...k->...", e, ny)     # d_{n_y} Phi_T
    dnx = -0.25j * mat.kT * h1a * np.einsum("...k,...k->...", e, nx)    # d_{n_x} Phi_T
    gy = (-0.25j * mat.kT * a * E)[..., None] * e                       # grad_y dPhi
    gx = -gy                                                            # grad_x dPhi
    al, mu = mat.alpha, mat.mu
    rw2 = mat.rho * mat.omega ** 2
    J = _J
    I2 = np.eye(2)
    outer = lambda p, q: p[..., :, None] * q[..., None, :]
    sc = lambda s: s[..., None, None]
    M1 = (sc(phiT - 0.5j * E) * J - sc(0.5j * chi) * outer(e, je)
          + 2.0 * al * mu * (sc(dnx) * J - outer(nx, rot(gx))))
    M2 = 4.0 * al * mu * 0.25j * (sc(-E) * I2 + sc(chi) * outer(je, je))
    M3 = (sc(dny) * I2 + outer(gy, ny)
          + al * rw2 * (sc(phiL) * outer(nx, ny) + sc(phiT) * outer(tx, ty)))
    M4 = -2.0 * al * mu * (sc(dny) * J + outer(rot(gy), ny))
    return M1, M2, M3, M4
