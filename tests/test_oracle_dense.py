"""Pins of the closed-form series, the load vectors and the dense BEM.

* The series satisfies the traction-free condition on r = a and the
  Navier-Cauchy equation (finite differences of the series itself).
* The plane-wave tractions used in the load vectors agree with finite
  differences of the incident displacement (P and S waves).
* The dense Galerkin solution converges to the series at second order
  (P1 elements on an inscribed polygon), and solves its system to rounding.
* Discrete rotational symmetry on the regular N-gon.
"""
import math

import numpy as np
import pytest

import synthetic as sy
from oracle import dense, galerkin, series
from oracle.kernels import Material

MAT = dict(lam=2.0, mu=1.0, rho=1.0, omega=1.0)


def _num_grad(f, x, h=1e-4):
    g = []
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        g.append((-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * h))
    return g    # g[k][P, c] = d_k u_c


def _stress(g, lam, mu):
    div = g[0][:, 0] + g[1][:, 1]
    s = np.zeros((len(div), 2, 2), dtype=np.complex128)
    for i in range(2):
        for j in range(2):
            s[:, i, j] = mu * (g[j][:, i] + g[i][:, j]) + (lam * div if i == j else 0)
    return s


@pytest.mark.parametrize("omega", [1.0, 2.5])
def test_series_is_traction_free_and_solves_navier(omega):
    mat = Material(2.0, 1.0, 1.0, omega)
    th = np.linspace(0.1, 2 * math.pi, 7)
    x = np.stack([np.cos(th), np.sin(th)], axis=1)
    u = lambda p: series.displacement(mat, p)
    s = _stress(_num_grad(u, x), mat.lam, mat.mu)
    trac = np.einsum("pij,pj->pi", s, x)
    scale = np.max(np.abs(s))
    assert np.max(np.abs(trac)) < 1e-7 * scale
    # Navier residual at r = 1.6
    y = 1.6 * x
    H = [_num_grad(lambda p, k=k: _num_grad(u, p, 1e-3)[k], y, 1e-3) for k in range(2)]
    lap = H[0][0] + H[1][1]
    gd = np.stack([H[0][0][:, 0] + H[1][0][:, 1], H[0][1][:, 0] + H[1][1][:, 1]], axis=1)
    res = mat.mu * lap + (mat.lam + mat.mu) * gd + mat.rho * omega ** 2 * u(y)
    assert np.max(np.abs(res)) < 1e-6 * np.max(np.abs(u(y)))


@pytest.mark.parametrize("kind", [0, 1])
def test_plane_wave_traction(kind):
    mat = Material(2.0, 1.0, 1.0, 3.0)
    ang = 0.7
    x = np.array([[0.3, -0.2], [1.1, 0.9]])
    n = np.array([[0.6, 0.8], [-1.0, 0.0]])
    _, t = galerkin.incident_field(x, n, kind, ang, mat)
    f = lambda p: galerkin.incident_field(p, n, kind, ang, mat)[0]
    s = _stress(_num_grad(f, x, 1e-3), mat.lam, mat.mu)
    assert np.max(np.abs(np.einsum("pij,pj->pi", s, n) - t)) < 1e-9 * np.max(np.abs(t))


def test_dense_converges_to_series_at_second_order():
    mat = Material(**MAT)
    errs = []
    for n in (32, 64, 128):
        nodes = sy.circle(n)
        X, A, F = dense.dense_solve([nodes], kinds=[0], angles=[0.0], return_matrix=True, **MAT)
        assert np.linalg.norm(A @ X - F) < 1e-13 * np.linalg.norm(F) * 10
        ex = series.displacement(mat, nodes)
        errs.append(np.linalg.norm(X[:, 0].reshape(-1, 2) - ex) / np.linalg.norm(ex))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.1), orders
    assert errs[-1] < 2e-4


def test_rotational_symmetry_on_regular_polygon():
    n = 40
    nodes = sy.circle(n)
    j = 3
    ang = 2 * math.pi * j / n
    X = dense.dense_solve([nodes], kinds=[0, 0], angles=[0.0, ang], **MAT)
    u0 = X[:, 0].reshape(-1, 2)
    u1 = X[:, 1].reshape(-1, 2)
    c, s = math.cos(ang), math.sin(ang)
    Rm = np.array([[c, -s], [s, c]])
    # field for the rotated wave at node t+j is the rotated field at node t
    pred = (Rm @ u0.T).T
    assert np.max(np.abs(np.roll(u1, -j, axis=0) - pred)) < 1e-11 * np.max(np.abs(u0))
