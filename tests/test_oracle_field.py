"""Pins of the oracle's field away from the boundary (the integral
representation of Section 3).

* The double-layer kernel K_ij = T^{n_y}_{jk} G_ik agrees with the traction,
  contracted with the full elastic tensor C_jpkq of Section 2, of
  finite-difference derivatives of the fundamental solution (pins the
  third-derivative algebra and where each index goes).
* With the closed-form circular-cavity solution as nodal boundary values,
  the representation reproduces the closed-form field outside the cavity
  and gives zero inside it (the incident field is cancelled there), both
  converging at second order in the element length.
* With the dense Galerkin solution as boundary values, the field outside
  agrees with the closed form (the whole chain).
* A rotated wave and rotated targets on the regular N-gon give the rotated
  field.
* Near the boundary the kernel takes the difference of the two Hankel
  functions from its power series; its derivatives match 40-digit mpmath.
"""
import math

import numpy as np
import pytest

import synthetic as sy
from oracle import dense, field, series
from oracle.kernels import Material, fundamental_solution

MAT = dict(lam=2.0, mu=1.0, rho=1.0, omega=1.0)
OUT = np.array([[1.5 * math.cos(t), 1.5 * math.sin(t)] for t in (0.3, 1.9, 4.0)]
               + [[2.5 * math.cos(t), 2.5 * math.sin(t)] for t in (0.0, 2.2)])
IN = np.array([[0.3 * math.cos(t), 0.3 * math.sin(t)] for t in (0.5, 2.5)]
              + [[0.6 * math.cos(t), 0.6 * math.sin(t)] for t in (1.0, 4.4)])


def _elastic_tensor(lam, mu):
    d = np.eye(2)
    C = np.zeros((2, 2, 2, 2))
    for j in range(2):
        for p in range(2):
            for k in range(2):
                for q in range(2):
                    C[j, p, k, q] = lam * d[j, p] * d[k, q] + mu * (d[j, k] * d[p, q] + d[j, q] * d[p, k])
    return C


@pytest.mark.parametrize("omega", [0.4, 1.7, 6.0])
def test_traction_kernel_matches_finite_differences(omega):
    mat = Material(2.0, 1.0, 1.3, omega)
    rng = np.random.default_rng(4)
    C = _elastic_tensor(mat.lam, mat.mu)
    for _ in range(4):
        x = rng.uniform(-1, 1, 2)
        y = x + rng.uniform(0.4, 1.5) * np.array([math.cos(rng.uniform(0, 6.3)), math.sin(rng.uniform(0, 6.3))])
        a = rng.uniform(0, 2 * math.pi)
        ny = np.array([math.cos(a), math.sin(a)])
        h = 1e-4
        dG = np.zeros((2, 2, 2), dtype=np.complex128)      # [i, k, q] = d_{y_q} G_ik(x - y)
        for q in range(2):
            e = np.zeros(2)
            e[q] = h
            G = lambda yy: fundamental_solution(x, yy, mat)
            dG[:, :, q] = (-G(y + 2 * e) + 8 * G(y + e) - 8 * G(y - e) + G(y - 2 * e)) / (12 * h)
        ref = np.zeros((2, 2), dtype=np.complex128)
        for i in range(2):
            for j in range(2):
                ref[i, j] = sum(C[j, p, k, q] * ny[p] * dG[i, k, q]
                                for p in range(2) for k in range(2) for q in range(2))
        K = field.traction_kernel(x, y, ny, mat)
        assert np.max(np.abs(K - ref)) < 1e-8 * np.max(np.abs(ref)), (K, ref)


def _exact_boundary_field(n, pts):
    mat = Material(**MAT)
    nodes = sy.circle(n)
    X = series.displacement(mat, nodes).reshape(-1)
    U = field.field([nodes], X, pts, kinds=[0], angles=[0.0], **MAT)[0]
    return mat, U


def test_representation_reproduces_series_outside_at_second_order():
    errs = []
    for n in (64, 128, 256):
        mat, U = _exact_boundary_field(n, OUT)
        ex = series.displacement(mat, OUT)
        errs.append(np.max(np.abs(U - ex)) / np.max(np.abs(ex)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.15), (errs, orders)
    assert errs[-1] < 1e-4


def test_extinction_inside_the_cavity_at_second_order():
    errs = []
    for n in (64, 128, 256):
        _, U = _exact_boundary_field(n, IN)
        errs.append(np.max(np.abs(U)))      # |u^I| = 1
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.15), (errs, orders)
    assert errs[-1] < 1e-4


def test_dense_solution_field_matches_series():
    mat = Material(**MAT)
    nodes = sy.circle(128)
    X = dense.dense_solve([nodes], kinds=[0], angles=[0.0], **MAT)
    U = field.field([nodes], X, OUT, kinds=[0], angles=[0.0], **MAT)[0]
    ex = series.displacement(mat, OUT)
    assert np.max(np.abs(U - ex)) < 1e-3 * np.max(np.abs(ex))


def test_rotational_symmetry():
    n, j = 40, 3
    ang = 2 * math.pi * j / n
    nodes = sy.circle(n)
    X = dense.dense_solve([nodes], kinds=[1, 1], angles=[0.2, 0.2 + ang], **MAT)
    c, s = math.cos(ang), math.sin(ang)
    Rm = np.array([[c, -s], [s, c]])
    U0 = field.field([nodes], X[:, 0], OUT, kinds=[1], angles=[0.2], **MAT)[0]
    U1 = field.field([nodes], X[:, 1], OUT @ Rm.T, kinds=[1], angles=[0.2 + ang], **MAT)[0]
    assert np.max(np.abs(U1 - U0 @ Rm.T)) < 1e-11 * np.max(np.abs(U0))


def test_hankel_difference_series_matches_high_precision():
    # the small-argument path of the kernel: derivatives of
    # g = (H0(k_T r) - H0(k_L r)) / k_T^2 from the power series against
    # mpmath at 40 digits (the direct difference loses ~7 digits at r = 4e-4)
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for kT, kL in ((2.0, 2.0 / math.sqrt(3.0)), (0.7, 0.35)):
        f = lambda rr: (mp.hankel1(0, kT * rr) - mp.hankel1(0, kL * rr)) / kT ** 2
        for r in (0.9 / kT, 0.2, 1e-2, 4e-4, 1e-5):
            d1, d2, d3 = (complex(mp.diff(f, mp.mpf(r), m)) for m in (1, 2, 3))
            g1, A, g3 = field._g_series(np.array([r]), kT, kL)
            assert abs(g1[0] - d1) < 1e-14 * abs(d1)
            assert abs(A[0] - (d2 / r - d1 / r ** 2)) < 1e-14 * abs(d2 / r - d1 / r ** 2)
            assert abs(g3[0] - d3) < 1e-14 * abs(d3)
