"""Pins of the oracle's kernels and regularised Galerkin form.

* G satisfies the Navier-Cauchy equation away from the source (finite
  differences of the definition in the equation of the fundamental solution).
* On separated supports the regularised Galerkin entries equal the direct
  double integrals of psi T_y G phi and psi T_x T_y G phi, with the traction
  operators applied to G by finite differences (this is the traction operator
  of Section 2 written out, independent of the regularisation algebra).
* Static rigid-body identities: D applied to a translation gives half the
  mass matrix times it; N annihilates translations and the rotation.
* N is complex-symmetric: N(s,t)_ij = N(t,s)_ji.
"""
import numpy as np
import pytest

import synthetic as sy
from oracle import galerkin, quadrature as qr
from oracle.kernels import Material, fundamental_solution


def _fd_grad(f, p, h):
    """4th-order central differences of f (array-valued) at points p (..., 2)."""
    out = []
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        out.append((-f(p + 2 * e) + 8 * f(p + e) - 8 * f(p - e) + f(p - 2 * e)) / (12 * h))
    return out


def test_navier_equation_fd():
    mat = Material(2.0, 1.0, 1.0, 3.0)
    x = np.array([[0.7, -0.4], [1.9, 0.8]])
    y = np.zeros(2)
    h = 1e-3
    G = lambda p: fundamental_solution(p, y, mat)
    d11 = _fd_grad(lambda p: _fd_grad(G, p, h)[0], x, h)
    d22 = _fd_grad(lambda p: _fd_grad(G, p, h)[1], x, h)
    lap = d11[0] + d22[1]
    # grad div of each column field G[:, j]: (grad div)_i = d_i d_k G_kj
    H = [[d11[0], d11[1]], [d22[0], d22[1]]]   # H[a][b] = d_b d_a G
    gd = np.zeros_like(lap)
    for i in range(2):
        for k in range(2):
            gd[..., i, :] += H[k][i][..., k, :]
    res = mat.mu * lap + (mat.lam + mat.mu) * gd + mat.rho * mat.omega ** 2 * G(x)
    assert np.max(np.abs(res)) < 1e-6 * np.max(np.abs(G(x)))


def _traction(grad, n, lam, mu):
    """(T^n v)_j = lambda n_j div v + mu (n_k d_k v_j + n_k d_j v_k),
    grad[k][..., c] = d_k v_c."""
    div = grad[0][..., 0] + grad[1][..., 1]
    out = []
    for j in range(2):
        t = lam * n[..., j] * div
        for k in range(2):
            t = t + mu * (n[..., k] * grad[k][..., j] + n[..., k] * grad[j][..., k])
        out.append(t)
    return np.stack(out, axis=-1)


def _direct_kernels(x, y, nx, ny, mat, h=1e-3):
    """Gamma_ij = T^{n_y}_{jk} G_ik and N_ij = T^{n_x}_{ik} Gamma_kj by finite
    differences.  x, y, nx, ny of shape (P, 2)."""

    def gamma(xx):
        # derivative of G_ik(xx - y) with respect to y
        g = _fd_grad(lambda yy: fundamental_solution(xx, yy, mat), y, h)   # g[k][P, i, c]
        out = np.zeros(xx.shape[:-1] + (2, 2), dtype=np.complex128)
        for i in range(2):
            gi = [g[k][..., i, :] for k in range(2)]     # d_k v_c with v_c = G_ic
            out[..., i, :] = _traction(gi, ny, mat.lam, mat.mu)
        return out

    Gam = gamma(x)
    dG = _fd_grad(gamma, x, h)    # dG[k][P, i, j] = d_{x_k} Gamma_ij
    N = np.zeros_like(Gam)
    for j in range(2):
        gj = [dG[k][..., :, j] for k in range(2)]     # d_k w_c with w_c = Gamma_cj
        N[..., :, j] = _traction(gj, nx, mat.lam, mat.mu)
    return Gam, N


def _direct_entry(P, s, t, mat, q=8):
    """int int psi^s(x) [Gamma + alpha N](x, y) phi^t(y) over the supports."""
    g, w = qr.gauss01(q)
    D = np.zeros((2, 2), dtype=np.complex128)
    Nn = np.zeros((2, 2), dtype=np.complex128)
    for e, a in (((s - 1) % P.n, 1), (s, 0)):
        for f, b in (((t - 1) % P.n, 1), (t, 0)):
            U, V = np.meshgrid(g, g, indexing="ij")
            W = np.outer(w, w).ravel() * P.h[e] * P.h[f]
            U, V = U.ravel(), V.ravel()
            x = P.p0[e] + U[:, None] * (P.p1[e] - P.p0[e])
            y = P.p0[f] + V[:, None] * (P.p1[f] - P.p0[f])
            Na = (1 - U) if a == 0 else U
            Nb = (1 - V) if b == 0 else V
            nx = np.broadcast_to(P.normal[e], x.shape)
            ny = np.broadcast_to(P.normal[f], y.shape)
            Gam, NN = _direct_kernels(x, y, nx, ny, mat)
            wt = (W * Na * Nb)[:, None, None]
            D += np.sum(wt * Gam, axis=0)
            Nn += np.sum(wt * NN, axis=0)
    return D, Nn


@pytest.mark.parametrize("omega", [1.0, 4.0])
def test_regularised_form_matches_direct_kernels(omega):
    P = galerkin.Polygon(sy.ellipse(40, 1.0, 0.5))
    m0 = Material(2.0, 1.0, 1.0, omega, alpha=0.0)
    m1 = Material(2.0, 1.0, 1.0, omega, alpha=1.0)
    for s, t in ((3, 17), (0, 9), (25, 31)):
        A0 = galerkin.node_block(P, [s], P, [t], m0)[0, 0]
        A1 = galerkin.node_block(P, [s], P, [t], m1)[0, 0]
        Dd, Nd = _direct_entry(P, s, t, m0)
        assert np.max(np.abs(A0 - Dd)) < 1e-8 * np.max(np.abs(Dd))
        assert np.max(np.abs((A1 - A0) - Nd)) < 1e-7 * np.max(np.abs(Nd))


def test_static_rigid_body_identities():
    P = galerkin.Polygon(sy.ellipse(48, 1.0, 0.6))
    bnd = galerkin.Boundary([P.nodes])
    om = 1e-4
    m0 = Material(2.0, 1.0, 1.0, om, alpha=0.0)
    m1 = Material(2.0, 1.0, 1.0, om, alpha=1.0)
    A0 = galerkin.dense_matrix(bnd, m0)           # D + I0/2
    Nm = galerkin.dense_matrix(bnd, m1) - A0      # N
    n = bnd.n_nodes
    mass = np.zeros((n, n))
    for e in range(n):
        i, j = e, (e + 1) % n
        h = P.h[e]
        mass[i, i] += h / 3
        mass[j, j] += h / 3
        mass[i, j] += h / 6
        mass[j, i] += h / 6
    M2 = np.kron(mass, np.eye(2))
    for c in (np.array([1.0, 0.0]), np.array([0.3, -0.8])):
        u = np.tile(c, n)
        # (D + I0/2) c = I0 c  (D c = c/2 on the boundary in the static limit)
        assert np.linalg.norm(A0 @ u - M2 @ u) < 1e-6 * np.linalg.norm(M2 @ u)
        assert np.linalg.norm(Nm @ u) < 1e-6 * np.linalg.norm(Nm, 2) * np.linalg.norm(u)
    rotn = np.stack([-P.nodes[:, 1], P.nodes[:, 0]], axis=1).ravel()
    assert np.linalg.norm(Nm @ rotn) < 1e-6 * np.linalg.norm(Nm, 2) * np.linalg.norm(rotn)
    # a non-rigid field is not annihilated (the check has teeth)
    stretch = np.stack([P.nodes[:, 0], np.zeros(n)], axis=1).ravel()
    assert np.linalg.norm(Nm @ stretch) > 1e-2 * np.linalg.norm(Nm, 2) * np.linalg.norm(stretch)


def test_hypersingular_part_is_complex_symmetric():
    P = galerkin.Polygon(sy.ellipse(24, 1.0, 0.5))
    bnd = galerkin.Boundary([P.nodes])
    m0 = Material(2.0, 1.0, 1.0, 2.5, alpha=0.0)
    m1 = Material(2.0, 1.0, 1.0, 2.5, alpha=1.0)
    Nm = galerkin.dense_matrix(bnd, m1) - galerkin.dense_matrix(bnd, m0)
    assert np.max(np.abs(Nm - Nm.T)) < 1e-12 * np.max(np.abs(Nm))
