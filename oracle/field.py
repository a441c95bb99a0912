"""Field away from the boundary by the integral representation (oracle;
test infrastructure only).

After the boundary solution is known, the total displacement at a point x
of the solid is (Section 3, the equation of the integral representation)

    u_i(x) = u^I_i(x) - int_Gamma K_ij(x, y) u_j(y) ds(y),
    K_ij(x, y) = T^{n_y}_{jk} G_ik(x - y),

the traction at y (normal n_y, pointing into the cavity) of the column of
the fundamental solution G (its equation in Section 3) for a point force at
x in direction i.  The traction operator of Section 2 is
T^n_{jk} v_k = C_{jpkq} n_p d_q v_k with
C_{jpkq} = lambda d_jp d_kq + mu (d_jk d_pq + d_jq d_pk).  The boundary
values are the piecewise-linear interpolant of the nodal solution
(Section 4), and the traction-free condition removes the single-layer term.

K is written out from these definitions, with no integration by parts.
For a radial function f(r), r = |d|, e = d / r, derivatives in d = x - y:

    d_i d_k d_q f = f''' e_i e_k e_q
                    + (f''/r - f'/r^2)(d_iq e_k + d_kq e_i + d_ik e_q - 3 e_i e_k e_q),

and the radial derivatives of H0(k r) are k^m times scipy's derivatives of
H0^(1).  d_{y_q} = -d_{d_q}.

For k_T r < 1 the difference g = (H0(k_T r) - H0(k_L r)) / k_T^2 is not
formed from the two Hankel functions (their third derivatives, each of
size 1/r^3, cancel to a result of size 1/r, losing about 2 log10(1/(k r))
digits).  It is summed from the power series of J0 and Y0 (Abramowitz and
Stegun 9.1.12-13), H0(k r) = sum_m c_m (k r / 2)^{2m} [1 + (2i/pi)(ln(k r / 2)
+ gamma - H_m)], c_m = (-1)^m / (m!)^2, H_m the harmonic numbers, with the
two wavenumbers' coefficients subtracted before any power of r multiplies
them, and differentiated term by term.

Quadrature: every element is split into S equal panels with
S = ceil(2 h / dist) (at least 1, at most ``max_panels``), dist the distance
from x to the element and h its length, and each panel gets 20-point
Gauss-Legendre.  A panel is then no longer than half its distance from x,
so the rule is exact to rounding for targets not on Gamma.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as sp

from .galerkin import Boundary, incident_field
from .kernels import Material

_Q = 20


def _radial(k, r, m):
    """m-th derivative in r of H0^(1)(k r)."""
    return k ** m * sp.h1vp(0, k * r, m)


def _g_series(r, kT, kL, terms=24):
    """(g', g''/r - g'/r^2, g''') of g = (H0(k_T r) - H0(k_L r)) / k_T^2 from
    the power series (for k_T r < 1)."""
    r = np.asarray(r, dtype=np.float64)
    lr = np.log(r)
    g1 = np.zeros(r.shape, dtype=np.complex128)
    A = np.zeros(r.shape, dtype=np.complex128)
    g3 = np.zeros(r.shape, dtype=np.complex128)
    two_i_pi = 2j / math.pi
    Hm = 0.0
    for m in range(1, terms):
        Hm += 1.0 / m
        cm = (-1.0) ** m / math.factorial(m) ** 2
        pT, pL = (kT / 2.0) ** (2 * m), (kL / 2.0) ** (2 * m)
        # coefficients of r^n and of r^n ln r in k_T^2 g, n = 2 m (the m = 0
        # term is a constant)
        a = cm * (pT * (1.0 + two_i_pi * (math.log(kT / 2.0) + np.euler_gamma - Hm))
                  - pL * (1.0 + two_i_pi * (math.log(kL / 2.0) + np.euler_gamma - Hm)))
        b = cm * two_i_pi * (pT - pL)
        n = 2 * m
        rn1, rn3 = r ** (n - 1), r ** (n - 3)
        g1 += a * n * rn1 + b * rn1 * (n * lr + 1.0)
        A += a * n * (n - 2) * rn3 + b * rn3 * (n * (n - 2) * lr + 2 * n - 2)
        g3 += a * n * (n - 1) * (n - 2) * rn3 + b * rn3 * (n * (n - 1) * (n - 2) * lr + 3 * n * n - 6 * n + 2)
    return g1 / kT ** 2, A / kT ** 2, g3 / kT ** 2


def _g_parts(r, kT, kL):
    """(g', g''/r - g'/r^2, g''') of g = (H0(k_T r) - H0(k_L r)) / k_T^2."""
    g1 = (_radial(kT, r, 1) - _radial(kL, r, 1)) / kT ** 2
    g2 = (_radial(kT, r, 2) - _radial(kL, r, 2)) / kT ** 2
    g3 = (_radial(kT, r, 3) - _radial(kL, r, 3)) / kT ** 2
    A = g2 / r - g1 / r ** 2
    small = kT * r < 1.0
    if np.any(small):
        s1, sA, s3 = _g_series(r[small], kT, kL)
        g1[small], A[small], g3[small] = s1, sA, s3
    return g1, A, g3


def _third_derivative(f1, A, f3, e):
    """d_i d_k d_q f for a radial f, given f', A = f''/r - f'/r^2 and the
    third derivative f3; shape (..., 2, 2, 2)."""
    I = np.eye(2)
    eee = e[..., :, None, None] * e[..., None, :, None] * e[..., None, None, :]
    S = (I[:, None, :] * e[..., None, :, None]          # d_iq e_k
         + I[None, :, :] * e[..., :, None, None]        # d_kq e_i
         + I[:, :, None] * e[..., None, None, :]        # d_ik e_q
         - 3.0 * eee)
    return f3[..., None, None, None] * eee + A[..., None, None, None] * S


def traction_kernel(x, y, ny, mat: Material):
    """K[..., i, j] = T^{n_y}_{jk} G_ik(x - y) for points x, y and unit
    normals n_y (arrays broadcastable to (..., 2))."""
    d = np.asarray(x, float) - np.asarray(y, float)
    ny = np.broadcast_to(np.asarray(ny, float), d.shape)
    r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    e = d / r[..., None]
    kT, kL = mat.kT, mat.kL
    # G_ik = (i / 4 mu) [h_T d_ik + d_i d_k g],  g = (h_T - h_L) / k_T^2
    hT1 = _radial(kT, r, 1)
    g1, A, g3 = (v.reshape(r.shape) for v in _g_parts(np.atleast_1d(r), kT, kL))
    I = np.eye(2)
    # dG[..., i, k, q] = d_{d_q} G_ik
    dG = (1j / (4.0 * mat.mu)) * ((hT1[..., None, None, None] * I[:, :, None] * e[..., None, None, :])
                                  + _third_derivative(g1, A, g3, e))
    dGy = -dG                                            # derivatives in y
    lam, mu = mat.lam, mat.mu
    # t_j = lam n_j d_k w_k + mu (n_q d_q w_j + n_k d_j w_k), w_k = G_ik(x - .)
    div = np.einsum("...ikk->...i", dGy)
    dn = np.einsum("...ijq,...q->...ij", dGy, ny)
    tr = np.einsum("...ikj,...k->...ij", dGy, ny)
    return lam * div[..., :, None] * ny[..., None, :] + mu * (dn + tr)


def element_integrals(x, P, mat: Material, max_panels: int = 4096):
    """For one target x and every element e of polygon P: the 2 x 2 integrals
    int_e K(x, y) phi(y) ds(y) for the hat of the element's first node
    (``start``) and of its second node (``end``); shapes (n, 2, 2)."""
    g, w = np.polynomial.legendre.leggauss(_Q)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    a, b = P.p0, P.p1
    ab = b - a
    t = np.clip(np.einsum("ek,ek->e", x - a, ab) / np.einsum("ek,ek->e", ab, ab), 0.0, 1.0)
    dist = np.linalg.norm(a + t[:, None] * ab - x, axis=1)
    with np.errstate(divide="ignore"):
        S = np.where(dist > 0, np.ceil(2.0 * P.h / np.maximum(dist, 1e-300)), max_panels)
    S = np.clip(S, 1, max_panels).astype(np.int64)
    start = np.zeros((P.n, 2, 2), dtype=np.complex128)
    end = np.zeros((P.n, 2, 2), dtype=np.complex128)
    for s in np.unique(S):
        idx = np.nonzero(S == s)[0]
        # parameter values on the element: panel p covers [p/s, (p+1)/s]
        u = ((np.arange(s)[:, None] + g[None, :]) / s).reshape(-1)             # (s q,)
        wu = np.tile(w, s) / s
        y = a[idx, None, :] + u[None, :, None] * ab[idx, None, :]              # (m, s q, 2)
        K = traction_kernel(x[None, None, :], y, P.normal[idx, None, :], mat)  # (m, s q, 2, 2)
        wh = wu[None, :] * P.h[idx, None]
        start[idx] = np.einsum("mp,mpij->mij", wh * (1.0 - u)[None, :], K)
        end[idx] = np.einsum("mp,mpij->mij", wh * u[None, :], K)
    return start, end


def field(curves, X, targets, lam, mu, rho, omega, kinds=None, angles=None, alpha=None):
    """Displacement at ``targets`` (M x 2) for the boundary solutions X
    (2N x nrhs, unknown 2 t + i; or a single vector of length 2N).  With
    ``kinds``/``angles`` (one plane wave per solution, as for the load
    vectors) the incident field is added; without them the result is the
    scattered part -int K u only.  Returns (nrhs, M, 2)."""
    mat = Material(lam, mu, rho, omega, alpha)
    bnd = Boundary(curves)
    X = np.asarray(X, dtype=np.complex128)
    if X.ndim == 1:
        X = X[:, None]
    nrhs = X.shape[1]
    targets = np.asarray(targets, dtype=np.float64).reshape(-1, 2)
    U = np.zeros((nrhs, len(targets), 2), dtype=np.complex128)
    for m, x in enumerate(targets):
        acc = np.zeros((nrhs, 2), dtype=np.complex128)
        for c, P in enumerate(bnd.polys):
            o = bnd.offsets[c]
            Xc = X[2 * o:2 * (o + P.n)].reshape(P.n, 2, nrhs)    # node, component, rhs
            start, end = element_integrals(x, P, mat)
            acc += np.einsum("eij,ejr->ri", start, Xc)
            acc += np.einsum("eij,ejr->ri", end, np.roll(Xc, -1, axis=0))
        U[:, m, :] = -acc
    if kinds is not None:
        for r, (k, a) in enumerate(zip(kinds, angles)):
            u, _ = incident_field(targets, np.zeros_like(targets), int(k), float(a), mat)
            U[r] += u
    return U
