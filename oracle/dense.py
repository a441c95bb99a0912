"""The conventional dense BEM ("Conv" of Section 8): assemble the full
2N x 2N Galerkin system of Section 5.2 and solve it by LU with partial
pivoting (LAPACK through scipy).  Oracle; test infrastructure only."""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import galerkin
from .kernels import Material


def dense_solve(curves, lam, mu, rho, omega, kinds, angles, alpha=None, return_matrix=False):
    """Solve A x = f for each incident wave (kind 0 = P, 1 = S; angle in
    radians).  Returns x of shape (2N, nrhs), unknown 2 t + i = u_{i+1} at node t."""
    mat = Material(lam, mu, rho, omega, alpha)
    bnd = galerkin.Boundary(curves)
    A = galerkin.dense_matrix(bnd, mat)
    F = np.stack([galerkin.load_vector(bnd, k, a, mat) for k, a in zip(kinds, angles)], axis=1)
    lu = sla.lu_factor(A)
    X = sla.lu_solve(lu, F)
    if return_matrix:
        return X, A, F
    return X
