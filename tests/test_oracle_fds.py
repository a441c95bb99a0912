"""Pins of the oracle's fast direct solver.

* CPQR gives the same pivots and |diag R| as LAPACK's pivoted QR when the
  column norms are well separated; the ID residual is at the tolerance.
* With an ID tolerance near rounding the compressed solve reproduces the
  dense LU solution (the elimination is exact algebra, Section 6.2).
* The error against the dense solution falls with the tolerance, the
  pattern of the paper's Table 1.
* The small validation case (256-node circle, tol 1e-10) matches the dense
  solution within 1e-9.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synthetic as sy
from oracle import dense, fds, galerkin


def test_cpqr_matches_lapack():
    rng = np.random.default_rng(0)
    M = (rng.standard_normal((40, 12)) + 1j * rng.standard_normal((40, 12))) * np.logspace(0, -6, 12)
    piv, R = fds.cpqr(M)
    Q2, R2, p2 = sla.qr(M, pivoting=True, mode="economic")
    assert np.array_equal(piv, p2)
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(R2)), rtol=1e-10)


def test_id_residual_at_tolerance():
    # smooth kernel matrix: well-separated source/target clusters
    x = np.linspace(0, 1, 60)
    y = np.linspace(3, 4, 50)
    M = 1.0 / (x[:, None] - y[None, :]) + 0j
    for tol in (1e-6, 1e-10):
        piv, R = fds.cpqr(M)
        k = fds.id_rank(R, tol)
        W = fds.id_matrix(piv, R, k, M.shape[1])
        err = np.linalg.norm(M - M[:, piv[:k]] @ W, 2)
        assert 0 < k < M.shape[1]
        assert err < 50 * tol * np.linalg.norm(M, 2)


MAT = dict(lam=2.0, mu=1.0, rho=1.0)


def _dense(nodes, omega, kinds, angles):
    return dense.dense_solve([nodes], omega=omega, kinds=kinds, angles=angles, return_matrix=True, **MAT)


def test_exact_algebra_at_rounding_tolerance():
    nodes = sy.ellipse(96, 1.0, 0.5)
    X, A, F = _dense(nodes, 2.0, [0, 1], [0.0, 1.0])
    S = fds.FDS([nodes], omega=2.0, tol=1e-15, leaf=12, root_level=1, **MAT)
    Y = S.solve(F)
    assert np.linalg.norm(Y - X) < 1e-11 * np.linalg.norm(X)


def test_error_falls_with_tolerance():
    nodes = sy.ellipse(128, 1.0, 0.5)
    X, A, F = _dense(nodes, 3.0, [0], [0.3])
    errs = []
    for tol in (1e-4, 1e-7, 1e-10):
        S = fds.FDS([nodes], omega=3.0, tol=tol, leaf=16, root_level=1, **MAT)
        errs.append(np.linalg.norm(S.solve(F) - X) / np.linalg.norm(X))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-8
    assert errs[1] < 1e-5


def test_small_validation_case():
    cfg = sy.config_small()
    nodes = cfg["curves"][0]
    X, A, F = _dense(nodes, cfg["omega"], cfg["kinds"], cfg["angles"])
    S = fds.FDS(cfg["curves"], cfg["lam"], cfg["mu"], cfg["rho"], cfg["omega"], cfg["tol"],
                leaf=cfg["leaf"], root_level=1)
    Y = S.solve(F)
    assert S.L == 3
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) < 1e-9


# ---------------------------------------------------------------- tree over several curves
def test_morton_order_visits_quadrants_in_z_order():
    # corners of a square: Z-order visits (0,0), (1,0), (0,1), (1,1)
    order = fds.morton_order([(0, 0), (1, 1), (1, 0), (0, 1)])
    assert list(order) == [0, 2, 3, 1]
    # nested: the four points of the lower-left quadrant come before any other
    pts = [(0.9, 0.9), (0.1, 0.1), (0.4, 0.1), (0.1, 0.4), (0.4, 0.4), (0.6, 0.1)]
    order = list(fds.morton_order(pts))
    assert order[:4] == [1, 2, 3, 4] and order[-1] == 0


def _check_tree(bnd, leaf):
    L, cells, perm = fds.build_tree(bnd, leaf)
    assert sorted(perm) == list(range(bnd.n_nodes))
    assert L == (0 if bnd.n_nodes <= leaf else int(np.ceil(np.log2(bnd.n_nodes / leaf))))
    # every node numbered position lies in exactly one leaf
    leaves = fds.level_cells(cells, L)
    cover = np.zeros(bnd.n_nodes, int)
    for c in leaves:
        assert c.hi > c.lo
        cover[c.lo:c.hi] += 1
    assert np.all(cover == 1)
    # curve index of each position of the numbering
    cur = bnd.curve_of[perm]
    for lev in range(L):
        for p in fds.level_cells(cells, lev):
            a, b = cells[2 * p.index + 1], cells[2 * p.index + 2]
            assert (a.lo, a.hi, b.lo, b.hi) == (p.lo, a.hi, a.hi, p.hi)
            curves = np.unique(cur[p.lo:p.hi])
            whole = all(np.sum(cur == k) == np.sum(cur[p.lo:p.hi] == k) for k in curves)
            if len(curves) >= 2 and whole:
                # split at a curve boundary, most balanced among all boundaries
                bounds = [i for i in range(p.lo + 1, p.hi) if cur[i] != cur[i - 1]]
                assert a.hi in bounds
                best = min(abs(2 * (i - p.lo) - (p.hi - p.lo)) for i in bounds)
                assert abs(2 * (a.hi - p.lo) - (p.hi - p.lo)) == best
            else:
                assert len(curves) == 1
                assert a.hi == p.lo + (p.hi - p.lo) // 2
    return L, cells, perm


def test_tree_over_several_curves():
    curves = sy.multi_cavity(3, 12, 3000)
    bnd = galerkin.Boundary(curves)
    _check_tree(bnd, 64)


def test_tree_of_one_curve_is_the_midpoint_tree():
    bnd = galerkin.Boundary([sy.ellipse(1000, 1.0, 0.5)])
    L, cells, perm = _check_tree(bnd, 64)
    assert np.array_equal(perm, np.arange(1000))


def test_timing_samples_do_the_factorisation_work():
    """The CPU baseline's timing samples: at the leaf level the stand-in
    active sets are the real ones, so a sampled leaf cell gets the ranks of
    the same cell in a full factorisation; above it the sets have the
    stand-in rank per component and child (sizes only); the root sample
    factors a system of the top cells' stand-in order."""
    nodes = sy.ellipse(256, 1.0, 0.5)
    F = fds.FDS([nodes], 2.0, 1.0, 1.0, 4.0, 1e-8, leaf=32)
    leaves = fds.level_cells(F.cells, F.L)
    got = fds.level_sample([nodes], 2.0, 1.0, 1.0, 4.0, 1e-8, 32, F.L, 0, [0, 5, 7])
    assert [k for _, k in got] == [leaves[q].k for q in (0, 5, 7)]
    assert all(t > 0 for t, _ in got)
    up = fds.level_sample([nodes], 2.0, 1.0, 1.0, 4.0, 1e-8, 32, F.L - 1, 8, [3])
    assert 0 < up[0][1][0] <= 16 and 0 < up[0][1][1] <= 16
    t, n = fds.root_sample([nodes], 2.0, 1.0, 1.0, 4.0, 32, 1, 8)
    assert n == 2 * 2 * 2 * 8 and t > 0
