"""Pins of the learned-form oracle (randomized ID, judge, MLP, Adam) against
facts fixed independently of its code: published generator outputs, exact
low-rank algebra, finite differences, the closed form of Adam's first step."""
import math

import numpy as np
import pytest

from oracle import learned as ol, fds as ofds
from oracle.kernels import Material

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_splitmix64_reference_outputs():
    # the first outputs of SplitMix64 from state 0 (reference implementation)
    got = [int(v) for v in ol.splitmix64(0, np.arange(3, dtype=np.uint64))]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sketch_entries_are_balanced_signs():
    O = ol.sketch_matrix(123, 7, 64, 4096)
    assert set(np.unique(O.real)) == {-1.0, 1.0} and set(np.unique(O.imag)) == {-1.0, 1.0}
    # +-1 with mean 0: |mean| within 5 standard deviations of a fair coin
    n = O.size
    assert abs(O.real.mean()) < 5 / math.sqrt(n) and abs(O.imag.mean()) < 5 / math.sqrt(n)
    assert abs(np.mean(O.real * O.imag)) < 5 / math.sqrt(n)
    # different problems and seeds give different sketches
    assert not np.array_equal(O, ol.sketch_matrix(123, 8, 64, 4096))
    assert not np.array_equal(O, ol.sketch_matrix(124, 7, 64, 4096))


def _low_rank(m, n, r, rng, noise=0.0):
    A = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r)))
    B = (rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n)))
    M = A @ B
    if noise:
        M = M + noise * (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    return M


def test_randomized_id_exact_rank():
    rng = np.random.default_rng(1)
    M = _low_rank(200, 60, 17, rng)
    res = ol.randomized_id(M, 17 + 6, 1e-10, seed=5, gid=0)
    assert res["rank"] == 17 and res["revealed"]
    assert res["ratio"] < 1e-12
    # the interpolation reproduces M from its skeleton columns
    J = res["piv"][:17]
    assert np.allclose(M[:, J] @ res["W"], M, atol=1e-10 * np.abs(M).max())


def test_randomized_id_too_small_sketch_is_not_revealed():
    rng = np.random.default_rng(2)
    M = _low_rank(200, 60, 30, rng)
    res = ol.randomized_id(M, 20, 1e-10, seed=5, gid=1)
    assert res["rank"] == 20 and not res["revealed"]
    assert res["ratio"] > 1e-3


def test_randomized_id_judge_on_decaying_spectrum():
    rng = np.random.default_rng(3)
    m, n = 180, 64
    U, _ = np.linalg.qr(rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    M = (U * np.logspace(0, -14, n)) @ V.conj().T
    tol = 1e-8
    res = ol.randomized_id(M, 48, tol, seed=9, gid=3)
    assert res["revealed"]
    # compare with the pivoted QR of M itself: the same kind of rank
    _, R = ofds.cpqr(M)
    k_full = ofds.id_rank(R, tol)
    assert abs(res["rank"] - k_full) <= 3
    # the best interpolation on the sketch's skeleton is at least as good
    J = res["piv"][:res["rank"]]
    assert ol.best_interpolation_ratio(M, J) <= res["ratio"] * (1 + 1e-9)
    # more pivots never hurt the best interpolation
    J2 = res["piv"][:res["rank"] + 4]
    assert ol.best_interpolation_ratio(M, J2) <= ol.best_interpolation_ratio(M, J) * (1 + 1e-9)


def _blob(rng):
    mu = rng.standard_normal(6)
    sigma = rng.uniform(0.5, 2.0, 6)
    return ol.init_blob(4, mu, sigma, 16.0)


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    blob = _blob(rng)
    blob[:ol.N_PARAM] += 0.05 * rng.standard_normal(ol.N_PARAM)   # nonzero biases
    X = rng.standard_normal((37, 6)) * 2.0
    y = rng.uniform(0, 60, 37)
    loss, g = ol.loss_grad(blob, X, y)
    idx = rng.choice(ol.N_PARAM, 60, replace=False)
    idx = np.concatenate([idx, [ol.N_PARAM - 1, 0]])
    h = 1e-6
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (ol.loss_grad(bp, X, y)[0] - ol.loss_grad(bm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, i


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    blob = _blob(rng)
    g = rng.standard_normal(ol.N_PARAM)
    z = np.zeros(ol.N_PARAM)
    nb, m, v = ol.adam_step(blob, g, z, z, 1, 1e-3)
    # with bias correction the first step is lr * g / (|g| + eps)
    assert np.allclose(nb[:ol.N_PARAM] - blob[:ol.N_PARAM], -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.array_equal(nb[ol.N_PARAM:], blob[ol.N_PARAM:])


def test_training_fits_a_smooth_target():
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (512, 6))
    y = 20 + 8 * X[:, 0] + 4 * X[:, 3] ** 2
    blob = ol.init_blob(1, X.mean(0), X.std(0), 16.0)
    m = np.zeros(ol.N_PARAM)
    v = np.zeros(ol.N_PARAM)
    l0 = ol.loss_grad(blob, X, y)[0]
    for t in range(1, 301):
        idx = ol.minibatch(77, t, 128, len(y))
        _, g = ol.loss_grad(blob, X[idx], y[idx])
        blob, m, v = ol.adam_step(blob, g, m, v, t, 3e-3)
    assert ol.loss_grad(blob, X, y)[0] < 0.05 * l0


def test_init_blob_is_he_uniform():
    mu, sd, ys = ol.standardise(np.array([[1.0, 2, 3, 4, 5, 8], [3.0, 2, 5, 4, 7, 8]]), [3.0, 40.0])
    assert np.allclose(mu, [2, 2, 4, 4, 6, 8]) and np.allclose(sd, [1, 1, 1, 1, 1, 1]) and ys == 40.0
    b = ol.init_blob(9, mu, sd, ys)
    p = ol.unpack(b)
    for name, fan in (("W1", 6), ("W2", 64), ("W3", 64), ("w4", 64)):
        w = p[name].ravel()
        lim = math.sqrt(6.0 / fan)
        assert np.all(np.abs(w) <= lim) and np.std(w) > 0.4 * lim   # uniform on (-lim, lim): std lim/sqrt(3)
    for name in ("b1", "b2", "b3", "b4"):
        assert not np.any(p[name])
    assert p["y_scale"] == 40.0 and np.array_equal(p["mu"], mu)


def test_minibatch_indices_in_range():
    idx = ol.minibatch(3, 11, 1000, 37)
    assert idx.min() >= 0 and idx.max() < 37 and len(np.unique(idx)) == 37


def test_cell_features_closed_form():
    mat = Material(2.0, 1.0, 1.0, 4.0)
    c = ofds.Cell(index=5, level=2)
    c.cols = np.arange(90)
    c.radius = 0.25
    f = ol.cell_features(c, mat, 1e-8, 64, 37)
    assert np.allclose(f, [math.log(4.0 * 0.5), math.log(2.0 * 0.5), 2.0, math.log(45.0), math.log(165.0), 8.0])
