"""Learned rank pre-sizing: randomized interpolative decomposition with a
residual judge, the rank predictor (a small MLP) and its training step, in
plain FP64 (oracle; test infrastructure only).

Randomized ID.  For a matrix M (m x n) and a sketch size s, Y = Omega M with
Omega an s x m matrix of random entries (+-1 +- i); a column-pivoted QR of
Y gives the skeleton columns J and the interpolation matrix
W = [I, R11^{-1} R12] P^T exactly as the ID of Section 7.1 does for M itself;
its rank is the first j with |R_jj| <= tol_s |R_11| of the sketch's QR
(tol_s = tol / 10 in the learned factorisation, see SKETCH_TOL_FACTOR).  The
sketch reveals the rank only if that crossing happens with a few rows to
spare (k + 4 <= s), or if s >= n.  The judge then checks the guarantee the
pivoted QR of M would give: every column of M - M[:, J] W has norm at most
tol times the largest column norm of M.  A prediction that fails either test
falls back to the pivoted QR of M.

Random numbers.  Entry (i, l) of the sketch of problem g is drawn from output
number c = g * 2^44 + i * 2^24 + l of the SplitMix64 generator (Steele, Lea
and Flood, 2014; the 64-bit finaliser with the golden-ratio increment)
seeded with ``seed``: bit 0 gives the sign of the real part, bit 1 that of
the imaginary part.

Rank predictor.  Features of a cell of the upward step: log(k_T d),
log(k_L d) (d the cell diameter 2 R, R the radius of the cell's disk), the
level (root 0), log of the active DOFs per component b / 2, log of the rows
of the proxy-plus-near matrix 2 n_proxy + (near rows), and -log10(tol);
target: the largest of the cell's four ID ranks.  Logarithms keep the
size-like inputs of different discretisations in one range.  Network 6-64-64-64-1 with ReLU, inputs standardised by
(mu, sigma), output scaled by y_scale.  Trained by minibatch Adam on the mean
squared error in units of y_scale.
"""
from __future__ import annotations

import math

import numpy as np

from . import fds as ofds

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
N_IN, N_H = 6, 64
# trainable parameter layout: W1 (64 x 6, row j = neuron j), b1, W2 (64 x 64), b2,
# W3 (64 x 64), b3, w4 (64), b4 (1); then mu (6), sigma (6), y_scale (1)
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H, N_H)),
          ("b3", (N_H,)), ("w4", (N_H,)), ("b4", (1,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)
N_BLOB = N_PARAM + 2 * N_IN + 1


# ---------------------------------------------------------------- generator
def splitmix64(seed: int, counter):
    """Output number ``counter`` (0-based) of SplitMix64 seeded with ``seed``;
    counter may be an int or a uint64 array."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK) + (c + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def sketch_matrix(seed: int, gid: int, s: int, m: int):
    """Omega (s x m) of problem ``gid``: entries (+-1) + i (+-1)."""
    i = np.arange(s, dtype=np.uint64)[:, None]
    l = np.arange(m, dtype=np.uint64)[None, :]
    c = (np.uint64(gid) << np.uint64(44)) | (i << np.uint64(24)) | l
    z = splitmix64(seed, c)
    re = 1.0 - 2.0 * (z & np.uint64(1)).astype(np.float64)
    im = 1.0 - 2.0 * ((z >> np.uint64(1)) & np.uint64(1)).astype(np.float64)
    return re + 1j * im


# ---------------------------------------------------------------- randomized ID
# The sketch's rank is taken at SKETCH_TOL_FACTOR * tol: the sketch's column
# norms are a random projection of M's, distorted by a factor of a few at
# these sizes, so a first crossing at tol itself leaves residuals of up to
# ~3 tol on M (and ~1.2 tol at tol / 4); at tol / 10 the judge (at tol, on M)
# passes with margin, at about one pivot more than the pivoted QR of M.
SKETCH_TOL_FACTOR = 0.1
# A sketch reveals a rank only with this many rows to spare.
REVEAL_MARGIN = 4


def randomized_id(M, s, tol, seed, gid, k_use=None, sketch_tol=None):
    """Randomized column ID of M from a sketch of s rows.

    Returns dict(piv, rank, revealed, W, ratio): ``rank`` is the sketch's
    first-crossing rank at ``sketch_tol`` (default tol); W and ``ratio``
    (largest residual column norm over largest column norm of M) use
    ``k_use`` pivots if given, else ``rank``."""
    M = np.asarray(M, dtype=np.complex128)
    m, n = M.shape
    Y = sketch_matrix(seed, gid, s, m) @ M
    piv, R = ofds.cpqr(Y)
    k = ofds.id_rank(R, tol if sketch_tol is None else sketch_tol)
    revealed = (k + REVEAL_MARGIN <= s) or (s >= n)
    kw = k if k_use is None else int(k_use)
    W = ofds.id_matrix(piv, R, kw, n)
    E = M - M[:, piv[:kw]] @ W
    cn = np.linalg.norm(M, axis=0)
    top = cn.max() if n else 0.0
    ratio = float(np.linalg.norm(E, axis=0).max() / top) if top > 0 else 0.0
    return {"piv": piv, "rank": k, "revealed": bool(revealed), "W": W, "ratio": ratio}


def best_interpolation_ratio(M, J):
    """min over W of max_j ||M[:, j] - M[:, J] W[:, j]|| / max_j ||M[:, j]||
    (least squares per column): the smallest judge ratio any interpolation
    on the skeleton J can reach."""
    M = np.asarray(M, dtype=np.complex128)
    if len(J) == 0:
        return 1.0 if np.any(M) else 0.0
    W, *_ = np.linalg.lstsq(M[:, J], M, rcond=None)
    E = M - M[:, J] @ W
    return float(np.linalg.norm(E, axis=0).max() / np.linalg.norm(M, axis=0).max())


# ---------------------------------------------------------------- features
def cell_features(c, mat, tol, n_proxy, n_near_rows):
    """Predictor inputs of a cell (see module docstring)."""
    d = 2.0 * c.radius
    return np.array([math.log(mat.kT * d), math.log(mat.kL * d), float(c.level),
                     math.log(len(c.cols) / 2.0), math.log(float(2 * n_proxy + n_near_rows)), -math.log10(tol)])


# ---------------------------------------------------------------- MLP
def unpack(blob):
    blob = np.asarray(blob, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = blob[o:o + k].reshape(shp)
        o += k
    out["mu"] = blob[o:o + N_IN]
    out["sigma"] = blob[o + N_IN:o + 2 * N_IN]
    out["y_scale"] = float(blob[o + 2 * N_IN])
    return out


def init_blob(seed, mu, sigma, y_scale):
    """He-uniform initial weights, zero biases, and the normalisation.  The
    weight at flat parameter index p is lim (2 u - 1), u = (z >> 11) 2^-53
    with z the SplitMix64(seed) output number p, lim = sqrt(6 / fan_in)."""
    parts, o = [], 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        if name.startswith("b"):
            parts.append(np.zeros(k))
        else:
            fan_in = shp[1] if len(shp) == 2 else shp[0]
            lim = math.sqrt(6.0 / fan_in)
            z = splitmix64(seed, np.arange(o, o + k, dtype=np.uint64))
            u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
            parts.append(lim * (2.0 * u - 1.0))
        o += k
    parts += [np.asarray(mu, float), np.asarray(sigma, float), [float(y_scale)]]
    return np.concatenate(parts)


def standardise(X, y):
    """mu, sigma (population standard deviation, 1 where it is 0) of the
    features and y_scale = max(1, max y)."""
    X = np.asarray(X, float)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd == 0.0] = 1.0
    return mu, sd, max(1.0, float(np.max(y)))


def forward(blob, X, cache=False):
    """Network output in units of y_scale (n,); the prediction is y_scale * out."""
    p = unpack(blob)
    Xn = (np.asarray(X, float) - p["mu"]) / p["sigma"]
    z1 = Xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(z3, 0.0)
    out = h3 @ p["w4"] + p["b4"][0]
    if cache:
        return out, (Xn, z1, h1, z2, h2, z3, h3)
    return out


def predict(blob, X):
    return unpack(blob)["y_scale"] * forward(blob, X)


def loss_grad(blob, X, y):
    """Mean squared error of forward(X) against y / y_scale, and its gradient
    with respect to the trainable parameters (layout of SHAPES), by the chain
    rule through the ReLU layers."""
    p = unpack(blob)
    out, (Xn, z1, h1, z2, h2, z3, h3) = forward(blob, X, cache=True)
    t = np.asarray(y, float) / p["y_scale"]
    n = len(t)
    r = out - t
    loss = float(np.mean(r * r))
    g_out = 2.0 * r / n
    g = {"w4": h3.T @ g_out, "b4": np.array([g_out.sum()])}
    d3 = np.outer(g_out, p["w4"]) * (z3 > 0)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ Xn
    g["b1"] = d1.sum(0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam_step(blob, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of the trainable part of ``blob``;
    t is the 1-based step number.  Returns new (blob, m, v)."""
    blob = np.array(blob, float)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    blob[:N_PARAM] -= lr * mh / (np.sqrt(vh) + eps)
    return blob, m, v


def minibatch(seed, step, batch, n):
    """Sample indices of a training step: output (step * 2^32 + slot) of
    SplitMix64 seeded with ``seed``, reduced mod n."""
    c = (np.uint64(step) << np.uint64(32)) | np.arange(batch, dtype=np.uint64)
    return (splitmix64(seed, c) % np.uint64(n)).astype(np.int64)
