"""Element-pair quadrature rules (oracle; test infrastructure only).

The paper does not state its quadrature.  The discrete operator used by both
implementations is defined by the following rules on a pair of straight
elements (test element e with local coordinate u in [0,1], trial element f
with v in [0,1]); every rule returns reference points (u, v) and weights that
already contain the reference Jacobians (the physical weight is w h_e h_f):

* regular pair (different elements that share no vertex): tensor
  Gauss-Legendre with q_e points along the test element and q_f along the
  trial element, each element's order chosen from the gap delta = dist(e, f)
  relative to that element's own length h:
  delta >= RATIO_Q2 h -> 2, >= RATIO_Q3 h -> 3, >= FAR_RATIO h -> Q_FAR,
  >= NEAR_RATIO h -> Q_MID, else Q_NEAR; and from the oscillation of the
  kernels over the element (k_T the larger wavenumber): at least 3 points
  when k_T h > KH_Q2, Q_FAR when k_T h > KH_Q3, Q_MID when k_T h > KH_Q4 and
  Q_NEAR when k_T h > KH_Q6 (Q_NEAR holds to about k_T h = 8, beyond which
  the mesh does not resolve the wave).  When either element needs Q_NEAR,
  both take it.  (A q-point Gauss rule along an element of length h at
  distance delta from the singularity converges like (h / 4 delta)^(2q); a
  factor oscillating with wavenumber k adds a term like (k h)^(2q)/(2q)!.)
* coincident pair (e == f): the square is split along its diagonal; on each
  triangle the offset d = |u - v| is mapped as d = s^P_COINC and s is
  integrated with Q_COINC Gauss points, the position along the diagonal with
  2 Gauss points on [0, 1 - d] (exact for the quadratic hat products).
* adjacent pair (one shared vertex): coordinates measured from the shared
  vertex; each of the two triangles is Duffy-mapped (u', v') = (xi, xi eta) or
  (xi eta, xi), xi = s^P_ADJ, with Q_ADJ x Q_ADJ Gauss points in (s, eta).
* both singular rules take Q_COINC_HI and Q_ADJ_HI points in place of
  Q_COINC and Q_ADJ when k_T h > KH_Q4 (h the longer element): the kernels
  then oscillate over the pair.  Boundary elements need k_T h <= KH_MAX.

The Gauss-Legendre nodes come from ``numpy.polynomial.legendre.leggauss``.
"""
from __future__ import annotations

import functools

import numpy as np

Q_FAR = 4
Q_MID = 6
Q_NEAR = 10
RATIO_Q2 = 512.0
RATIO_Q3 = 32.0
FAR_RATIO = 8.0
NEAR_RATIO = 2.0
KH_Q2 = 0.004
KH_Q3 = 0.02
KH_Q4 = 0.5
KH_Q6 = 2.5
KH_MAX = 5.0
Q_COINC = 20
P_COINC = 6
Q_ADJ = 12
P_ADJ = 4
Q_COINC_HI = 30
Q_ADJ_HI = 24
Q_RHS = 6


@functools.lru_cache(maxsize=None)
def gauss01(q: int):
    """q-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


@functools.lru_cache(maxsize=None)
def tensor_rule(qe: int, qf: int = None):
    """Points (u, v) and weights of the tensor Gauss rule with qe points
    along the test element (u) and qf along the trial element (v)."""
    qf = qe if qf is None else qf
    ge, we = gauss01(qe)
    gf, wf = gauss01(qf)
    u = np.repeat(ge, qf)
    v = np.tile(gf, qe)
    ww = np.repeat(we, qf) * np.tile(wf, qe)
    return u, v, ww


@functools.lru_cache(maxsize=None)
def coincident_rule(q: int = Q_COINC, p: int = P_COINC):
    """Points (u, v, w, u - v) on [0,1]^2 for a log-singular kernel on u = v;
    the signed offset u - v is returned exactly."""
    s, ws = gauss01(q)
    d = s ** p
    wd = ws * p * s ** (p - 1)
    g2, w2 = gauss01(2)
    us, vs, wts, offs = [], [], [], []
    for di, wdi in zip(d, wd):
        ell = 1.0 - di
        for gk, wk in zip(g2, w2):
            t = ell * gk
            # triangle u > v: u = t + d, v = t ; triangle u < v: u = t, v = t + d
            us += [t + di, t]
            vs += [t, t + di]
            wts += [wdi * ell * wk, wdi * ell * wk]
            offs += [di, -di]
    return np.array(us), np.array(vs), np.array(wts), np.array(offs)


@functools.lru_cache(maxsize=None)
def adjacent_rule(q: int = Q_ADJ, p: int = P_ADJ):
    """Points (u', v', w) on [0,1]^2 with the singular corner at (0, 0);
    u' and v' are distances from the shared vertex, normalised by the
    element lengths."""
    s, ws = gauss01(q)
    eta, we = gauss01(q)
    xi = s ** p
    wxi = ws * p * s ** (p - 1)
    XI = np.repeat(xi, q)
    WXI = np.repeat(wxi, q)
    ETA = np.tile(eta, q)
    WE = np.tile(we, q)
    w = WXI * WE * XI
    u1, v1 = XI, XI * ETA          # triangle u' >= v'
    u2, v2 = XI * ETA, XI          # triangle v' > u'
    return np.concatenate([u1, u2]), np.concatenate([v1, v2]), np.concatenate([w, w])


def element_order(delta, h, k):
    """Gauss points along one element of a regular pair: gap delta, the
    element's own length h, largest wavenumber k."""
    delta = np.asarray(delta, dtype=np.float64)
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), delta.shape)
    q = np.full(delta.shape, Q_NEAR, dtype=np.int64)
    q[delta >= NEAR_RATIO * h] = Q_MID
    q[delta >= FAR_RATIO * h] = Q_FAR
    q[delta >= RATIO_Q3 * h] = 3
    q[delta >= RATIO_Q2 * h] = 2
    kh = k * h
    q[(kh > KH_Q2) & (q < 3)] = 3
    q[(kh > KH_Q3) & (q < Q_FAR)] = Q_FAR
    q[(kh > KH_Q4) & (q < Q_MID)] = Q_MID
    q[kh > KH_Q6] = Q_NEAR
    return q


def regular_orders(delta, he, hf, k):
    """Orders (q_e, q_f) of the tensor rule of regular pairs with gap delta,
    element lengths he (test) and hf (trial) and largest wavenumber k; both
    Q_NEAR when either element needs it."""
    qe = element_order(delta, he, k)
    qf = element_order(delta, hf, k)
    near = (qe == Q_NEAR) | (qf == Q_NEAR)
    qe[near] = Q_NEAR
    qf[near] = Q_NEAR
    return qe, qf
