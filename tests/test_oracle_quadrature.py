"""Pins of the oracle's element-pair quadrature (the rules of
``oracle/quadrature.py``, which both implementations share as the
definition of the discrete operator).

Every class of pair is integrated a second way, by rules that share nothing
with the oracle's maps, and the two must agree within 1e-11 of the pair's
largest entry:

* coincident pairs: the square split along its diagonal, the offset
  d = |u - v| integrated by composite Gauss on panels graded geometrically
  toward d = 0 (ratio 0.15, 40 panels, 16 points each), the position along
  the diagonal by 6-point Gauss; the mass term by Gauss too;
* adjacent pairs: distances from the shared vertex, a tensor product of two
  such graded rules (24 panels of 20 points each; the 1/r corner
  singularity);
* regular pairs (2, 3, 4, 6 or 10 points along each element, chosen by the
  gap, that element's length and the wavenumber): each element cut into
  panels with 20 points each;
* proxy pairs (a cell's proxy polygon against its own elements, both
  orientations): as regular pairs;
* load vectors: 40-point Gauss per element.

The references are converged themselves: refining them changes the result
by less than 1e-12 of the pair maximum, 3e-12 for the tensor graded rule of
adjacent pairs (checked once per class at the largest k_T h).

Workloads: the 131072-node ellipse (omega = 4), the paper's tripod with
6400 nodes (lambda = mu = 1, omega = 2 and 14.5) and a coarse 64-gon at
omega = 1, 4 and 14.5 (about 4.4 elements per transverse wavelength at the
top).  Also the closed-form series of the small case at the point (1, 0), a
value derived independently of the oracle, and the dense small-case solution
there within the discretisation error.
"""
import numpy as np
import pytest

import synthetic as sy
from oracle import fds as ofds, galerkin, quadrature as qr, series
from oracle.galerkin import Polygon, _integrate
from oracle.kernels import Material

TOL = 1e-11


# ------------------------------------------------------------------ reference rules
def _gl01(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def _graded01(levels=40, sigma=0.15, q=16):
    """Composite Gauss on (0, 1], panels [sigma^(j+1), sigma^j] and a last
    panel [0, sigma^levels]."""
    g, w = _gl01(q)
    e = [sigma ** j for j in range(levels + 1)] + [0.0]
    pts, wts = [], []
    for b, a in zip(e[:-1], e[1:]):
        pts.append(a + (b - a) * g)
        wts.append((b - a) * w)
    return np.concatenate(pts), np.concatenate(wts)


def _panels01(p, q):
    g, w = _gl01(q)
    return np.concatenate([(i + g) / p for i in range(p)]), np.concatenate([w / p] * p)


def _one(PA, e, PB, f, u, v, w, dvec, mat):
    return _integrate(PA, np.array([e]), PB, np.array([f]), u, v, w, dvec[None], mat)[0]


def ref_coincident(P, e, mat, levels=40, q=16):
    d, wd = _graded01(levels, 0.15, q)
    t, wt = _gl01(6)
    D = np.repeat(d, len(t))
    WD = np.repeat(wd, len(t))
    T = np.tile(t, len(d)) * (1.0 - D)
    W = WD * np.tile(wt, len(d)) * (1.0 - D)
    side = P.p1[e] - P.p0[e]
    out = 0
    # u > v: u = v + d ; u < v: v = u + d  (x - y = (u - v)(p1 - p0))
    for u, v, s in ((T + D, T, 1.0), (T, T + D, -1.0)):
        out = out + _one(P, e, P, e, u, v, W, (s * D)[:, None] * side[None, :], mat)
    # + I0/2 on the coincident pair: int N_a N_b ds, 4-point Gauss
    g, wg = _gl01(4)
    Nh = np.stack([1.0 - g, g], axis=1)
    I0 = P.h[e] * np.einsum("q,qa,qb->ab", wg, Nh, Nh)
    return out + 0.5 * I0[:, :, None, None] * np.eye(2)[None, None]


def ref_adjacent(PA, e, PB, f, mat, follows, levels=24, q=20, sigma=0.15):
    """``follows``: f follows e (shared vertex = end of e = start of f);
    otherwise e follows f (shared vertex = start of e = end of f)."""
    s, ws = _graded01(levels, sigma, q)
    up = np.repeat(s, len(s))
    vp = np.tile(s, len(s))
    w = np.repeat(ws, len(s)) * np.tile(ws, len(s))
    if follows:
        A_ = PA.p0[e] - PA.p1[e]
        B_ = PB.p1[f] - PB.p0[f]
        u, v = 1.0 - up, vp
    else:
        A_ = PA.p1[e] - PA.p0[e]
        B_ = PB.p0[f] - PB.p1[f]
        u, v = up, 1.0 - vp
    dvec = up[:, None] * A_[None, :] - vp[:, None] * B_[None, :]
    return _one(PA, e, PB, f, u, v, w, dvec, mat)


def ref_regular(PA, e, PB, f, mat, p=4, q=20):
    s, ws = _panels01(p, q)
    u = np.repeat(s, len(s))
    v = np.tile(s, len(s))
    w = np.repeat(ws, len(s)) * np.tile(ws, len(s))
    dvec = ((PA.p0[e] - PB.p0[f])[None, :] + u[:, None] * (PA.p1[e] - PA.p0[e])[None, :]
            - v[:, None] * (PB.p1[f] - PB.p0[f])[None, :])
    return _one(PA, e, PB, f, u, v, w, dvec, mat)


def _rel(a, r):
    return np.max(np.abs(a - r)) / np.max(np.abs(r))


def _oracle_pair(PA, e, PB, f, mat):
    return galerkin.element_pairs(PA, np.array([e]), PB, np.array([f]), mat)[0]


def _regular_classes(P, e, mat, span=60):
    """The first pair (smallest gap) of each regular tensor order (q_e, q_f),
    with trial elements e + 2 ... e + span and three far ones."""
    n = P.n
    picks = {}
    for j in list(range(2, min(span, n - 2))) + [n // 8, n // 4, n // 2]:
        f = (e + j) % n
        if f in ((e - 1) % n, e, (e + 1) % n):
            continue
        d = galerkin.segment_distance(P.p0[e], P.p1[e], P.p0[f], P.p1[f])
        qe, qf = qr.regular_orders(np.array([d]), P.h[e], P.h[f], mat.kT)
        picks.setdefault((int(qe[0]), int(qf[0])), f)
    return picks


WORKLOADS = {
    "ellipse131072_w4": (lambda: sy.ellipse(131072, 1.0, 0.5), (2.0, 1.0, 1.0, 4.0), [0, 32768, 70001]),
    "tripod6400_w2": (lambda: sy.tripod(6400), (1.0, 1.0, 1.0, 2.0), [0, 1067, 3201]),
    "tripod6400_w14.5": (lambda: sy.tripod(6400), (1.0, 1.0, 1.0, 14.5), [0, 1067]),
    "circle64_w1": (lambda: sy.circle(64), (2.0, 1.0, 1.0, 1.0), [0, 17]),
    "circle64_w4": (lambda: sy.circle(64), (2.0, 1.0, 1.0, 4.0), [0, 17]),
    "circle64_w14.5": (lambda: sy.circle(64), (2.0, 1.0, 1.0, 14.5), [0, 17]),
}


@pytest.fixture(scope="module", params=sorted(WORKLOADS))
def workload(request):
    make, m, elems = WORKLOADS[request.param]
    return request.param, Polygon(make(), +1), Material(*m), elems


def test_coincident_pairs(workload):
    name, P, mat, elems = workload
    for e in elems:
        assert _rel(_oracle_pair(P, e, P, e, mat), ref_coincident(P, e, mat)) < TOL, (name, e)


def test_adjacent_pairs_both_orientations(workload):
    name, P, mat, elems = workload
    n = P.n
    for e in elems:
        assert _rel(_oracle_pair(P, e, P, (e + 1) % n, mat), ref_adjacent(P, e, P, (e + 1) % n, mat, True)) < TOL
        assert _rel(_oracle_pair(P, e, P, (e - 1) % n, mat), ref_adjacent(P, e, P, (e - 1) % n, mat, False)) < TOL


def test_regular_pairs_each_order(workload):
    name, P, mat, elems = workload
    seen = set()
    for e in elems:
        for q, f in _regular_classes(P, e, mat).items():
            seen.add(q)
            assert _rel(_oracle_pair(P, e, P, f, mat), ref_regular(P, e, P, f, mat)) < TOL, (name, e, f, q)
    kh = mat.kT * P.h.max()
    if kh <= qr.KH_Q2:
        assert {(2, 2), (3, 3), (4, 4), (6, 6)} <= seen, (name, seen)
    elif kh <= qr.KH_Q3:
        assert {(3, 3), (4, 4), (6, 6)} <= seen and (2, 2) not in seen, (name, seen)


def test_proxy_pairs_both_orientations(workload):
    """A cell of 1/16 and one of 1/4 of the curve against the proxy polygon
    of radius 1.5 R about it (outward normal): the closest and a far proxy
    element for every cell element at the cell's ends and middle."""
    name, P, mat, elems = workload
    n = P.n
    for frac in (16, 4):
        nodes = np.arange(n // frac + 1)
        pts = P.nodes[nodes]
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        c = 0.5 * (lo + hi)
        R = float(np.max(np.hypot(*(pts - c).T)))
        px = ofds.proxy_polygon(c, ofds.PROXY_RATIO * R, ofds.proxy_count(mat.kT, ofds.PROXY_RATIO * R))
        for e in (0, len(nodes) // 2, len(nodes) - 2):
            gaps = galerkin.segment_distance(px.p0, px.p1, np.broadcast_to(P.p0[e], px.p0.shape),
                                             np.broadcast_to(P.p1[e], px.p1.shape))
            for i in (int(np.argmin(gaps)), int(np.argmax(gaps))):
                assert _rel(_oracle_pair(px, i, P, e, mat), ref_regular(px, i, P, e, mat)) < TOL, (name, frac, e, i)
                assert _rel(_oracle_pair(P, e, px, i, mat), ref_regular(P, e, px, i, mat)) < TOL, (name, frac, e, i)


def test_load_vectors(workload):
    name, P, mat, elems = workload
    if P.n > 10000:
        pytest.skip("load vectors of the large curves: the 64-gon and the tripod cover the rule")
    bnd = galerkin.Boundary([P.nodes])
    g, w = _gl01(40)
    for kind in (0, 1):
        f = galerkin.load_vector(bnd, kind, 0.7, mat)
        x = P.p0[:, None, :] + g[None, :, None] * (P.p1 - P.p0)[:, None, :]
        nrm = np.broadcast_to(P.normal[:, None, :], x.shape)
        u, t = galerkin.incident_field(x.reshape(-1, 2), nrm.reshape(-1, 2), kind, 0.7, mat)
        val = (u + mat.alpha * t).reshape(P.n, len(g), 2)
        wh = w[None, :] * P.h[:, None]
        ref = (np.einsum("eq,eqi->ei", wh * (1.0 - g)[None, :], val)
               + np.roll(np.einsum("eq,eqi->ei", wh * g[None, :], val), 1, axis=0)).reshape(-1)
        assert np.max(np.abs(f - ref)) < TOL * np.max(np.abs(ref)), (name, kind)


def test_graded_references_are_converged():
    """Refining the references moves them by < 1e-12 of the pair max (3e-12
    for adjacent pairs), so the 1e-11 comparisons above measure the oracle's
    rules."""
    P = Polygon(sy.circle(64), +1)
    mat = Material(2.0, 1.0, 1.0, 14.5)
    a = ref_coincident(P, 3, mat)
    b = ref_coincident(P, 3, mat, levels=60, q=24)
    assert _rel(a, b) < 1e-12
    a = ref_adjacent(P, 3, P, 4, mat, True)
    b = ref_adjacent(P, 3, P, 4, mat, True, levels=40, q=24, sigma=0.1)
    assert _rel(a, b) < 3e-12
    a = ref_regular(P, 3, P, 5, mat)
    b = ref_regular(P, 3, P, 5, mat, p=8, q=24)
    assert _rel(a, b) < 1e-12


def test_frequency_rule_is_needed():
    """At k_T h = 1.4 (64-gon, omega = 14.5) the gap rule alone (4 points for a
    far pair) and the low-frequency adjacent rule are off by more than 1e-9:
    the wavenumber terms of the order choice keep such pairs converged."""
    P = Polygon(sy.circle(64), +1)
    mat = Material(2.0, 1.0, 1.0, 14.5)
    e, f = 0, 20
    u, v, w = qr.tensor_rule(4)
    dvec = (P.p0[e] - P.p0[f])[None, :] + u[:, None] * (P.p1[e] - P.p0[e]) - v[:, None] * (P.p1[f] - P.p0[f])
    q4 = _one(P, e, P, f, u, v, w, dvec, mat)
    ref = ref_regular(P, e, P, f, mat)
    assert _rel(q4, ref) > 1e-9
    assert _rel(_oracle_pair(P, e, P, f, mat), ref) < TOL
    up, vp, w = qr.adjacent_rule(qr.Q_ADJ)
    dvec = up[:, None] * (P.p0[e] - P.p1[e])[None, :] - vp[:, None] * (P.p1[e + 1] - P.p0[e + 1])[None, :]
    lo = _one(P, e, P, e + 1, 1.0 - up, vp, w, dvec, mat)
    ref = ref_adjacent(P, e, P, e + 1, mat, True)
    assert _rel(lo, ref) > 1e-9
    assert _rel(_oracle_pair(P, e, P, e + 1, mat), ref) < TOL


def test_low_orders_need_their_limits():
    """The 2- and 3-point rules hold only far away and at small k_T h: on the
    tripod at omega = 14.5 (k_T h = 0.018) a pair 480 elements apart is off
    by more than 1e-11 on 2 x 2 points (the oscillation over an element),
    and on the ellipse a pair 16 elements apart is off by more than 1e-12 on
    3 x 3 points (the gap); the oracle's choices for both are within 1e-11."""
    P = Polygon(sy.tripod(6400), +1)
    mat = Material(1.0, 1.0, 1.0, 14.5)
    e, f = 0, 480
    assert qr.KH_Q2 < mat.kT * max(P.h[e], P.h[f]) <= qr.KH_Q3
    ref = ref_regular(P, e, P, f, mat)
    assert _rel(_tensor_pair(P, e, P, f, mat, 2, 2), ref) > 1e-11
    assert _rel(_oracle_pair(P, e, P, f, mat), ref) < TOL
    P = Polygon(sy.ellipse(131072, 1.0, 0.5), +1)
    mat = Material(2.0, 1.0, 1.0, 4.0)
    e, f = 0, 16
    ref = ref_regular(P, e, P, f, mat)
    assert _rel(_tensor_pair(P, e, P, f, mat, 3, 3), ref) > 1e-12
    assert _rel(_oracle_pair(P, e, P, f, mat), ref) < TOL


def _tensor_pair(P, e, Q, f, mat, qe, qf):
    u, v, w = qr.tensor_rule(qe, qf)
    dvec = (P.p0[e] - Q.p0[f])[None, :] + u[:, None] * (P.p1[e] - P.p0[e]) - v[:, None] * (Q.p1[f] - Q.p0[f])
    return _one(P, e, Q, f, u, v, w, dvec, mat)


# ------------------------------------------------------------------ small case
def test_series_reference_value_small_case():
    """The series at the small case's material and frequency (lambda=2, mu=1,
    rho=1, omega=1, radius 1, unit P-wave along +x_1) at the point (1, 0):
    u = (-0.26248583 + 0.91639948 i, 0), a value derived independently of
    the oracle when the problem was set up."""
    mat = Material(2.0, 1.0, 1.0, 1.0)
    u = series.displacement(mat, np.array([[1.0, 0.0]])).reshape(-1)
    assert abs(u[0] - (-0.26248583 + 0.91639948j)) < 1e-8
    assert abs(u[1]) < 1e-12


def test_dense_small_case_at_the_reference_point():
    """The dense Galerkin solution of the small case (256 nodes) at node 0 =
    (1, 0) is within the discretisation error of the series value: the
    polygon and P1 give O(h^2), h = 2 pi / 256, so well under 1e-3."""
    from oracle import dense
    cfg = sy.config_small()
    X = dense.dense_solve(cfg["curves"], cfg["lam"], cfg["mu"], cfg["rho"], cfg["omega"], cfg["kinds"],
                          cfg["angles"])
    x = np.asarray(X).reshape(-1)
    assert abs(x[0] - (-0.26248583 + 0.91639948j)) < 1e-3
    assert abs(x[1]) < 1e-3
