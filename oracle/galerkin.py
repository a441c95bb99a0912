"""Galerkin entries and load vectors (oracle; test infrastructure only).

Discretisation (Section 4): the boundary is an N-gon with nodes x^t;
unknowns are nodal values of piecewise-linear hats phi^t, test functions
psi^s = phi^s.  The system matrix (Section 5.2) has 2x2 blocks

    A(s, t) = D(s, t) + I0(s, t)/2 + alpha N(s, t),  I0(s, t) = int psi^s phi^t,

and the load vector is f^s_i = int psi^s (u^I_i + alpha (T u^I)_i).
Global unknown 2 t + i holds component i (0-based) at node t.

A polygon carries an orientation sign: +1 for a cavity boundary (the
normal n = J tau points into the cavity, Section 2), -1 for a proxy circle
(outward normal, away from the cell it encloses).  Tangential derivatives are
taken along t = J n.
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature as qr
from .kernels import Material, point_blocks, rot


class Polygon:
    """A closed polygon; element e joins node e to node (e + 1) mod n."""

    _next_id = 0

    def __init__(self, nodes, sign: int = +1):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self.n = len(self.nodes)
        self.sign = int(sign)
        Polygon._next_id += 1
        self.pid = Polygon._next_id
        p0 = self.nodes
        p1 = np.roll(self.nodes, -1, axis=0)
        d = p1 - p0
        self.p0, self.p1 = p0, p1
        self.h = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
        self.tau = d / self.h[:, None]
        self.normal = self.sign * rot(self.tau)
        self.tang = rot(self.normal)
        tt = np.einsum("ek,ek->e", self.tau, self.tang)        # +-1
        self.dN = np.stack([-tt / self.h, tt / self.h], axis=1)  # d_s of the two hats


def segment_distance(a0, a1, b0, b1):
    """Distance between segments [a0, a1] and [b0, b1] (non-intersecting)."""

    def pt_seg(p, s0, s1):
        d = s1 - s0
        t = np.einsum("...k,...k->...", p - s0, d) / np.einsum("...k,...k->...", d, d)
        t = np.clip(t, 0.0, 1.0)
        q = s0 + t[..., None] * d
        return np.sqrt(np.sum((p - q) ** 2, axis=-1))

    return np.minimum(np.minimum(pt_seg(a0, b0, b1), pt_seg(a1, b0, b1)),
                      np.minimum(pt_seg(b0, a0, a1), pt_seg(b1, a0, a1)))


def _integrate(PA, ea, PB, fb, u, v, w, dvec, mat):
    """Integrate element pairs (ea[k], fb[k]) at reference points u, v (shape
    (P,)) with reference weights w; ``dvec`` (K, P, 2) holds x - y at those
    points, formed by the caller without cancellation.  Returns
    (K, 2, 2, 2, 2) indexed [k, a, b, i, j] (a: test hat, b: trial hat)."""
    K = len(ea)
    u = np.broadcast_to(u, (K,) + np.shape(u)[-1:])
    v = np.broadcast_to(v, u.shape)
    w = np.broadcast_to(w, u.shape)
    nx = np.broadcast_to(PA.normal[ea][:, None, :], dvec.shape)
    ny = np.broadcast_to(PB.normal[fb][:, None, :], dvec.shape)
    M1, M2, M3, M4 = point_blocks(dvec, 0.0, nx, ny, mat)
    ww = w * (PA.h[ea] * PB.h[fb])[:, None]
    Na = np.stack([1.0 - u, u], axis=-1)          # (K, P, 2)
    Nb = np.stack([1.0 - v, v], axis=-1)
    S1 = np.einsum("kp,kpa,kpij->kaij", ww, Na, M1)
    S2 = np.einsum("kp,kpij->kij", ww, M2)
    S3 = np.einsum("kp,kpa,kpb,kpij->kabij", ww, Na, Nb, M3)
    S4 = np.einsum("kp,kpb,kpij->kbij", ww, Nb, M4)
    dA = PA.dN[ea]      # (K, 2)
    dB = PB.dN[fb]
    res = (S1[:, :, None] * dB[:, None, :, None, None]
           + (dA[:, :, None] * dB[:, None, :])[..., None, None] * S2[:, None, None]
           + S3
           + dA[:, :, None, None, None] * S4[:, None])
    return res


def element_pairs(PA: Polygon, ea, PB: Polygon, fb, mat: Material, chunk: int = 4096):
    """Element-pair contributions [k, a, b, i, j] of A = D + I0/2 + alpha N
    for test elements ea of PA and trial elements fb of PB."""
    ea = np.asarray(ea, dtype=np.int64)
    fb = np.asarray(fb, dtype=np.int64)
    K = len(ea)
    out = np.zeros((K, 2, 2, 2, 2), dtype=np.complex128)
    same = PA is PB
    if same:
        n = PA.n
        coinc = ea == fb
        nxt = fb == (ea + 1) % n          # f follows e: shared vertex p1_e = p0_f
        prv = (fb == (ea - 1) % n) & ~nxt  # e follows f: shared vertex p0_e = p1_f
    else:
        coinc = np.zeros(K, bool)
        nxt = np.zeros(K, bool)
        prv = np.zeros(K, bool)
    regular = ~(coinc | nxt | prv)

    for hi in (False, True):
        sel = coinc & ((mat.kT * PA.h[ea] > qr.KH_Q4) == hi)
        if not np.any(sel):
            continue
        idx = np.nonzero(sel)[0]
        u, v, w, off = qr.coincident_rule(qr.Q_COINC_HI if hi else qr.Q_COINC)
        for c0 in range(0, len(idx), chunk // 4):
            ii = idx[c0:c0 + chunk // 4]
            # x - y = (u - v)(p1 - p0) with u - v taken exactly from the rule
            dvec = off[None, :, None] * (PA.p1[ea[ii]] - PA.p0[ea[ii]])[:, None, :]
            r = _integrate(PA, ea[ii], PB, fb[ii], u, v, w, dvec, mat)
            h = PA.h[ea[ii]]
            mass = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
            r += 0.5 * (h[:, None, None, None, None] * mass[None, :, :, None, None]
                        * np.eye(2)[None, None, None])
            out[ii] = r
    hi_pair = mat.kT * np.maximum(PA.h[ea], PB.h[fb]) > qr.KH_Q4
    for mask, flip_u, hi in ((nxt, True, False), (prv, False, False), (nxt, True, True), (prv, False, True)):
        mask = mask & (hi_pair == hi)
        if not np.any(mask):
            continue
        idx = np.nonzero(mask)[0]
        up, vp, w = qr.adjacent_rule(qr.Q_ADJ_HI if hi else qr.Q_ADJ)
        if flip_u:      # shared vertex is node 1 of e and node 0 of f
            u, v = 1.0 - up, vp
        else:           # shared vertex is node 0 of e and node 1 of f
            u, v = up, 1.0 - vp
        for c0 in range(0, len(idx), chunk // 8):
            ii = idx[c0:c0 + chunk // 8]
            e_, f_ = ea[ii], fb[ii]
            # x - y = u' (e's far end - c) - v' (f's far end - c), c the shared vertex
            if flip_u:
                A_ = PA.p0[e_] - PA.p1[e_]
                B_ = PB.p1[f_] - PB.p0[f_]
            else:
                A_ = PA.p1[e_] - PA.p0[e_]
                B_ = PB.p0[f_] - PB.p1[f_]
            dvec = up[None, :, None] * A_[:, None, :] - vp[None, :, None] * B_[:, None, :]
            out[ii] = _integrate(PA, e_, PB, f_, u, v, w, dvec, mat)
    if np.any(regular):
        idx = np.nonzero(regular)[0]
        delta = segment_distance(PA.p0[ea[idx]], PA.p1[ea[idx]], PB.p0[fb[idx]], PB.p1[fb[idx]])
        qe, qf = qr.regular_orders(delta, PA.h[ea[idx]], PB.h[fb[idx]], mat.kT)
        code = qe * 100 + qf
        for c in np.unique(code):
            jj = idx[code == c]
            u, v, w = qr.tensor_rule(int(c // 100), int(c % 100))
            step = max(1, chunk * 16 // len(w))
            for c0 in range(0, len(jj), step):
                ii = jj[c0:c0 + step]
                e_, f_ = ea[ii], fb[ii]
                dvec = ((PA.p0[e_] - PB.p0[f_])[:, None, :]
                        + u[None, :, None] * (PA.p1[e_] - PA.p0[e_])[:, None, :]
                        - v[None, :, None] * (PB.p1[f_] - PB.p0[f_])[:, None, :])
                out[ii] = _integrate(PA, e_, PB, f_, u, v, w, dvec, mat)
    return out


def node_block(PA: Polygon, sa, PB: Polygon, tb, mat: Material):
    """Entries A(s, t) as (len(sa), len(tb), 2, 2) for local nodes sa of PA
    (test) and tb of PB (trial)."""
    sa = np.asarray(sa, dtype=np.int64)
    tb = np.asarray(tb, dtype=np.int64)
    # hat of node s lives on element s-1 (as its node 1) and element s (as its node 0)
    re = np.stack([(sa - 1) % PA.n, sa], axis=1)
    ce = np.stack([(tb - 1) % PB.n, tb], axis=1)
    ur, rinv = np.unique(re.ravel(), return_inverse=True)
    uc, cinv = np.unique(ce.ravel(), return_inverse=True)
    rinv = rinv.reshape(-1, 2)
    cinv = cinv.reshape(-1, 2)
    EA = np.repeat(ur, len(uc))
    FB = np.tile(uc, len(ur))
    res = element_pairs(PA, EA, PB, FB, mat).reshape(len(ur), len(uc), 2, 2, 2, 2)
    out = np.zeros((len(sa), len(tb), 2, 2), dtype=np.complex128)
    loc = (1, 0)
    for ks in range(2):
        for kt in range(2):
            out += res[rinv[:, ks][:, None], cinv[:, kt][None, :], loc[ks], loc[kt]]
    return out


class Boundary:
    """The discretised scatterer: one or more closed curves, nodes numbered
    consecutively over the curves in input order."""

    def __init__(self, curves):
        self.polys = [Polygon(c, +1) for c in curves]
        self.offsets = np.cumsum([0] + [p.n for p in self.polys])
        self.n_nodes = int(self.offsets[-1])
        self.curve_of = np.repeat(np.arange(len(self.polys)), [p.n for p in self.polys])
        self.nodes = np.concatenate([p.nodes for p in self.polys])

    def local(self, g):
        g = np.asarray(g, dtype=np.int64)
        c = self.curve_of[g]
        return c, g - self.offsets[c]


def dof_block(bnd: Boundary, rows, cols, mat: Material):
    """Dense block A(rows, cols) for global DOF lists (index 2 t + i)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    rn, ri = rows // 2, rows % 2
    cn, ci = cols // 2, cols % 2
    urn, rmap = np.unique(rn, return_inverse=True)
    ucn, cmap = np.unique(cn, return_inverse=True)
    blk = np.zeros((len(urn), len(ucn), 2, 2), dtype=np.complex128)
    rc, rl = bnd.local(urn)
    cc, cl = bnd.local(ucn)
    for a in np.unique(rc):
        for b in np.unique(cc):
            ia = np.nonzero(rc == a)[0]
            ib = np.nonzero(cc == b)[0]
            blk[np.ix_(ia, ib)] = node_block(bnd.polys[a], rl[ia], bnd.polys[b], cl[ib], mat)
    return blk[rmap[:, None], cmap[None, :], ri[:, None], ci[None, :]]


def dense_matrix(bnd: Boundary, mat: Material):
    """The full 2N x 2N Galerkin matrix (the conventional BEM of Section 8)."""
    n = bnd.n_nodes
    A = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    for a, PA in enumerate(bnd.polys):
        for b, PB in enumerate(bnd.polys):
            blk = node_block(PA, np.arange(PA.n), PB, np.arange(PB.n), mat)
            oa, ob = bnd.offsets[a], bnd.offsets[b]
            for i in range(2):
                for j in range(2):
                    A[2 * oa + i:2 * (oa + PA.n):2, 2 * ob + j:2 * (ob + PB.n):2] = blk[:, :, i, j]
    return A


def incident_field(x, normal, kind: int, angle: float, mat: Material):
    """Plane wave u^I and its traction T^n u^I at points x with normals n.

    kind 0: P-wave u = d exp(i k_L d.x); kind 1: S-wave u = (J d) exp(i k_T d.x);
    d = (cos angle, sin angle), unit amplitude, phase 0 at the origin.
    """
    d = np.array([math.cos(angle), math.sin(angle)])
    dp = np.array([-d[1], d[0]])
    nd = normal @ d
    if kind == 0:
        k = mat.kL
        E = np.exp(1j * k * (x @ d))
        u = E[:, None] * d[None, :]
        t = (1j * k * E)[:, None] * (mat.lam * normal + 2.0 * mat.mu * nd[:, None] * d[None, :])
    else:
        k = mat.kT
        E = np.exp(1j * k * (x @ d))
        ndp = normal @ dp
        u = E[:, None] * dp[None, :]
        t = (1j * k * mat.mu * E)[:, None] * (nd[:, None] * dp[None, :] + ndp[:, None] * d[None, :])
    return u, t


def load_vector(bnd: Boundary, kind: int, angle: float, mat: Material):
    """f with f[2 s + i] = int psi^s (u^I_i + alpha (T u^I)_i) ds (Section 5.2),
    Q_RHS-point Gauss per element."""
    g, w = qr.gauss01(qr.Q_RHS)
    f = np.zeros(2 * bnd.n_nodes, dtype=np.complex128)
    for c, P in enumerate(bnd.polys):
        x = P.p0[:, None, :] + g[None, :, None] * (P.p1 - P.p0)[:, None, :]      # (n, q, 2)
        nrm = np.broadcast_to(P.normal[:, None, :], x.shape)
        u, t = incident_field(x.reshape(-1, 2), nrm.reshape(-1, 2), kind, angle, mat)
        val = (u + mat.alpha * t).reshape(P.n, len(g), 2)
        wh = w[None, :] * P.h[:, None]
        f0 = np.einsum("eq,eqi->ei", wh * (1.0 - g)[None, :], val)   # to node e
        f1 = np.einsum("eq,eqi->ei", wh * g[None, :], val)           # to node e+1
        fn = f0 + np.roll(f1, 1, axis=0)
        o = bnd.offsets[c]
        f[2 * o:2 * (o + P.n)] = fn.reshape(-1)
    return f
