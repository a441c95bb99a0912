"""The proxy-surface fast direct solver, step by step in plain FP64
(oracle; test infrastructure only).

Follows the paper's algorithm summary (Section 7.3):

1. mesh and binary tree of contiguous node ranges (Section 5.1);
2. leaf index sets J_p;
3. upward loop over levels l = L ... l0+1:
   (a) U_i, V_i and skeletons from proxy-surface interaction matrices and
       interpolative decompositions by column-pivoted QR (Sections 7.1, 7.2);
   (b) A_i^{-1} U_i, A~_i = (V_i A_i^{-1} U_i)^{-1}  (Section 6.2; A_i^{-1}
       is applied through its LU factors, never formed);
   (c) the parent's diagonal block from [[A~_a, R_ab], [R_ba, A~_b]] in
       component-major order (equation of the rearrangement of A, Section 6.2);
4. dense solve of the compressed system at level l0 (Section 6.3);
5. downward loop x_i = A_i^{-1} f_i - A_i^{-1} U_i f~_i + A_i^{-1} U_i A~_i y_i
   (equation of the downward conversion, Section 6.3).

Readings where the paper is silent or ambiguous:
* four skeleton index sets per cell (rows/columns x displacement component);
  each pair (row, column) of a component shares one rank
  k_c = max(k_row, k_col) and uses the first k_c pivots of each pivoted QR
  (pivots are nested), so that A~_i is square;
* the ID rank is the first j with |R_jj| <= tol |R_11|; the pivot is the column of
  largest exactly recomputed remaining norm, ties within a relative 1e-12
  going to the lowest original column index;
* the proxy surface of a cell is an m-gon of radius rho = 1.5 R about the
  centre of the bounding box of the supports of its active hats (R the
  largest distance from that centre to those support nodes), with P1 hats
  and the outward normal; m = max(m_min, ceil(2 k_T rho) + 40) with m_min = 64
  by default: an outgoing field on a circle of radius rho carries Fourier
  modes up to about k_T rho, so the polygon must grow with the frequency
  and the cell size once k_T rho exceeds about 12;
* the near field of a cell at level l is every active row (column) DOF of
  the other level-l cells whose hat support meets the proxy disk;
* entries between overlapping supports include I0/2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import galerkin
from .galerkin import Boundary, Polygon
from .kernels import Material

N_PROXY = 64          # smallest proxy polygon
PROXY_RATIO = 1.5
TIE = 1e-12


# ---------------------------------------------------------------- ID / CPQR
def cpqr(M, kmax=None):
    """Column-pivoted Householder QR, stopped after kmax steps.

    Returns (piv, R) with M[:, piv] = Q R on the computed steps; R is the
    (steps x n) upper-trapezoidal factor in pivoted column order."""
    A = np.array(M, dtype=np.complex128, copy=True)
    m, n = A.shape
    steps = min(m, n) if kmax is None else min(m, n, kmax)
    piv = np.arange(n)
    for j in range(steps):
        norms = np.sum(np.abs(A[j:, j:]) ** 2, axis=0)
        top = norms.max()
        cand = np.nonzero(norms >= top * (1.0 - TIE))[0]
        p = j + cand[np.argmin(piv[j + cand])]
        if p != j:
            A[:, [j, p]] = A[:, [p, j]]
            piv[[j, p]] = piv[[p, j]]
        x = A[j:, j].copy()
        nx = np.linalg.norm(x)
        if nx == 0.0:
            continue
        ph = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        alpha = -ph * nx
        v = x
        v[0] -= alpha
        v /= np.linalg.norm(v)
        A[j:, j:] -= 2.0 * np.outer(v, v.conj() @ A[j:, j:])
        A[j + 1:, j] = 0.0
    return piv, np.triu(A[:steps, :])


def id_rank(R, tol):
    """Rank of the ID: the first j with |R_jj| <= tol |R_11| (the diagonal
    of a pivoted QR with exact norms does not increase)."""
    d = np.abs(np.diag(R))
    if len(d) == 0 or d[0] == 0.0:
        return 0
    small = np.nonzero(d <= tol * d[0])[0]
    return int(small[0]) if len(small) else len(d)


def id_matrix(piv, R, k, n):
    """Interpolation matrix W = [I, R1^{-1} R2] P^T (k x n) of the column ID
    M ~ M[:, piv[:k]] W (Section 7.1)."""
    W = np.zeros((k, n), dtype=np.complex128)
    W[np.arange(k), piv[:k]] = 1.0
    if k < n:
        T = sla.solve_triangular(R[:k, :k], R[:k, k:])
        W[:, piv[k:]] = T
    return W


# ---------------------------------------------------------------- tree
@dataclass
class Cell:
    index: int
    level: int
    lo: int = 0          # leaf node range [lo, hi)
    hi: int = 0
    rows: np.ndarray = None    # active row DOFs (global 2t+i), component-major
    cols: np.ndarray = None
    A: np.ndarray = None       # diagonal block A_i
    lu: tuple = None
    X: np.ndarray = None       # A_i^{-1} U_i
    At: np.ndarray = None      # A~_i
    V: np.ndarray = None
    rskel: np.ndarray = None   # row skeleton DOFs, component-major
    cskel: np.ndarray = None
    k: tuple = (0, 0)
    ranks: dict = field(default_factory=dict)
    centre: np.ndarray = None
    radius: float = 0.0
    n_near: tuple = (0, 0)     # near rows / near columns of the proxy matrices
    n_proxy: int = 0           # vertices of the proxy polygon


def morton_order(centres):
    """Order of the curves along the Morton (Z-order) curve of their centres:
    each coordinate scaled to the bounding box of the centres, quantised to
    16 bits (floor of 65535 times the scaled value), bits interleaved with x
    in the even positions; equal codes keep the input order."""
    C = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
    if len(C) <= 1:
        return np.arange(len(C))
    lo, hi = C.min(axis=0), C.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = np.clip(np.floor((C - lo) / span * 65535.0), 0, 65535).astype(np.int64)
    code = np.zeros(len(C), dtype=np.int64)
    for b in range(16):
        code |= ((q[:, 0] >> b) & 1) << (2 * b)
        code |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return np.argsort(code, kind="stable")


def curve_centres(bnd: Boundary):
    """Bounding-box centre of each curve's nodes."""
    return np.array([0.5 * (p.nodes.min(axis=0) + p.nodes.max(axis=0)) for p in bnd.polys])


def build_tree(bnd: Boundary, leaf: int):
    """Complete binary tree with heap indexing (Section 5.1): cell 0 is the
    root, children of i are 2i+1 and 2i+2, depth L = ceil(log2(N / leaf)).
    Cells are contiguous ranges [lo, hi) of a node numbering that takes the
    curves in Morton order of their centres.  A cell holding two or more
    whole curves splits its curve list into two groups of node counts as
    equal as possible (curves kept whole; ties to the first such split);
    a cell within one curve splits its node range at the midpoint.
    Returns (L, cells, perm) with perm[p] the input index of node p."""
    n_nodes = bnd.n_nodes
    order = morton_order(curve_centres(bnd))
    sizes = np.array([bnd.polys[c].n for c in order])
    perm = np.concatenate([np.arange(bnd.offsets[c], bnd.offsets[c + 1]) for c in order])
    pstart = np.concatenate([[0], np.cumsum(sizes)])
    L = max(0, int(math.ceil(math.log2(n_nodes / leaf)))) if n_nodes > leaf else 0
    cells = {0: Cell(0, 0, 0, n_nodes)}
    cav = {0: (0, len(order))}      # whole curves [a, b) held by a cell; None within one curve
    for lev in range(L):
        for i in range(2 ** lev - 1, 2 ** (lev + 1) - 1):
            c = cells[i]
            g = cav[i]
            if g is not None and g[1] - g[0] >= 2:
                a, b = g
                cand = np.arange(a + 1, b)
                left = pstart[cand] - c.lo
                sp = int(cand[np.argmin(np.abs(2 * left - (c.hi - c.lo)))])
                mid = int(pstart[sp])
                ga, gb = (a, sp), (sp, b)
            else:
                mid = c.lo + (c.hi - c.lo) // 2
                ga = gb = None
            if mid == c.lo or mid == c.hi:
                raise ValueError("a tree cell would have no nodes: use a larger leaf size")
            cells[2 * i + 1] = Cell(2 * i + 1, lev + 1, c.lo, mid)
            cells[2 * i + 2] = Cell(2 * i + 2, lev + 1, mid, c.hi)
            cav[2 * i + 1], cav[2 * i + 2] = ga, gb
    return L, cells, perm


def level_cells(cells, lev):
    return [cells[i] for i in range(2 ** lev - 1, 2 ** (lev + 1) - 1)]


# ---------------------------------------------------------------- helpers
def _node_neighbours(bnd: Boundary, t):
    c, l = bnd.local(t)
    n = np.array([bnd.polys[ci].n for ci in c])
    o = bnd.offsets[c]
    return o + (l - 1) % n, o + (l + 1) % n


def _supports(bnd, nodes):
    pv, nx = _node_neighbours(bnd, nodes)
    return np.unique(np.concatenate([pv, nodes, nx]))


def _seg_dist(c, a, b):
    d = b - a
    t = np.clip(np.einsum("ik,ik->i", c[None, :] - a, d) / np.einsum("ik,ik->i", d, d), 0.0, 1.0)
    q = a + t[:, None] * d
    return np.hypot(q[:, 0] - c[0], q[:, 1] - c[1])


def _support_meets_disk(bnd, nodes, c, rho):
    pv, nx = _node_neighbours(bnd, nodes)
    X = bnd.nodes
    d1 = _seg_dist(c, X[pv], X[nodes])
    d2 = _seg_dist(c, X[nodes], X[nx])
    return np.minimum(d1, d2) < rho


def entries(bnd: Boundary, rows, cols, mat, proxy_rows=None, proxy_cols=None):
    """A(rows, cols) for global DOF lists; a proxy polygon may replace the
    boundary on the row side (proxy_rows) or the column side (proxy_cols),
    in which case rows/cols are DOFs 2s+i of that polygon's nodes."""
    if proxy_rows is None and proxy_cols is None:
        return galerkin.dof_block(bnd, rows, cols, mat)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    if proxy_rows is not None:
        P = proxy_rows
        cn, ci = cols // 2, cols % 2
        out = np.zeros((len(rows), len(cols)), dtype=np.complex128)
        cc, cl = bnd.local(cn)
        rn, ri = rows // 2, rows % 2
        urn, rmap = np.unique(rn, return_inverse=True)
        for b in np.unique(cc):
            ib = np.nonzero(cc == b)[0]
            ucl, cmap = np.unique(cl[ib], return_inverse=True)
            blk = galerkin.node_block(P, urn, bnd.polys[b], ucl, mat)
            out[:, ib] = blk[rmap[:, None], cmap[None, :], ri[:, None], ci[ib][None, :]]
        return out
    P = proxy_cols
    rn, ri = rows // 2, rows % 2
    out = np.zeros((len(rows), len(cols)), dtype=np.complex128)
    rc, rl = bnd.local(rn)
    cn, ci = cols // 2, cols % 2
    ucn, cmap = np.unique(cn, return_inverse=True)
    for a in np.unique(rc):
        ia = np.nonzero(rc == a)[0]
        url, rmap = np.unique(rl[ia], return_inverse=True)
        blk = galerkin.node_block(bnd.polys[a], url, P, ucn, mat)
        out[ia, :] = blk[rmap[:, None], cmap[None, :], ri[ia][:, None], ci[None, :]]
    return out


def proxy_count(k, rho, m_min=N_PROXY):
    """Vertices of the proxy polygon of radius rho at wavenumber k."""
    return max(int(m_min), int(math.ceil(2.0 * k * rho)) + 40)


def proxy_polygon(c, rho, m=N_PROXY):
    t = 2.0 * np.pi * np.arange(m) / m
    return Polygon(np.stack([c[0] + rho * np.cos(t), c[1] + rho * np.sin(t)], axis=1), sign=-1)


def cell_disk(bnd, c):
    """Centre (bounding-box midpoint of the supports of the cell's active
    hats) and radius of a cell."""
    act = np.unique(np.concatenate([c.rows, c.cols]) // 2)
    sup = bnd.nodes[_supports(bnd, act)]
    lo, hi = sup.min(axis=0), sup.max(axis=0)
    c.centre = 0.5 * (lo + hi)
    c.radius = float(np.max(np.hypot(sup[:, 0] - c.centre[0], sup[:, 1] - c.centre[1])))


def interaction_matrices(bnd, mat, c, others, m_min=N_PROXY):
    """Proxy-plus-near interaction matrices of a cell (Sections 7.1, 7.2):
    MV = A(proxy + near rows, cols) and MU = A(rows, proxy + near cols)."""
    rho = PROXY_RATIO * c.radius
    m = proxy_count(mat.kT, rho, m_min)
    P = proxy_polygon(c.centre, rho, m)
    near_r = np.concatenate([o.rows for o in others]) if others else np.zeros(0, np.int64)
    near_c = np.concatenate([o.cols for o in others]) if others else np.zeros(0, np.int64)
    near_r = near_r[_support_meets_disk(bnd, near_r // 2, c.centre, rho)] if len(near_r) else near_r
    near_c = near_c[_support_meets_disk(bnd, near_c // 2, c.centre, rho)] if len(near_c) else near_c
    c.n_near = (len(near_r), len(near_c))
    c.n_proxy = m
    pdofs = np.arange(2 * m)
    MV = entries(bnd, pdofs, c.cols, mat, proxy_rows=P)
    MU = entries(bnd, c.rows, pdofs, mat, proxy_cols=P)
    if len(near_r):
        MV = np.vstack([MV, entries(bnd, near_r, c.cols, mat)])
    if len(near_c):
        MU = np.hstack([MU, entries(bnd, c.rows, near_c, mat)])
    return MV, MU


def compress_cell(bnd, mat, tol, c, others, m_min=N_PROXY):
    """One cell of the upward step (Section 7.3, steps 3a-3b): proxy and
    near interaction matrices (Sections 7.1, 7.2), four IDs, and
    X = A_i^{-1} U_i, A~_i = (V_i X)^{-1} (Section 6.2)."""
    MV, MU = interaction_matrices(bnd, mat, c, others, m_min)
    nc = [int(np.sum(c.cols % 2 == q)) for q in (0, 1)]
    nr = [int(np.sum(c.rows % 2 == q)) for q in (0, 1)]
    assert nc == nr
    Vb, Ub, rsk, csk, ks = [], [], [], [], []
    off = 0
    for q in (0, 1):
        cidx = np.arange(off, off + nc[q])
        pc, Rc = cpqr(MV[:, cidx])
        pr, Rr = cpqr(MU[cidx, :].conj().T)
        kc, kr = id_rank(Rc, tol), id_rank(Rr, tol)
        k = max(kc, kr)
        c.ranks[q] = (kr, kc)
        Vb.append(id_matrix(pc, Rc, k, nc[q]))
        Ub.append(id_matrix(pr, Rr, k, nc[q]).conj().T)
        csk.append(c.cols[cidx][pc[:k]])
        rsk.append(c.rows[cidx][pr[:k]])
        ks.append(k)
        off += nc[q]
    c.k = tuple(ks)
    c.V = sla.block_diag(*Vb)
    U = sla.block_diag(*Ub)
    c.cskel = np.concatenate(csk)
    c.rskel = np.concatenate(rsk)
    c.lu = sla.lu_factor(c.A)
    c.X = sla.lu_solve(c.lu, U)
    S = c.V @ c.X
    c.At = np.linalg.inv(S)


def leaf_sample(curves, lam, mu, rho, omega, tol, leaf, sample):
    """The upward-step work of a few leaf cells of the full tree (leaf block
    assembly plus compress_cell), for timing the oracle on a bounded sample.
    Returns the cells."""
    mat = Material(lam, mu, rho, omega)
    bnd = Boundary(curves)
    L, cells, perm = build_tree(bnd, leaf)
    leaves = level_cells(cells, L)
    for c in leaves:
        nodes = perm[c.lo:c.hi]
        c.rows = np.concatenate([2 * nodes, 2 * nodes + 1])
        c.cols = c.rows.copy()
    out = []
    for q in sample:
        c = leaves[q]
        c.A = entries(bnd, c.rows, c.cols, mat)
        cell_disk(bnd, c)
        compress_cell(bnd, mat, tol, c, [o for o in leaves if o is not c])
        out.append(c)
    return out


def _stand_in_sets(perm, cells, lev, L, k):
    """Active DOFs of every level-lev cell for the timing samples: at the
    leaves all of the cell's DOFs; above them, per component, k evenly
    spaced nodes of each child's node range, ordered as the rearrangement
    orders skeletons (child a, child b, component by component).  They have
    the sizes of skeletons of rank k, not their positions."""
    out = []
    for c in level_cells(cells, lev):
        if lev == L:
            nodes = perm[c.lo:c.hi]
            c.rows = np.concatenate([2 * nodes, 2 * nodes + 1])
        else:
            a, b = cells[2 * c.index + 1], cells[2 * c.index + 2]
            pick = [perm[ch.lo + (np.arange(min(k, ch.hi - ch.lo)) * (ch.hi - ch.lo)) // max(1, min(k, ch.hi - ch.lo))]
                    for ch in (a, b)]
            c.rows = np.concatenate([2 * pick[0], 2 * pick[1], 2 * pick[0] + 1, 2 * pick[1] + 1])
        c.cols = c.rows.copy()
        out.append(c)
    return out


def level_sample(curves, lam, mu, rho, omega, tol, leaf, lev, k, sample):
    """Timing sample of one level of the factorisation: every level-lev cell
    gets the stand-in active DOFs of _stand_in_sets (rank k above the
    leaves), then each sampled cell's diagonal block is assembled and
    compress_cell runs on it (the work of one cell of the upward loop,
    Section 7.3 step 3).  Returns a list of (seconds, ranks) per sampled
    cell; only the timing and the sizes are meaningful."""
    import time
    mat = Material(lam, mu, rho, omega)
    bnd = Boundary(curves)
    L, cells, perm = build_tree(bnd, leaf)
    cs = _stand_in_sets(perm, cells, lev, L, k)
    out = []
    for q in sample:
        c = cs[q]
        t0 = time.perf_counter()
        c.A = entries(bnd, c.rows, c.cols, mat)
        cell_disk(bnd, c)
        compress_cell(bnd, mat, tol, c, [o for o in cs if o is not c])
        out.append((time.perf_counter() - t0, c.k))
    return out


def root_sample(curves, lam, mu, rho, omega, leaf, root_level, k):
    """Timing sample of the root step (Section 7.3 step 4): the compressed
    system of the level-root_level cells with stand-in skeletons of rank k
    assembled and LU-factored.  Returns (seconds, order)."""
    import time
    mat = Material(lam, mu, rho, omega)
    bnd = Boundary(curves)
    L, cells, perm = build_tree(bnd, leaf)
    top = _stand_in_sets(perm, cells, min(root_level, L), L, k)
    rows = np.concatenate([c.rows for c in top])
    cols = np.concatenate([c.cols for c in top])
    t0 = time.perf_counter()
    sla.lu_factor(entries(bnd, rows, cols, mat))
    return time.perf_counter() - t0, len(rows)


# ---------------------------------------------------------------- factor
class FDS:
    """Factorisation of the Galerkin system; ``solve`` applies it."""

    def __init__(self, curves, lam, mu, rho, omega, tol, leaf=64, root_level=1, alpha=None, n_proxy=N_PROXY):
        self.mat = Material(lam, mu, rho, omega, alpha)
        self.n_proxy = int(n_proxy)
        self.bnd = Boundary(curves)
        self.tol = float(tol)
        self.L, self.cells, self.perm = build_tree(self.bnd, leaf)
        self.l0 = min(root_level, self.L)
        self._factor()

    def _compress_level(self, lev):
        bnd, mat = self.bnd, self.mat
        cells = level_cells(self.cells, lev)
        for c in cells:
            cell_disk(bnd, c)
        for c in cells:
            compress_cell(bnd, mat, self.tol, c, [o for o in cells if o is not c], self.n_proxy)

    def _merge(self, lev):
        """Diagonal blocks of the level-(lev-1) cells (rearrangement, Section 6.2)."""
        bnd, mat = self.bnd, self.mat
        for p in level_cells(self.cells, lev - 1):
            a, b = self.cells[2 * p.index + 1], self.cells[2 * p.index + 2]
            ka, kb = a.k, b.k
            p.rows = np.concatenate([a.rskel[:ka[0]], b.rskel[:kb[0]], a.rskel[ka[0]:], b.rskel[kb[0]:]])
            p.cols = np.concatenate([a.cskel[:ka[0]], b.cskel[:kb[0]], a.cskel[ka[0]:], b.cskel[kb[0]:]])
            # position of each parent DOF inside its child's skeleton list
            own_r = np.concatenate([np.zeros(ka[0], int), np.ones(kb[0], int), np.zeros(ka[1], int), np.ones(kb[1], int)])
            pos_r = np.concatenate([np.arange(ka[0]), np.arange(kb[0]), ka[0] + np.arange(ka[1]), kb[0] + np.arange(kb[1])])
            A = entries(bnd, p.rows, p.cols, mat)
            ia = np.nonzero(own_r == 0)[0]
            ib = np.nonzero(own_r == 1)[0]
            A[np.ix_(ia, ia)] = a.At[np.ix_(pos_r[ia], pos_r[ia])]
            A[np.ix_(ib, ib)] = b.At[np.ix_(pos_r[ib], pos_r[ib])]
            p.A = A
            p.own, p.pos = own_r, pos_r

    def _factor(self):
        bnd, mat = self.bnd, self.mat
        for c in level_cells(self.cells, self.L):
            nodes = self.perm[c.lo:c.hi]
            c.rows = np.concatenate([2 * nodes, 2 * nodes + 1])
            c.cols = c.rows.copy()
            c.A = entries(bnd, c.rows, c.cols, mat)
        for lev in range(self.L, self.l0, -1):
            self._compress_level(lev)
            self._merge(lev)
        top = level_cells(self.cells, self.l0)
        self.root_rows = np.concatenate([c.rows for c in top])
        self.root_cols = np.concatenate([c.cols for c in top])
        Ar = entries(bnd, self.root_rows, self.root_cols, mat)
        o = 0
        for c in top:
            n = len(c.rows)
            Ar[o:o + n, o:o + n] = c.A
            o += n
        self.root_A = Ar
        self.root_lu = sla.lu_factor(Ar)

    # ------------------------------------------------------------ solve
    def solve(self, F):
        F = np.asarray(F, dtype=np.complex128)
        one = F.ndim == 1
        if one:
            F = F[:, None]
        f = {}
        g = {}
        ft = {}
        for c in level_cells(self.cells, self.L):
            f[c.index] = F[c.rows]
        for lev in range(self.L, self.l0, -1):
            for c in level_cells(self.cells, lev):
                g[c.index] = sla.lu_solve(c.lu, f[c.index])
                ft[c.index] = c.At @ (c.V @ g[c.index])
            for p in level_cells(self.cells, lev - 1):
                a, b = 2 * p.index + 1, 2 * p.index + 2
                fa, fb = ft[a], ft[b]
                ka, kb = self.cells[a].k, self.cells[b].k
                f[p.index] = np.vstack([fa[:ka[0]], fb[:kb[0]], fa[ka[0]:], fb[kb[0]:]])
        top = level_cells(self.cells, self.l0)
        xr = sla.lu_solve(self.root_lu, np.vstack([f[c.index] for c in top]))
        x = {}
        o = 0
        for c in top:
            n = len(c.cols)
            x[c.index] = xr[o:o + n]
            o += n
        for lev in range(self.l0 + 1, self.L + 1):
            for c in level_cells(self.cells, lev):
                p = self.cells[(c.index - 1) // 2]
                side = 0 if c.index == 2 * p.index + 1 else 1
                sel = np.nonzero(p.own == side)[0]
                y = np.empty((len(c.cskel), F.shape[1]), dtype=np.complex128)
                y[p.pos[sel]] = x[p.index][sel]
                x[c.index] = g[c.index] + c.X @ (c.At @ y - ft[c.index])
        out = np.zeros_like(F)
        for c in level_cells(self.cells, self.L):
            out[c.cols] = x[c.index]
        return out[:, 0] if one else out

    def rank_table(self):
        return {i: (c.level, c.k, c.ranks) for i, c in self.cells.items() if c.ranks}
