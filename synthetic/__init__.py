"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *generates inputs*: polygon node coordinates of the
scatterers and the list of incident plane waves.  It contains none of the
solver's arithmetic (no normals, no kernels, no quadrature, no linear
algebra), so the CPU oracle and the GPU path can both consume it without
sharing any computation.

Geometry convention: every closed curve is returned as an ``(n, 2)`` float64
array of vertices in counter-clockwise order; the polygon is closed
implicitly (the last vertex connects back to the first).  The paper
approximates the boundary by an N-gon whose vertices are the nodes
(Section 4).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "field_targets",
    "random_boundary_values",
    "circle",
    "ellipse",
    "tripod",
    "multi_cavity",
    "plane_wave_angles",
    "config_small",
    "config_scale",
]


def circle(n: int, radius: float = 1.0, center=(0.0, 0.0), phase: float = 0.0) -> np.ndarray:
    """n vertices uniformly spaced on a circle, counter-clockwise."""
    t = phase + 2.0 * np.pi * np.arange(n) / n
    return np.stack([center[0] + radius * np.cos(t), center[1] + radius * np.sin(t)], axis=1)


def ellipse(n: int, a: float = 1.0, b: float = 0.5, center=(0.0, 0.0), angle: float = 0.0) -> np.ndarray:
    """n vertices uniform in the parameter angle of an ellipse with semi-axes a, b,
    rotated by ``angle`` about its centre; counter-clockwise."""
    t = 2.0 * np.pi * np.arange(n) / n
    px, py = a * np.cos(t), b * np.sin(t)
    c, s = math.cos(angle), math.sin(angle)
    return np.stack([center[0] + c * px - s * py, center[1] + s * px + c * py], axis=1)


def _ellipse_perimeter(a: float, b: float) -> float:
    # Ramanujan's second approximation
    h = ((a - b) / (a + b)) ** 2
    return math.pi * (a + b) * (1.0 + 3.0 * h / (10.0 + math.sqrt(4.0 - 3.0 * h)))


def multi_cavity(seed: int, n_cavities: int, total_nodes: int, half_width: float = 20.0,
                 radius_range=(0.2, 1.0), aspect_range=(0.5, 1.0), separation: float = 0.5,
                 min_nodes: int = 32, max_tries: int = 200000):
    """Seeded non-overlapping elliptical cavities.

    Centres uniform in [-half_width, half_width]^2, major semi-axis uniform in
    ``radius_range``, aspect ratio (minor/major) uniform in ``aspect_range``,
    orientation uniform in [0, pi).  A candidate is rejected when its
    circumscribed circle comes within ``separation`` of an accepted one.
    Node counts are proportional to the perimeters (largest-remainder
    rounding, each at least ``min_nodes``) and sum to ``total_nodes``.

    Returns a list of ``(n_i, 2)`` arrays.
    """
    rng = np.random.default_rng(seed)
    cav = []
    tries = 0
    while len(cav) < n_cavities:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place cavities")
        c = rng.uniform(-half_width, half_width, size=2)
        a = rng.uniform(*radius_range)
        asp = rng.uniform(*aspect_range)
        ang = rng.uniform(0.0, math.pi)
        ok = True
        for (c2, a2, _, _) in cav:
            if math.hypot(c[0] - c2[0], c[1] - c2[1]) < a + a2 + separation:
                ok = False
                break
        if ok:
            cav.append((c, a, asp, ang))
    per = np.array([_ellipse_perimeter(a, a * asp) for (_, a, asp, _) in cav])
    if total_nodes < min_nodes * n_cavities:
        raise ValueError("total_nodes too small")
    spare = total_nodes - min_nodes * n_cavities
    share = spare * per / per.sum()
    base = np.floor(share).astype(np.int64)
    rem = spare - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    counts = base + min_nodes
    assert int(counts.sum()) == total_nodes
    return [ellipse(int(m), a, a * asp, center=(c[0], c[1]), angle=ang)
            for (c, a, asp, ang), m in zip(cav, counts)]


def tripod(n: int, r: float = 1.0, a: float = 0.3, b: float = 3.0) -> np.ndarray:
    """The scatterer of the paper's numerical examples (Section 8, figure of
    the scatterer): x = (r + a cos(b t)) (cos t, sin t) / (1 + a), n vertices
    uniform in t, counter-clockwise."""
    t = 2.0 * np.pi * np.arange(n) / n
    rad = (r + a * np.cos(b * t)) / (1.0 + a)
    return np.stack([rad * np.cos(t), rad * np.sin(t)], axis=1)


def config_tripod(n: int, tol: float, single_level: bool = False):
    """Accuracy experiment of Section 8.1 (Tables 1 and 2): the tripod with n
    nodes, c_L = sqrt(3), c_T = 1, rho = 1 (so mu = 1, lambda = 1), omega = 2,
    cells of 100 nodes (L = log2(n / 100)), root at level 1 (multi-level) or
    at level L - 1 (single-level variant), one plane P-wave at angle 0."""
    L = int(round(math.log2(n / 100)))
    return dict(curves=[tripod(n)], lam=1.0, mu=1.0, rho=1.0, omega=2.0, tol=tol, leaf=100,
                root_level=(L - 1) if single_level else 1, L=L)


def plane_wave_angles(nrhs: int, step_deg: float = 2.0) -> np.ndarray:
    """Incidence angles 0, step, 2 step, ... in radians."""
    return np.deg2rad(step_deg * np.arange(nrhs))


def config_small():
    """Small validation case: circle of radius 1 with 256 nodes, lambda=2, mu=1,
    rho=1, omega=1 (k_T a = 1), leaf 32 nodes, ID tolerance 1e-10, one plane
    P-wave at incidence angle 0."""
    return dict(curves=[circle(256)], lam=2.0, mu=1.0, rho=1.0, omega=1.0, tol=1e-10,
                leaf=32, kinds=[0], angles=[0.0])


def config_scale(nrhs: int = 180):
    """Full-size case: ellipse with semi-axes 1 and 0.5, 131072 nodes
    (262144 complex unknowns), lambda=2, mu=1, rho=1, omega=4 (k_T a = 4),
    leaf 64 nodes, ID tolerance 1e-8, plane P-waves at 0, 2, ..., 358 degrees."""
    return dict(curves=[ellipse(131072, 1.0, 0.5)], lam=2.0, mu=1.0, rho=1.0, omega=4.0,
                tol=1e-8, leaf=64, kinds=[0] * nrhs, angles=list(plane_wave_angles(nrhs)))


def config_batching(nrhs: int = 180):
    """Uneven-leaf case: 64 cavities (seed 3) in [-20, 20]^2, 65536 nodes,
    lambda=2, mu=1, rho=1, omega=2 (k_T = 2), leaf 64 nodes on average, ID
    tolerance 1e-8, plane waves at 0, 2, ..., 358 degrees alternating P
    (even index) and S (odd index)."""
    return dict(curves=multi_cavity(3, 64, 65536), lam=2.0, mu=1.0, rho=1.0, omega=2.0, tol=1e-8, leaf=64,
                kinds=[k % 2 for k in range(nrhs)], angles=list(plane_wave_angles(nrhs)))


def training_geometry(i: int, nodes: int = 16384):
    """Training geometry i of the rank predictor: seed 1000 + i, between 8
    and 40 cavities in [-20, 20]^2 with ``nodes`` nodes in total, and k_T
    uniform in [1, 10] (omega = k_T for mu = rho = 1).  Returns (curves, k_T)."""
    rng = np.random.default_rng(1000 + i)
    n_cav = int(rng.integers(8, 41))
    k_t = float(rng.uniform(1.0, 10.0))
    return multi_cavity(1000 + i, n_cav, nodes), k_t


def config_learned_eval():
    """Evaluation case of the rank predictor: 128 cavities (seed 5), 131072
    nodes (262144 complex unknowns), k_T = 8, lambda=2, mu=1, rho=1, leaf 64,
    ID tolerance 1e-8."""
    return dict(curves=multi_cavity(5, 128, 131072), lam=2.0, mu=1.0, rho=1.0, omega=8.0, tol=1e-8, leaf=64)


def random_boundary_values(n_unknowns: int, nrhs: int, seed: int) -> np.ndarray:
    """Seeded complex nodal values (nrhs, n_unknowns), real and imaginary
    parts standard normal: inputs for checks of operations that are linear
    in the boundary solution."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, n_unknowns)) + 1j * rng.standard_normal((nrhs, n_unknowns))


def field_targets(curves, seed: int, n_far: int = 12, n_mid: int = 8,
                  scales=(0.2, 0.05, 0.01, 0.002, 0.0005, 0.00005), n_inside: int = 4) -> np.ndarray:
    """Seeded evaluation points around star-shaped curves: ``n_far`` on a
    circle of 2.5 times the largest node radius about the centroid of all
    nodes; per curve, ``n_mid`` random edge midpoints pushed away from the
    curve's centroid by each factor in ``scales`` (1 + s), which puts them
    at distances from about 1/5 of the curve size down to far below one
    element length; and ``n_inside`` points pulled towards the centroid,
    inside the curve.  Returns an (M, 2) float64 array."""
    rng = np.random.default_rng(seed)
    allp = np.concatenate(curves)
    c0 = allp.mean(axis=0)
    rad = 2.5 * np.max(np.linalg.norm(allp - c0, axis=1))
    th = rng.uniform(0.0, 2.0 * math.pi, n_far)
    pts = [c0 + rad * np.stack([np.cos(th), np.sin(th)], axis=1)]
    for nodes in curves:
        cc = nodes.mean(axis=0)
        n = len(nodes)
        e = rng.integers(0, n, n_mid)
        mid = 0.5 * (nodes[e] + nodes[(e + 1) % n])
        for s in scales:
            pts.append(cc + (1.0 + s) * (mid - cc))
        e = rng.integers(0, n, n_inside)
        mid = 0.5 * (nodes[e] + nodes[(e + 1) % n])
        pts.append(cc + rng.uniform(0.1, 0.7, n_inside)[:, None] * (mid - cc))
    return np.concatenate(pts)
