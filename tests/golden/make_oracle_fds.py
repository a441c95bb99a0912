"""Writes the oracle's fast-direct-solver results that the GPU parity tests
compare against (tests/golden/oracle_fds_<name>.npz).

Calls only ``oracle/`` (and the seeded input generators of ``synthetic/``):
for each named case it factors the system with ``oracle.fds.FDS`` (the
algorithm summary of Section 7.3, step by step in plain FP64), solves the
listed plane waves and stores, per compressed cell, the four ID ranks, the
row and column skeletons and the proxy polygon size, plus the solutions.

Usage:  python tests/golden/make_oracle_fds.py [name ...]   (default: all)
Each case runs in its own process; the 16384-node ellipse takes about half
an hour on one core, the others a minute or less.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

os.environ.setdefault("OMP_NUM_THREADS", "1")       # one BLAS thread per case process
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402


def cases():
    """name -> (curves, lam, mu, rho, omega, tol, leaf, root_level, alpha, n_proxy, kinds, angles).
    root_level None = L - 1 (the single-level variant of Table 2)."""
    import synthetic as sy
    trip = [sy.tripod(800)]
    base = dict(lam=1.0, mu=1.0, rho=1.0, omega=2.0, tol=1e-8, leaf=100, root_level=1, alpha=None, n_proxy=64,
                kinds=[0], angles=[0.0])
    out = {
        # the full-size ellipse's parameters at 2^14 nodes (L = 8)
        "ellipse16384": dict(curves=[sy.ellipse(16384, 1.0, 0.5)], lam=2.0, mu=1.0, rho=1.0, omega=4.0, tol=1e-8,
                             leaf=64, root_level=1, alpha=None, n_proxy=64, kinds=[0, 1], angles=[0.0, 1.3]),
        # the paper's tripod (Section 8.1 material and cell size), 800 nodes, L = 3
        "tripod800": dict(base, curves=trip),
        "tripod800_single_level": dict(base, curves=trip, root_level=None),
        "tripod800_alpha0": dict(base, curves=trip, alpha=0.0),
        "tripod800_proxy128": dict(base, curves=trip, n_proxy=128),
        # omega = 14.5: proxy polygons above 64 vertices at level 2, 6-point proxy pairs
        "tripod800_w14.5": dict(base, curves=trip, omega=14.5),
        # 8 cavities at k_T = 8: proxy polygons of several hundred vertices at the top levels.
        # Every cavity gets an odd node count (the last node of an even one is
        # dropped): an ellipse sampled at 2 pi t / n with n even is centrally
        # symmetric, so in a cell that holds just that cavity (proxy circle about
        # its centre) DOF pairs tie exactly in the pivoted QR, and two
        # implementations may break such a tie differently.
        "cavities8_w8": dict(curves=[c if len(c) % 2 else c[:-1] for c in sy.multi_cavity(5, 8, 1024)], lam=2.0,
                             mu=1.0, rho=1.0, omega=8.0, tol=1e-8, leaf=64, root_level=1, alpha=None, n_proxy=64,
                             kinds=[0, 1], angles=[0.0, 2.0]),
    }
    return out


def run_case(name):
    from oracle import fds as ofds, galerkin
    from oracle.kernels import Material
    c = cases()[name]
    t0 = time.time()
    import math
    n_nodes = sum(len(x) for x in c["curves"])
    rl = c["root_level"]
    if rl is None:
        rl = max(0, int(math.ceil(math.log2(n_nodes / c["leaf"]))) - 1)
    F = ofds.FDS(c["curves"], c["lam"], c["mu"], c["rho"], c["omega"], c["tol"], leaf=c["leaf"], root_level=rl,
                 alpha=c["alpha"], n_proxy=c["n_proxy"])
    mat = Material(c["lam"], c["mu"], c["rho"], c["omega"], c["alpha"])
    bnd = galerkin.Boundary(c["curves"])
    rhs = np.stack([galerkin.load_vector(bnd, k, a, mat) for k, a in zip(c["kinds"], c["angles"])], axis=1)
    X = F.solve(rhs)
    cells = sorted(i for i, cl in F.cells.items() if cl.ranks)
    ranks = np.array([[F.cells[i].ranks[0][0], F.cells[i].ranks[0][1], F.cells[i].ranks[1][0],
                       F.cells[i].ranks[1][1]] for i in cells], dtype=np.int64)
    rsk = [np.asarray(F.cells[i].rskel, dtype=np.int64) for i in cells]
    csk = [np.asarray(F.cells[i].cskel, dtype=np.int64) for i in cells]
    off = np.cumsum([0] + [len(r) for r in rsk])
    np.savez_compressed(
        os.path.join(HERE, f"oracle_fds_{name}.npz"),
        cells=np.array(cells, dtype=np.int64), ranks=ranks, rskel=np.concatenate(rsk), cskel=np.concatenate(csk),
        skel_off=off, n_proxy_cell=np.array([F.cells[i].n_proxy for i in cells], dtype=np.int64),
        levels=np.int64(F.L), root_level=np.int64(F.l0), root_size=np.int64(len(F.root_rows)),
        kinds=np.array(c["kinds"], dtype=np.int64), angles=np.array(c["angles"], dtype=np.float64), x=X.T.copy())
    return name, time.time() - t0


def main(names):
    names = names or list(cases())
    with cf.ProcessPoolExecutor(max_workers=min(len(names), os.cpu_count() or 1)) as ex:
        for name, dt in ex.map(run_case, names):
            print(f"{name}: {dt:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
