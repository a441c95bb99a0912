"""GPU factorisation against the oracle's fast direct solver on the same tree,
case by case (results of the oracle stored by tests/golden/make_oracle_fds.py,
which calls only ``oracle/``):

* the full-size ellipse's parameters at 2^14 nodes (omega = 4, leaf 64,
  tol 1e-8, L = 8, 511 cells): every compressed cell's four ranks and both
  skeletons identical, the solutions of a P- and an S-wave element-wise
  within 1e-10 of the largest oracle value;
* the paper's tripod (800 nodes, Section 8.1 material, cells of 100 nodes):
  root at level 1, the single-level variant (root at L - 1, Table 2), the
  equation without the Burton-Miller term (alpha = 0), 128-vertex proxy
  polygons, and omega = 14.5 (proxy polygons grown past 64 vertices at
  level 2 and their pairs on the 6-point rule);
* eight cavities at k_T = 8 (proxy polygons of a few hundred vertices at the
  top levels).

Tolerance: the two sides take the same decisions (pivots, ranks) from
independently computed entries that agree to rounding; the solutions then
differ by rounding amplified by the small dense blocks' conditioning.
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_oracle_fds as golden  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAMES = ["ellipse16384", "tripod800", "tripod800_single_level", "tripod800_alpha0", "tripod800_proxy128",
         "tripod800_w14.5", "cavities8_w8"]


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


@pytest.mark.parametrize("name", NAMES)
def test_factor_and_solutions_match_oracle(fdsmod, name):
    print(f"case {name}", flush=True)
    g = np.load(os.path.join(HERE, "golden", f"oracle_fds_{name}.npz"), allow_pickle=False)
    c = golden.cases()[name]
    F = fdsmod.Factor(c["curves"], c["omega"], c["lam"], c["mu"], c["rho"], c["tol"], leaf=c["leaf"],
                      n_proxy=c["n_proxy"], root_level=int(g["root_level"]), alpha=c["alpha"])
    st = F.stats()
    assert st["levels"] == int(g["levels"]) and st["root_level"] == int(g["root_level"])
    assert st["root_size"] == int(g["root_size"])
    rk = F.ranks()
    off = g["skel_off"]
    for i, cell in enumerate(g["cells"]):
        assert tuple(rk[cell]) == tuple(g["ranks"][i]), (name, int(cell))
        r, cc = F.skeleton(int(cell))
        assert np.array_equal(r, g["rskel"][off[i]:off[i + 1]]), (name, int(cell))
        assert np.array_equal(cc, g["cskel"][off[i]:off[i + 1]]), (name, int(cell))
    x = F.solve(F.rhs_plane(list(g["kinds"]), list(g["angles"]))).cpu().numpy().reshape(len(g["kinds"]), -1)
    xo = g["x"]
    for j in range(len(xo)):
        assert np.max(np.abs(x[j] - xo[j])) <= 1e-10 * np.max(np.abs(xo[j])), (name, j)
