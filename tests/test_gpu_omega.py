"""Angular frequency (Section 8.4, the elapsed-time and error figures): on
the 6400-node tripod at tol 1e-8, at both ends of the paper's range
(omega = 0.5 and 14.5), the factor's solution agrees with a dense solve of
the same system to within ten times the paper's Table 1 error for this size
and tolerance, and a proxy polygon of twice the vertices (128 instead of 64)
changes the solution by no more than that: the default proxy resolution
still holds at the top of the range."""
import os

import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tripod_error_tables.txt")


def _paper_error(table, n, eps):
    for line in open(GOLDEN):
        f = line.split()
        if f and not line.startswith("#") and int(f[0]) == table and int(f[1]) == n and float(f[4]) == eps:
            return float(f[5])
    raise KeyError((table, n, eps))


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


@pytest.mark.parametrize("omega", [0.5, 14.5])
def test_error_flat_across_the_frequency_range(fdsmod, omega):
    n = 6400
    bound = 10.0 * _paper_error(1, n, 1e-8)
    c = sy.config_tripod(n, 1e-8)
    xs = {}
    for npx in (64, 128):
        F = fdsmod.Factor(c["curves"], omega, c["lam"], c["mu"], c["rho"], c["tol"], leaf=c["leaf"],
                          n_proxy=npx, autotune=False)
        b = F.rhs_plane([0], [0.0])
        xs[npx] = F.solve(b)[0]
        if npx == 64:
            rhs = b[0]
            assert F.stats()["max_rank"] <= 64
        del F
    dofs = np.arange(2 * n)
    A = fdsmod.entries(c["curves"], omega, c["lam"], c["mu"], c["rho"], dofs, dofs)
    ref = torch.linalg.solve(A, rhs)
    del A
    nref = torch.linalg.norm(ref)
    assert float(torch.linalg.norm(xs[64] - ref) / nref) < bound
    assert float(torch.linalg.norm(xs[128] - ref) / nref) < bound
    assert float(torch.linalg.norm(xs[128] - xs[64]) / nref) < bound
