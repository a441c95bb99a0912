"""Linear complexity needs ranks that stay bounded as the mesh is refined at
a fixed frequency (Section 8.2; the proxy surfaces keep the near sets of
fixed size, Section 7.1): on the ellipse of the full case (omega 4, leaf 64,
tol 1e-8) with 2^12, 2^13 and 2^14 nodes the largest skeleton rank and the
root size stay within a few percent while the tree gains a level per
doubling, and each factor solves its system to the accuracy that the
multi-level error at this tolerance allows (against a dense solve of the
same system)."""
import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


# about twice the measured errors (3.0e-7, 6.7e-7, 8.0e-6): a regression of
# the compression at any size fails
ERR_BOUND = {12: 6e-7, 13: 1.4e-6, 14: 1.6e-5}


def test_ranks_bounded_under_refinement(fdsmod):
    stats = []
    for e in (12, 13, 14):
        n = 2 ** e
        print(f"ellipse {n} nodes", flush=True)
        curves = [sy.ellipse(n, 1.0, 0.5)]
        F = fdsmod.Factor(curves, 4.0, 2.0, 1.0, 1.0, 1e-8, leaf=64, autotune=False)
        st = F.stats()
        stats.append(st)
        b = F.rhs_plane([0], [0.0])
        x = F.solve(b)[0]
        dofs = np.arange(2 * n)
        A = fdsmod.entries(curves, 4.0, 2.0, 1.0, 1.0, dofs, dofs)
        xd = torch.linalg.solve(A, b[0])
        err = float(torch.linalg.norm(x - xd) / torch.linalg.norm(xd))
        print(f"ellipse {n} nodes: max rank {st['max_rank']}, root {st['root_size']}, error {err:.2e}", flush=True)
        del A, F
        assert err < ERR_BOUND[e], (n, err)
    lev = [s["levels"] for s in stats]
    assert lev[1] == lev[0] + 1 and lev[2] == lev[1] + 1
    ranks = [s["max_rank"] for s in stats]
    roots = [s["root_size"] for s in stats]
    assert max(ranks) <= 1.1 * min(ranks), ranks
    assert max(roots) <= 1.1 * min(roots), roots
