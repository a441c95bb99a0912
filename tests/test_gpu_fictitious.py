"""Fictitious eigenfrequencies (Section 8.4, the wave-intensity figure): on
the tripod, the equation without the Burton-Miller term (alpha = 0, the
non-BM equation of that section) becomes nearly singular at isolated real
frequencies, while the Burton-Miller system of Section 3 does not, and the
factor of the Burton-Miller system reproduces its dense solve there.
omega = 4.55 is the first such frequency of the 400-node tripod on the
0.05 grid (the bench's sweep over 0.05 ... 40 finds about fifty); omega = 3
is an ordinary frequency for reference."""
import numpy as np
import pytest
import scipy.linalg as sla

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


def _sigma_min(A):
    return float(np.linalg.svd(A, compute_uv=False)[-1])


def _case(fdsmod, omega, alpha):
    curves = [sy.tripod(400)]
    dofs = np.arange(800)
    A = fdsmod.entries(curves, omega, 1.0, 1.0, 1.0, dofs, dofs, alpha=alpha).cpu().numpy()
    F = fdsmod.Factor(curves, omega, 1.0, 1.0, 1.0, 1e-8, leaf=100, alpha=alpha, autotune=False)
    b = F.rhs_plane([0], [0.0])
    x = F.solve(b).cpu().numpy()[0]
    return A, b.cpu().numpy()[0], x


def test_burton_miller_removes_the_fictitious_frequency(fdsmod):
    s = {}
    for omega in (3.0, 4.55):
        for alpha in (None, 0.0):
            A, b, x = _case(fdsmod, omega, alpha)
            s[(omega, alpha)] = _sigma_min(A)
            if alpha is None:
                # the factor of the Burton-Miller system agrees with its dense solve
                xd = sla.solve(A, b)
                assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-6
    # alpha = 0: the smallest singular value collapses at the fictitious frequency
    assert s[(4.55, 0.0)] < 0.1 * s[(3.0, 0.0)]
    # Burton-Miller: no such collapse
    assert s[(4.55, None)] > 0.3 * s[(3.0, None)]


def test_nonbm_intensity_spikes_where_burton_miller_stays_smooth(fdsmod):
    # omega located by golden-section search on the smallest singular value of
    # the alpha = 0 matrix near the 0.05-grid dip at 35.70 (the bench's sweep)
    omega = 35.700482
    A0, b0, _ = _case(fdsmod, omega, 0.0)
    A, b, x = _case(fdsmod, omega, None)
    i_nbm = (abs(sla.solve(A0, b0)[:2]) ** 2).sum()
    xd = sla.solve(A, b)
    i_bm = (abs(xd[:2]) ** 2).sum()
    i_fds = (abs(x[:2]) ** 2).sum()
    assert abs(i_fds - i_bm) / i_bm < 1e-6
    assert abs(i_nbm - i_bm) / i_bm > 1.0
