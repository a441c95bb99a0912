"""Matrix-core upward sweep (one launch per level: LU solve with inverted
16 x 16 diagonal blocks and f~ = (A~ V) g on FP64 16x16x4 products) against
the LU-solve and GEMM kernels of the same factor (mfma_sweeps=0), through
the C ABI.  The two differ only in rounding (the inverted diagonal blocks,
W = A~ V formed once); the compressed system's conditioning (about 1e5 at
the largest size) amplifies unit roundoff to some 1e-10 (measured 1.1e-10
at tol 1e-11, where the blocks are largest), so every solution column must
agree within 1e-9 of its largest value, as the GPU and oracle solutions
do.  Cases: the full-size ellipse
at tol 1e-8 and 1e-11 (blocks of 128 to about 250 unknowns), the 6400-node
tripod (cells of 100 nodes: partial 16-row blocks), the uneven 64-cavity
leaves, and column counts 1 to 4 (one workgroup per cell on the vector
units), 5 (LU-solve kernel and a GEMM with A~ V), 16, 17 and 179 (partial
and several 16-column slabs); graph replays equal the eager runs bitwise."""
import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "ellipse131072_tol1e-8": (lambda: [sy.ellipse(131072, 1.0, 0.5)], (4.0, 2.0, 1.0, 1.0, 1e-8), 64),
    "ellipse131072_tol1e-11": (lambda: [sy.ellipse(131072, 1.0, 0.5)], (4.0, 2.0, 1.0, 1.0, 1e-11), 64),
    "tripod6400": (lambda: [sy.tripod(6400)], (2.0, 1.0, 1.0, 1.0, 1e-8), 100),
    "cavities64": (lambda: sy.config_batching()["curves"], (2.0, 2.0, 1.0, 1.0, 1e-8), 64),
}


def _cmp(x, y):
    d = torch.abs(x - y).amax(dim=-1)
    m = torch.abs(y).amax(dim=-1)
    return float((d / m).max())


@pytest.mark.parametrize("name", list(CASES))
def test_matrix_core_sweeps_match_gemm_sweeps(name):
    import paper_2411_18026_amd as fds
    make, (omega, lam, mu, rho, tol), leaf = CASES[name]
    curves = make()
    print(f"case {name}", flush=True)
    Fm = fds.Factor(curves, omega, lam, mu, rho, tol, leaf=leaf)
    Fg = fds.Factor(curves, omega, lam, mu, rho, tol, leaf=leaf, mfma_sweeps=False)
    assert np.array_equal(Fm.ranks(), Fg.ranks())
    n = 179
    rhs = Fm.rhs_plane([k % 2 for k in range(n)], sy.plane_wave_angles(n))
    for cols in (1, 2, 3, 4, 5, 16, 17, 179):
        xm = Fm.solve(rhs[:cols])
        xg = Fg.solve(rhs[:cols])
        e = _cmp(xm, xg)
        print(f"{name} cols {cols}: {e:.2e}", flush=True)
        assert e < 1e-9, (name, cols)
    # a column alone or among others of the same path: the same sums
    assert torch.equal(Fm.solve(rhs[:1]), Fm.solve(rhs[:3])[:1])       # vector-unit kernels
    assert torch.equal(Fm.solve(rhs[:16]), Fm.solve(rhs[:40])[:16])    # matrix-core kernel


def test_matrix_core_sweeps_graph_replay_bitwise():
    import paper_2411_18026_amd as fds
    curves = [sy.tripod(6400)]
    F = fds.Factor(curves, 2.0, 1.0, 1.0, 1.0, 1e-8, leaf=100)
    Fgr = fds.Factor(curves, 2.0, 1.0, 1.0, 1.0, 1e-8, leaf=100, solve_graph=True)
    rhs = F.rhs_plane([0] * 40, sy.plane_wave_angles(40))
    ref, ref1 = F.solve(rhs), F.solve(rhs[:1])
    for _ in range(3):
        x, x1 = Fgr.solve(rhs), Fgr.solve(rhs[:1])
        torch.cuda.synchronize()
        assert torch.equal(x, ref) and torch.equal(x1, ref1)
        F.solve(rhs[:3])   # eager work between the replays
