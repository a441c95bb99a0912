"""fds_solve_noalloc (the solve that allocates nothing, for callers that
cannot allocate) against fds_solve through the C ABI: two calls in a row on
the shared device scratch, the second with fewer right-hand sides (so the
scratch holds the first call's values beyond the second's), each bitwise
equal to fds_solve on the same input; sizes beyond the scratch and mixed
factors are refused."""
import ctypes

import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solve_noalloc(fds, F, rhs, out):
    L = fds.load()
    s = torch.cuda.current_stream().cuda_stream
    code = L.fds_solve_noalloc(F._h, rhs.shape[0], ctypes.c_void_p(rhs.data_ptr()), F.n_unknowns,
                               ctypes.c_void_p(out.data_ptr()), F.n_unknowns, ctypes.c_void_p(s))
    torch.cuda.synchronize()
    return code


@pytest.mark.parametrize("case", ["tripod6400", "ellipse131072"])
def test_noalloc_solve_matches_solve(case):
    import paper_2411_18026_amd as fds
    if case == "tripod6400":
        F = fds.Factor([sy.tripod(6400)], 2.0, 1.0, 1.0, 1.0, 1e-8, leaf=100)
        n1, n2 = 24, 5
    else:
        F = fds.Factor([sy.ellipse(131072, 1.0, 0.5)], 4.0, 2.0, 1.0, 1.0, 1e-8, leaf=64)
        n1, n2 = 4, 1
    print(f"case {case} nrhs {n1}, {n2}", flush=True)
    angles = sy.plane_wave_angles(n1)
    kinds = [k % 2 for k in range(n1)]
    rhs = F.rhs_plane(kinds, angles)
    for nrhs in (n1, n2):
        r = rhs[:nrhs].contiguous()
        ref = F.solve(r)
        out = torch.full_like(r, complex(float("nan"), float("nan")))
        assert _solve_noalloc(fds, F, r, out) == 0
        assert torch.equal(out, ref), (case, nrhs)


def test_noalloc_solve_refusals():
    import paper_2411_18026_amd as fds
    F = fds.Factor([sy.ellipse(131072, 1.0, 0.5)], 4.0, 2.0, 1.0, 1.0, 1e-8, leaf=64)
    rhs = F.rhs_plane([0] * 16, sy.plane_wave_angles(16))
    out = torch.empty_like(rhs)
    assert _solve_noalloc(fds, F, rhs, out) == 1          # 16 x ~19 MiB > 128 MiB
    assert b"MiB" in fds.load().fds_last_error()
    cfg = sy.config_small()
    Fm = fds.Factor(cfg["curves"], cfg["omega"], cfg["lam"], cfg["mu"], cfg["rho"], cfg["tol"], leaf=cfg["leaf"],
                    mixed=True)
    r = Fm.rhs_plane([0], [0.0])
    assert _solve_noalloc(fds, Fm, r, torch.empty_like(r)) == 1
