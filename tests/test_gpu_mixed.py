"""GPU checks of the mixed-precision form: FP32 elimination and sweeps with
iterative refinement against the FP64 compressed operator A_c.

* The IDs run in FP64 in both forms, so the mixed factor has the plain
  factor's ranks and skeletons: it compresses to the same A_c.
* fds_apply (the FP64 product with A_c in nested form) inverts the oracle's
  FDS solve: A_c (A_c^{-1} f) = f to rounding, with A_c^{-1} f taken from the
  CPU oracle (independent code).
* The refined solutions match the plain FP64 solutions per right-hand side:
  <= 1e-6 relative at the default stop rule (residual <= 1e-8, last
  correction <= 1e-6), <= 1e-9 when
  refined to ir_rtol = 1e-12.
* The step limit is honoured: ir_max_iter = 0 returns FDS_ENOCONV with the
  unrefined FP32 solution written.
"""
import numpy as np
import pytest

import synthetic as sy
from oracle import dense, fds as ofds

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


CASES = {
    "ragged": ([sy.ellipse(300, 1.0, 0.5)], 32, 1, 3.0),
    "multi": ([sy.ellipse(40, 0.6, 0.3, center=(-1.0, 0.2), angle=0.4), sy.circle(33, 0.5, center=(1.2, -0.3))],
              16, 1, 2.0),
    "deep_root0": ([sy.tripod(256)], 16, 0, 2.0),
}


def _rel_cols(a, b):
    return (torch.linalg.norm(a - b, dim=1) / torch.linalg.norm(b, dim=1)).max().item()


@pytest.mark.parametrize("case", list(CASES))
def test_mixed_against_plain_and_oracle(fdsmod, case):
    curves, leaf, l0, omega = CASES[case]
    kinds, angles = [0, 1, 0], [0.0, 0.9, 3.0]
    Fp = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, root_level=l0)
    Fm = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, root_level=l0, mixed=True)
    assert np.array_equal(Fp.ranks(), Fm.ranks())
    rhs = Fp.rhs_plane(kinds, angles)
    xp = Fp.solve(rhs)
    xm = Fm.solve(rhs)
    st = Fm.stats()
    assert st["precision"] == fdsmod.PREC_MIXED
    assert st["ir_residual"] <= 1e-8 and st["ir_correction"] <= 1e-6 and st["ir_iterations"] >= 1
    assert _rel_cols(xm, xp) < 1e-6
    # A_c applied to the oracle's FDS solution gives back the right-hand side
    X, A, Fmat = dense.dense_solve(curves, 2.0, 1.0, 1.0, omega, kinds, angles, return_matrix=True)
    S = ofds.FDS(curves, 2.0, 1.0, 1.0, omega, 1e-9, leaf=leaf, root_level=l0)
    Yo = S.solve(Fmat)
    y = Fm.apply(torch.from_numpy(np.ascontiguousarray(Yo.T)).to("cuda")).cpu().numpy().T
    assert np.linalg.norm(y - Fmat) / np.linalg.norm(Fmat) < 1e-10
    # A_c is close to the dense Galerkin matrix (compression at tol 1e-9)
    v = np.random.default_rng(5).standard_normal((A.shape[0], 2)) + 0j
    yv = Fm.apply(torch.from_numpy(np.ascontiguousarray(v.T)).to("cuda")).cpu().numpy().T
    assert np.linalg.norm(yv - A @ v) / np.linalg.norm(A @ v) < 1e-6
    # refined to a tight residual the mixed form reproduces the plain FP64 solution
    Ft = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, root_level=l0, mixed=True, ir_rtol=1e-12)
    xt = Ft.solve(rhs)
    assert _rel_cols(xt, xp) < 1e-9
    assert np.linalg.norm(xt.cpu().numpy().T - Yo) / np.linalg.norm(Yo) < 1e-9


def test_mixed_step_limit(fdsmod):
    curves, leaf, l0, omega = CASES["ragged"]
    Fp = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf)
    Fm = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, mixed=True, ir_max_iter=0)
    rhs = Fp.rhs_plane([0, 1], [0.2, 1.1])
    xp = Fp.solve(rhs)
    with pytest.raises(fdsmod.NotConverged) as e:
        Fm.solve(rhs)
    st = Fm.stats()
    assert st["ir_iterations"] == 0 and st["ir_residual"] > 1e-8
    # the unrefined FP32 solution is written: FP32-accurate, not FP64-accurate
    err = _rel_cols(e.value.x, xp)
    assert 1e-12 < err < 1e-3


def test_plain_factor_has_no_apply(fdsmod):
    curves, leaf, l0, omega = CASES["ragged"]
    Fp = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf)
    with pytest.raises(fdsmod.FdsError):
        Fp.apply(torch.zeros(Fp.n_unknowns, dtype=torch.complex128, device="cuda"))


def test_mixed_graph_replays_match_eager(fdsmod):
    """Mixed solve with its FP32 sweeps and A_c products captured as hipGraphs:
    every replay, with eager work in between, reproduces the eager solve."""
    curves, leaf, l0, omega = CASES["ragged"]
    Fe = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, mixed=True)
    Fg = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, mixed=True, solve_graph=True)
    rhs = Fe.rhs_plane([0, 1, 0], [0.0, 0.9, 3.0])
    rhs2 = (rhs * (0.5 - 2.0j)).contiguous()
    xe = Fe.solve(rhs)
    xe2 = Fe.solve(rhs2)
    for k in range(3):
        xg = Fg.solve(rhs)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), k
        _ = Fe.solve(rhs2)
        assert torch.equal(Fg.solve(rhs2), xe2), k
