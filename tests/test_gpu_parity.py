"""GPU parity: each HIP step against the CPU oracle on the same seeded inputs,
through the C ABI.

Tolerances: the two sides evaluate the same integrals with the same
quadrature rules but independent code (special functions, summation
order), so entries agree to rounding (<= 1e-12 of the block's largest entry);
pivoted-QR decisions (pivots, ranks) must be identical; solutions agree to
1e-10 relative (same skeletons, rounding amplified by the conditioning of
the small dense blocks).
"""
import math

import numpy as np
import pytest

import synthetic as sy
from oracle import dense, fds as ofds, galerkin, special
from oracle.kernels import Material

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


def test_special_functions(fdsmod):
    from scipy import special as sp
    x = np.concatenate([np.logspace(-7, 2.7, 300), np.linspace(1.5, 20, 200)])
    out, outc = fdsmod.special_eval(torch.from_numpy(x), 0.5)
    out = out.cpu().numpy()
    outc = outc.cpu().numpy()
    ref = np.stack([sp.j0(x), sp.j1(x), sp.y0(x), sp.y1(x)], 1)
    err = np.abs(out - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() < 5e-15
    E, C = special.e_chi(x, 0.5)
    assert np.max(np.abs(outc[:, 0] - E) / np.abs(E)) < 1e-13
    assert np.max(np.abs(outc[:, 1] - C) / np.abs(C)) < 1e-13


GEOMS = {
    "circle64": [sy.circle(64)],
    "ellipse97": [sy.ellipse(97, 1.0, 0.5)],
    "two_cavities": [sy.ellipse(40, 0.6, 0.3, center=(-1.0, 0.2), angle=0.4), sy.circle(33, 0.5, center=(1.2, -0.3))],
}


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("omega", [1.0, 4.0, 14.5])
def test_dense_entries(fdsmod, name, omega):
    """At omega = 14.5 the 64-gon has k_T h = 1.4: the singular pairs take
    the longer rules and the regular pairs at least 6 points."""
    curves = GEOMS[name]
    mat = Material(2.0, 1.0, 1.0, omega)
    bnd = galerkin.Boundary(curves)
    A = galerkin.dense_matrix(bnd, mat)
    n = A.shape[0]
    G = fdsmod.entries(curves, omega, 2.0, 1.0, 1.0, np.arange(n), np.arange(n)).cpu().numpy()
    assert np.max(np.abs(G - A)) <= 1e-12 * np.max(np.abs(A))


def test_elements_too_long_for_the_wavenumber(fdsmod):
    """The quadrature rules hold up to k_T h = 5: a 16-gon at omega = 40
    (k_T h = 15.6) is refused with FDS_EGEOM."""
    with pytest.raises(fdsmod.FdsError) as e:
        fdsmod.Factor([sy.circle(16)], 40.0, 2.0, 1.0, 1.0, 1e-8, leaf=8)
    assert e.value.code == 2


def test_scattered_entries_and_alpha(fdsmod):
    curves = GEOMS["ellipse97"]
    rng = np.random.default_rng(7)
    rows = rng.choice(2 * 97, 37, replace=False)
    cols = rng.choice(2 * 97, 53, replace=False)
    for alpha in (None, 0.0, 0.3 - 0.7j):
        mat = Material(1.0, 1.0, 1.0, 2.5, alpha)
        ref = galerkin.dof_block(galerkin.Boundary(curves), rows, cols, mat)
        G = fdsmod.entries(curves, 2.5, 1.0, 1.0, 1.0, rows, cols, alpha=alpha).cpu().numpy()
        assert np.max(np.abs(G - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_cpqr_matches_oracle(fdsmod):
    rng = np.random.default_rng(3)
    mats = []
    for (m, n) in ((150, 40), (90, 64), (33, 70), (200, 7)):
        M = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * np.logspace(0, -12, n)[None, rng.permutation(n)]
        mats.append(M)
    # symmetric ties: two identical columns
    T = rng.standard_normal((50, 20)) + 0j
    T[:, 7] = T[:, 3]
    mats.append(T)
    res = fdsmod.cpqr_batched(mats, 1e-8)
    for M, (piv, k, R) in zip(mats, res):
        p_o, R_o = ofds.cpqr(M)
        k_o = ofds.id_rank(R_o, 1e-8)
        assert k == k_o
        assert np.array_equal(piv[:k], p_o[:k])
        assert np.allclose(np.abs(np.diag(R)[:k]), np.abs(np.diag(R_o)[:k]), rtol=1e-10)


def test_cpqr_register_variants_match_oracle(fdsmod):
    """Batches of small problems only (m <= 256, n <= 64) run the
    register-resident kernel, sized by the batch's largest problem: one
    batch within 128 x 32, one up to 256 x 64.  Edge cases: a zero matrix
    (rank 0), an exact rank-one matrix, fewer rows than columns."""
    rng = np.random.default_rng(21)
    for shapes in (((100, 30), (64, 32), (20, 25)), ((180, 50), (256, 64), (5, 64))):
        mats = []
        for (m, n) in shapes:
            M = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * \
                np.logspace(0, -12, n)[None, rng.permutation(n)]
            mats.append(M)
        mats.append(np.zeros((40, 10), dtype=np.complex128))
        u = rng.standard_normal(60) + 1j * rng.standard_normal(60)
        mats.append(np.outer(u, rng.standard_normal(12)))
        res = fdsmod.cpqr_batched(mats, 1e-8)
        for M, (piv, k, R) in zip(mats, res):
            p_o, R_o = ofds.cpqr(M)
            k_o = ofds.id_rank(R_o, 1e-8)
            assert k == k_o
            assert np.array_equal(piv[:k], p_o[:k])
            assert np.allclose(np.abs(np.diag(R)[:k]), np.abs(np.diag(R_o)[:k]), rtol=1e-10)


def test_interpolation_matrices_match_oracle(fdsmod):
    """W = [I, R11^{-1} R12] P^T of each ID against the oracle's, formed from
    the same pivots and R factor.  The first batch (ranks 1 to 64) runs the
    kernel that stages R11 in LDS, the second (ranks above 64) the
    column-per-thread loop; up to 200 columns span several 64-column chunks
    with ragged tails, and rank = n leaves no R12."""
    rng = np.random.default_rng(31)
    batches = ((((90, 60), 37), ((70, 64), 64), ((200, 150), 63), ((130, 200), 1), ((33, 5), 4),
                ((100, 130), 64)),
               (((300, 120), 90), ((260, 90), 65)))
    for batch in batches:
        mats = [rng.standard_normal(sh) + 1j * rng.standard_normal(sh) for sh, _ in batch]
        kmax = [k for _, k in batch]
        res = fdsmod.cpqr_batched(mats, 1e-8, kmax=kmax, stop_at_tol=False, interp=True)
        for M, kk, (piv, k, R, W) in zip(mats, kmax, res):
            n = M.shape[1]
            assert k == kk and W.shape == (k, n)
            assert np.array_equal(W[:, piv[:k]], np.eye(k))
            Wo = ofds.id_matrix(piv, R, k, n)
            assert np.max(np.abs(W - Wo)) <= 1e-10 * max(1.0, np.max(np.abs(Wo))), (M.shape, k)


@pytest.mark.parametrize("name", ["circle64", "two_cavities"])
def test_load_vectors(fdsmod, name):
    curves = GEOMS[name]
    F = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-8, leaf=16)
    kinds = [0, 1, 0, 1]
    angles = [0.0, 0.3, 2.0, 4.4]
    got = F.rhs_plane(kinds, angles).cpu().numpy()
    mat = Material(2.0, 1.0, 1.0, 3.0)
    bnd = galerkin.Boundary(curves)
    for k in range(4):
        ref = galerkin.load_vector(bnd, kinds[k], angles[k], mat)
        assert np.max(np.abs(got[k] - ref)) <= 1e-13 * np.max(np.abs(ref))


def _oracle_problem(curves, omega, kinds, angles, lam=2.0):
    X, A, Fm = dense.dense_solve(curves, lam, 1.0, 1.0, omega, kinds, angles, return_matrix=True)
    return X, A, Fm


def test_small_validation_case(fdsmod):
    cfg = sy.config_small()
    curves = cfg["curves"]
    X, A, Fm = _oracle_problem(curves, cfg["omega"], [0, 1], [0.0, 1.0])
    F = fdsmod.Factor(curves, cfg["omega"], cfg["lam"], cfg["mu"], cfg["rho"], cfg["tol"], leaf=cfg["leaf"])
    rhs = torch.from_numpy(np.ascontiguousarray(Fm.T)).to("cuda")
    Y = F.solve(rhs).cpu().numpy().T
    err = np.linalg.norm(Y - X) / np.linalg.norm(X)
    assert err < 1e-9
    S = ofds.FDS(curves, cfg["lam"], cfg["mu"], cfg["rho"], cfg["omega"], cfg["tol"], leaf=cfg["leaf"])
    Yo = S.solve(Fm)
    assert np.linalg.norm(Y - Yo) / np.linalg.norm(Yo) < 1e-10
    # identical ranks and skeletons as the oracle
    rk = F.ranks()
    for i, c in S.cells.items():
        if c.ranks:
            assert tuple(rk[i]) == (c.ranks[0][0], c.ranks[0][1], c.ranks[1][0], c.ranks[1][1])
            r, cc = F.skeleton(i)
            assert np.array_equal(r, c.rskel) and np.array_equal(cc, c.cskel)


@pytest.mark.parametrize("case", ["ragged", "multi", "deep_root0", "cavities4"])
def test_fds_against_oracle(fdsmod, case):
    if case == "ragged":
        curves, leaf, l0, omega = [sy.ellipse(300, 1.0, 0.5)], 32, 1, 3.0
    elif case == "multi":
        curves, leaf, l0, omega = GEOMS["two_cavities"], 16, 1, 2.0
    elif case == "cavities4":  # tree over several curves (Morton order, whole-curve groups)
        curves, leaf, l0, omega = sy.multi_cavity(21, 4, 220, half_width=2.5), 16, 1, 2.0
    else:
        curves, leaf, l0, omega = [sy.tripod(256)], 16, 0, 2.0
    kinds, angles = [0, 1, 0], [0.0, 0.9, 3.0]
    X, A, Fm = _oracle_problem(curves, omega, kinds, angles)
    F = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, 1e-9, leaf=leaf, root_level=l0)
    rhs = torch.from_numpy(np.ascontiguousarray(Fm.T)).to("cuda")
    Y = F.solve(rhs).cpu().numpy().T
    S = ofds.FDS(curves, 2.0, 1.0, 1.0, omega, 1e-9, leaf=leaf, root_level=l0)
    Yo = S.solve(Fm)
    assert np.linalg.norm(Y - Yo) / np.linalg.norm(Yo) < 1e-10
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) < 1e-6
    # the GPU load vectors reproduce the oracle's
    G = F.rhs_plane(kinds, angles).cpu().numpy().T
    assert np.max(np.abs(G - Fm)) <= 1e-13 * np.max(np.abs(Fm))


def test_graph_solve_replays_match_eager(fdsmod):
    """Solve sweeps captured as a hipGraph: every replay (with eager work in
    between) reproduces the eager solve."""
    curves = [sy.ellipse(300, 1.0, 0.5)]
    Fe = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    Fg = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32, solve_graph=True)
    rhs = Fe.rhs_plane([0, 1, 0], [0.0, 0.9, 3.0])
    rhs2 = (rhs * (0.5 - 2.0j)).contiguous()
    xe = Fe.solve(rhs)
    xe2 = Fe.solve(rhs2)
    for k in range(4):
        xg = Fg.solve(rhs)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), k
        _ = Fe.solve(rhs2)               # eager work between replays
        xg2 = Fg.solve(rhs2)
        assert torch.equal(xg2, xe2), k
    x1 = Fg.solve(rhs[1])                # another nrhs: a second graph
    assert torch.equal(x1, Fe.solve(rhs[1]))


def test_device_block_cache_reuse_and_release(fdsmod):
    """Device buffers come from the library's block cache: a destroyed
    factor's blocks stay cached and are reused by the next factor (which
    gives bitwise the same solution), the cache empties on release, and a
    factor built after the release (fresh allocations) again gives the same
    solution."""
    import gc
    curves = [sy.ellipse(400, 1.0, 0.5)]
    F1 = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    rhs = F1.rhs_plane([0, 1], [0.2, 1.1])
    x1 = F1.solve(rhs)
    torch.cuda.synchronize()
    del F1
    gc.collect()
    cached = fdsmod.cached_bytes()
    assert cached > 0
    F2 = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    assert fdsmod.cached_bytes() < cached
    assert torch.equal(F2.solve(rhs), x1)
    del F2
    gc.collect()
    fdsmod.release_cache()
    assert fdsmod.cached_bytes() == 0
    F3 = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    assert torch.equal(F3.solve(rhs), x1)


def test_cpqr_tall_variant_matches_oracle(fdsmod):
    """Matrices beyond the LDS-staged sizes (more than 2048 rows or 1024
    columns) go through the variant that reads the reflector in place."""
    rng = np.random.default_rng(8)
    A = (rng.standard_normal((2500, 70)) + 1j * rng.standard_normal((2500, 70))) * np.logspace(0, -12, 70)[None, :]
    B = rng.standard_normal((300, 1100)) + 1j * rng.standard_normal((300, 1100))
    resA = fdsmod.cpqr_batched([A], 1e-8)
    p_o, R_o = ofds.cpqr(A)
    k_o = ofds.id_rank(R_o, 1e-8)
    piv, k, R = resA[0]
    assert k == k_o and np.array_equal(piv[:k], p_o[:k])
    assert np.allclose(np.abs(np.diag(R)[:k]), np.abs(np.diag(R_o)[:k]), rtol=1e-10)
    resB = fdsmod.cpqr_batched([B], 1e-8, kmax=[25], stop_at_tol=False)
    p_o, R_o = ofds.cpqr(B, kmax=25)
    piv, k, R = resB[0]
    assert k == 25 and np.array_equal(piv[:25], p_o[:25])
    assert np.allclose(np.abs(np.diag(R)[:25]), np.abs(np.diag(R_o)[:25]), rtol=1e-10)


def test_lu_batched_is_a_partial_pivoting_lu(fdsmod):
    """P A = L U to rounding with |L| <= 1 and every pivot the column's
    largest modulus, for sizes on both sides of the one-workgroup limit
    (384 rows; 128 in batches of at most 8): the one-workgroup kernel (7),
    and the multi-workgroup blocked form with 32-column panels in LDS (130,
    300), 16-column panels in LDS (500) and panels in memory (900, 1300)."""
    rng = np.random.default_rng(12)
    batches = [[7, 130, 300], [500], [900, 1300]]
    mats, res = [], []
    for sizes in batches:
        ms = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for n in sizes]
        mats += ms
        res += fdsmod.lu_batched(ms)
    for A, (LU, piv, info) in zip(mats, res):
        n = A.shape[0]
        assert info == 0
        L = np.tril(LU, -1) + np.eye(n)
        U = np.triu(LU)
        PA = A.copy()
        for k in range(n):
            assert k <= piv[k] < n
            PA[[k, piv[k]]] = PA[[piv[k], k]]
        assert np.linalg.norm(PA - L @ U) <= 1e-13 * n * np.linalg.norm(A)
        assert np.abs(L).max() <= 1.0 + 1e-12
    # a zero column is reported at its step, by each form: panels in memory
    # (900), in LDS (300), and the one-workgroup kernel (a batch of nine 100s)
    Z = rng.standard_normal((900, 900)) + 0j
    Z[:, 5] = 0.0
    assert fdsmod.lu_batched([Z])[0][2] == 6
    Z = rng.standard_normal((300, 300)) + 0j
    Z[:, 40] = 0.0
    assert fdsmod.lu_batched([Z])[0][2] == 41
    Zs = [rng.standard_normal((100, 100)) + 0j for _ in range(9)]
    Zs[4][:, 17] = 0.0
    assert [r[2] for r in fdsmod.lu_batched(Zs)] == [0, 0, 0, 0, 18, 0, 0, 0, 0]


def test_autotuned_shapes_give_identical_solutions(fdsmod):
    """The autotuner only repartitions the sweeps' outputs: solutions with and
    without it are bitwise equal for every nrhs class."""
    curves = [sy.ellipse(1200, 1.0, 0.5)]
    Ft = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    Ff = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32, autotune=False)
    st = Ft.stats()
    assert all(c >= 1 for c in st["tune_chunk"]) and all(c in (16, 64) for c in st["tune_gemm_cols"])
    assert Ff.stats()["tune_seconds"] == 0.0
    for nrhs in (1, 5, 20, 40):
        rhs = Ft.rhs_plane([k % 2 for k in range(nrhs)], np.linspace(0.0, 6.0, nrhs))
        assert torch.equal(Ft.solve(rhs), Ff.solve(rhs)), nrhs
