"""GPU checks of the learned form: randomized ID and judge, the predictor's
forward / backward / Adam kernels, and the learned factorisation.

* Randomized IDs: same pivots, ranks and reveal decisions as the oracle on
  the same sketches (the two sides draw them from their own SplitMix64
  implementations); judge ratios to rounding.
* MLP: FP32 forward, loss and gradient against the FP64 oracle; the bf16
  forward within bf16 rounding; initialisation and Adam training against the
  oracle's steps on the same minibatches.
* Learned factor: a predictor that under-sizes every sketch sends every cell
  back to the pivoted QR (identical factor to the adaptive form); a
  generous one gets its IDs from the sketches, and every accepted skeleton
  admits an interpolation within the tolerance (checked on the oracle's
  interaction matrices by least squares), with the solution as accurate as
  the adaptive form's against the dense oracle.
"""
import numpy as np
import pytest

import synthetic as sy
from oracle import dense, fds as ofds, galerkin, learned as ol
from oracle.kernels import Material

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdsmod():
    import paper_2411_18026_amd as m
    m.load()
    assert torch.cuda.is_available()
    return m


def _gapped(m, n, k, rng):
    """m x n matrix with k singular values in [1e-6, 1] and the rest <= 1e-12:
    its rank at tolerance 1e-8 is k with a wide margin."""
    U, _ = np.linalg.qr(rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    sv = np.concatenate([np.logspace(0, -6, k), np.logspace(-12, -15, n - k)])
    return (U[:, :n] * sv) @ V.conj().T


def test_randomized_id_matches_oracle(fdsmod):
    rng = np.random.default_rng(11)
    cases = [(200, 64, 20, 30), (350, 100, 37, 45), (150, 40, 12, 40), (300, 128, 50, 40), (97, 33, 5, 9)]
    mats = [_gapped(m, n, k, rng) for m, n, k, _ in cases]
    sizes = [s for *_, s in cases]
    gids = [3, 17, 4096, 5, 123456]
    res = fdsmod.rid_batched(mats, sizes, 1e-8, seed=2024, gids=gids)
    for M, s, g, (piv, k, rev, ratio), case in zip(mats, sizes, gids, res, cases):
        o = ol.randomized_id(M, s, 1e-8, 2024, g)
        assert k == o["rank"], case
        assert rev == o["revealed"], case
        assert np.array_equal(piv[:k], o["piv"][:k]), case
        assert abs(ratio - o["ratio"]) <= 1e-6 * o["ratio"] + 1e-13, case
    # the under-sized sketch (50 > 40 rows) is not revealed; the others pass the judge
    assert not res[3][2] and all(r[2] for i, r in enumerate(res) if i != 3)
    assert all(r[3] <= 1e-8 for i, r in enumerate(res) if i != 3)


def test_large_randomized_id_matches_oracle(fdsmod):
    """Sketches beyond the LDS kernel (more than 64 rows or 128 columns) go
    through Omega + GEMM and the GEMM residual judge."""
    rng = np.random.default_rng(13)
    cases = [(700, 200, 90, 110), (900, 150, 60, 72), (400, 300, 140, 120)]
    mats = [_gapped(m, n, k, rng) for m, n, k, _ in cases]
    sizes = [s for *_, s in cases]
    res = fdsmod.rid_batched(mats, sizes, 1e-8, seed=77, gids=[9, 10, 11])
    for M, s, g, (piv, k, rev, ratio), case in zip(mats, sizes, [9, 10, 11], res, cases):
        o = ol.randomized_id(M, s, 1e-8, 77, g)
        assert k == o["rank"] and rev == o["revealed"], case
        assert np.array_equal(piv[:k], o["piv"][:k]), case
        assert abs(ratio - o["ratio"]) <= 1e-6 * o["ratio"] + 1e-13, case
    assert res[0][2] and res[1][2] and not res[2][2]


def _rand_blob(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    b = ol.init_blob(seed, rng.standard_normal(6), rng.uniform(0.5, 2, 6), 24.0)
    b[:ol.N_PARAM] += scale * rng.standard_normal(ol.N_PARAM) * 0.1
    return b.astype(np.float32)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 6)).astype(np.float32) * 2
    y = (10 + 5 * X[:, 0] + X[:, 2] ** 2).astype(np.float32)
    return X, y


def test_mlp_forward_matches_oracle(fdsmod):
    blob = _rand_blob(1)
    X, _ = _data(3000, 2)
    ref = ol.predict(blob.astype(np.float64), X.astype(np.float64))
    got = fdsmod.mlp_forward(blob, X).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    got16 = fdsmod.mlp_forward(blob, X, bf16=True).cpu().numpy()
    err16 = np.max(np.abs(got16 - ref)) / np.max(np.abs(ref))
    assert 1e-5 < err16 < 3e-2   # bf16 rounding: visible, and bounded


def test_mlp_loss_grad_matches_oracle(fdsmod):
    blob = _rand_blob(3)
    X, y = _data(1500, 4)
    loss, g = fdsmod.mlp_loss_grad(blob, X, y)
    lo, go = ol.loss_grad(blob.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * lo
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_mlp_init_and_training_match_oracle(fdsmod):
    X, y = _data(700, 5)
    blob = fdsmod.mlp_init(X, y, seed=99)
    mu, sd, ys = ol.standardise(X.astype(np.float64), y.astype(np.float64))
    ref = ol.init_blob(99, mu, sd, ys)
    assert np.max(np.abs(blob - ref)) <= 1e-6 * np.max(np.abs(ref))
    steps, batch, lr = 40, 64, 3e-3
    trained, hist = fdsmod.mlp_train(blob, X, y, steps, batch, lr, seed=7)
    b = ref.copy()
    m = np.zeros(ol.N_PARAM)
    v = np.zeros(ol.N_PARAM)
    hist_o = []
    for t in range(1, steps + 1):
        idx = ol.minibatch(7, t, batch, len(y))
        l, g = ol.loss_grad(b, X[idx].astype(np.float64), y[idx].astype(np.float64))
        hist_o.append(l)
        b, m, v = ol.adam_step(b, g, m, v, t, lr)
    hist_o = np.array(hist_o)
    assert np.max(np.abs(hist - hist_o) / hist_o) < 1e-2
    assert hist[-1] < 0.5 * hist[0]
    assert np.array_equal(trained[ol.N_PARAM:], blob[ol.N_PARAM:])


def _const_blob(value, y_scale=64.0):
    """A predictor whose output is ``value`` for every cell (wide sigma: it
    never abstains)."""
    b = np.zeros(ol.N_BLOB, np.float32)
    b[ol.N_PARAM - 1] = value / y_scale      # b4
    b[ol.N_PARAM + 6:ol.N_PARAM + 12] = 1e3  # sigma
    b[-1] = y_scale
    return b


def test_undersized_sketches_fall_back_to_the_adaptive_factor(fdsmod):
    curves = [sy.ellipse(300, 1.0, 0.5)]
    Fa = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    Fl = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32, predictor=_const_blob(0.0), oversample=2)
    log = Fl.rank_log()
    assert np.all(log["k_pred"] == 0)
    assert np.all(log["fallback"] == 1)            # every rank exceeds the 2-row sketch
    st = Fl.stats()
    assert st["cells_fallback_rank"] == st["cells_compressed"] and st["cells_sketched"] == 0
    assert np.array_equal(Fa.ranks(), Fl.ranks())
    rhs = Fa.rhs_plane([0, 1], [0.3, 2.0])
    assert torch.equal(Fa.solve(rhs), Fl.solve(rhs))


def test_predictor_abstains_outside_its_training_range(fdsmod):
    curves = [sy.ellipse(300, 1.0, 0.5)]
    b = _const_blob(30.0)
    b[ol.N_PARAM + 6:ol.N_PARAM + 12] = 1e-3   # every input far from mu in sigma units
    Fl = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32, predictor=b)
    log = Fl.rank_log()
    assert np.all(log["k_pred"] == -1) and np.all(log["fallback"] == 3)
    Fa = fdsmod.Factor(curves, 3.0, 2.0, 1.0, 1.0, 1e-9, leaf=32)
    assert np.array_equal(Fa.ranks(), Fl.ranks())


def test_learned_factor_accepts_sketches_and_stays_accurate(fdsmod):
    curves = [sy.ellipse(1024, 1.0, 0.5)]
    omega, tol, leaf = 3.0, 1e-9, 64
    Fa = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, tol, leaf=leaf)
    Fl = fdsmod.Factor(curves, omega, 2.0, 1.0, 1.0, tol, leaf=leaf, predictor=_const_blob(36.0))
    st = Fl.stats()
    log = Fl.rank_log()
    assert np.all(log["k_pred"] == 36)
    assert st["cells_sketched"] >= 0.5 * st["cells_compressed"]
    assert set(np.unique(log["fallback"])) <= {0, 1, 2}
    # solutions against the dense oracle: as accurate as the adaptive form
    kinds, angles = [0, 1], [0.0, 1.3]
    X, A, Fm = dense.dense_solve(curves, 2.0, 1.0, 1.0, omega, kinds, angles, return_matrix=True)
    rhs = torch.from_numpy(np.ascontiguousarray(Fm.T)).to("cuda")
    ea = np.linalg.norm(Fa.solve(rhs).cpu().numpy().T - X) / np.linalg.norm(X)
    el = np.linalg.norm(Fl.solve(rhs).cpu().numpy().T - X) / np.linalg.norm(X)
    print(f"error vs dense: learned {el:.3e}, adaptive {ea:.3e}", flush=True)
    assert el <= 2 * ea + 1e-12, (el, ea)
    # every accepted leaf skeleton admits an interpolation within tol
    S = ofds.FDS(curves, 2.0, 1.0, 1.0, omega, tol, leaf=leaf)
    mat = Material(2.0, 1.0, 1.0, omega)
    bnd = galerkin.Boundary(curves)
    leaves = ofds.level_cells(S.cells, S.L)
    acc = [i for i in range(len(log["cell"])) if log["level"][i] == S.L and log["fallback"][i] == 0]
    assert acc
    for i in acc[:: max(1, len(acc) // 6)]:
        c = next(cc for cc in leaves if cc.index == log["cell"][i])
        MV, MU = ofds.interaction_matrices(bnd, mat, c, [o for o in leaves if o is not c])
        rs, cs = Fl.skeleton(int(c.index))
        for q in (0, 1):
            cidx = np.nonzero(c.cols % 2 == q)[0]
            J = [int(np.nonzero(c.cols[cidx] == d)[0][0]) for d in cs if d % 2 == q]
            assert ol.best_interpolation_ratio(MV[:, cidx], J) <= tol * 1.0000001
            ridx = np.nonzero(c.rows % 2 == q)[0]
            Jr = [int(np.nonzero(c.rows[ridx] == d)[0][0]) for d in rs if d % 2 == q]
            assert ol.best_interpolation_ratio(MU[ridx, :].T, Jr) <= tol * 1.0000001


def test_rank_log_features_match_oracle(fdsmod):
    cfg = sy.config_small()
    curves = cfg["curves"]
    F = fdsmod.Factor(curves, cfg["omega"], cfg["lam"], cfg["mu"], cfg["rho"], cfg["tol"], leaf=cfg["leaf"])
    S = ofds.FDS(curves, cfg["lam"], cfg["mu"], cfg["rho"], cfg["omega"], cfg["tol"], leaf=cfg["leaf"])
    log = F.rank_log()
    mat = Material(cfg["lam"], cfg["mu"], cfg["rho"], cfg["omega"])
    assert len(log["cell"]) == sum(1 for c in S.cells.values() if c.ranks)
    for i, cell in enumerate(log["cell"]):
        c = S.cells[int(cell)]
        f = ol.cell_features(c, mat, cfg["tol"], 64, c.n_near[0])
        assert np.allclose(log["feat"][i], f, rtol=1e-6), (cell, log["feat"][i], f)
        assert tuple(log["rank"][i]) == (c.ranks[0][0], c.ranks[0][1], c.ranks[1][0], c.ranks[1][1])
    assert np.all(log["k_pred"] == -1) and np.all(log["fallback"] == 0)


def test_trained_predictor_against_the_adaptive_method(fdsmod):
    """The predictor trained by the library's own kernels on ranks the solver
    recorded (12 geometries of the training family at 4096 nodes), against
    the method without it (every ID by the pivoted QR of its proxy-plus-near
    matrix) on three held-out geometries of that family at tol 1e-8:

    * what it gains: most cells take their ID from a sketch of
      ceil(k_pred) + 10 rows instead of the full interaction matrix, and the
      pivoted QR then works on under two thirds of the rows the adaptive
      form factors (counted from the rank log, fallbacks charged with both
      the sketch and the full matrix; measured 0.55, 70 % of the cells
      from sketches);
    * what it keeps: every skeleton admits its interpolation (judge), the
      solutions differ from the adaptive ones by the compression error only
      (within 1e3 tol), and few ranks are under-predicted;
    * what it costs: both factor times and ID-stage times are measured (best
      of three) and printed.  On this GPU the register-resident pivoted QR
      reads each interaction matrix once, so a sketch (one more pass over
      the matrix, then the judge's pass) does not shorten the ID stage: the
      learned form is asserted to stay within 1.6x of the adaptive ID stage
      and 1.3x of its factor time (measured 1.35x and 1.14x), not to beat
      them."""
    import time
    from paper_2411_18026_amd import predictor as pr
    train = [sy.training_geometry(i, nodes=4096) for i in range(12)]
    held = [sy.training_geometry(100 + i, nodes=4096) for i in range(3)]
    x, y = pr.collect(train)
    blob0 = fdsmod.mlp_init(x, y, seed=3)
    blob, hist = fdsmod.mlp_train(blob0, x, y, 1500, 256, 2e-3, seed=4)
    assert hist[-1] < 0.05 * hist[0]

    def timed(curves, k_t, **kw):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F = fdsmod.Factor(curves, k_t, 2.0, 1.0, 1.0, 1e-8, leaf=64, **kw)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0, F.stats()["id_seconds"])
            best = t if best is None else (min(best[0], t[0]), min(best[1], t[1]))
        return F, best

    cells = accepted = 0
    rows_adaptive = rows_learned = 0.0
    t_a = t_l = id_a = id_l = 0.0
    under = []
    for curves, k_t in held:
        xh, yh = pr.rank_log_dataset(curves, k_t, 2.0, 1.0, 1.0, 1e-8)
        under.append(pr.evaluate(blob, xh, yh, oversample=10)["under"])
        Fa, (ta, ia) = timed(curves, k_t)
        Fl, (tl, il) = timed(curves, k_t, predictor=blob)
        t_a, t_l, id_a, id_l = t_a + ta, t_l + tl, id_a + ia, id_l + il
        log = Fl.rank_log()
        m = np.exp(log["feat"][:, 4])                   # rows of the proxy-plus-near matrix
        acc = log["fallback"] == 0
        s_rows = np.ceil(np.maximum(log["k_pred"], 0)) + 10
        cells += len(log["cell"])
        accepted += int(acc.sum())
        rows_adaptive += float(m.sum())
        rows_learned += float(np.where(acc, s_rows, m + s_rows * (log["k_pred"] >= 0)).sum())
        rhs = Fa.rhs_plane([0, 1], [0.0, 1.0])
        xa, xl = Fa.solve(rhs), Fl.solve(rhs)
        d = float((torch.linalg.norm(xa - xl, dim=1) / torch.linalg.norm(xa, dim=1)).max())
        assert d < 1e3 * 1e-8, d
        Fa.close()
        Fl.close()
    print(f"held-out: {accepted}/{cells} cells from sketches, QR rows {rows_learned / rows_adaptive:.3f} of the "
          f"adaptive form's; factor {t_l:.3f} s learned vs {t_a:.3f} s adaptive, ID stage {id_l:.3f} s vs "
          f"{id_a:.3f} s; under-predicted {np.mean(under):.3f}", flush=True)
    assert accepted >= 0.6 * cells
    assert rows_learned < 0.65 * rows_adaptive
    assert np.mean(under) < 0.25
    assert id_l < 1.6 * id_a and t_l < 1.3 * t_a
