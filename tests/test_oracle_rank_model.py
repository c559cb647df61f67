"""Pins of the oracle's learned-rank pieces (no GPU): the counter-based Gaussian
generator, the rank MLP (forward, gradient, Adam), the box features and the
sketched row ID.  Each pin is a known answer, a closed form, a special case or
a property of the mathematics, not the oracle's own formula retyped."""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

import workloads as W
from oracle import h2ulv_ref as O
from oracle import rank_model as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --- generator ---------------------------------------------------------------
def test_splitmix64_known_answers():
    g = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    assert R.splitmix64_at(0, 0) == int(g["seed0_first"], 16)
    want = [int(x) for x in g["seed1234567_first5"]]
    assert [R.splitmix64_at(1234567, c) for c in range(5)] == want
    # vectorised positions agree with the scalar reads
    v = R.splitmix64_at(1234567, np.arange(5, dtype=np.uint64))
    assert [int(x) for x in v] == want


def test_gaussian_deviates_are_standard_normal():
    z = R.gaussian(R.box_key(11, 3, 5), np.arange(200000, dtype=np.uint64))
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.06
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # distinct boxes give unrelated streams
    z2 = R.gaussian(R.box_key(11, 3, 6), np.arange(200000, dtype=np.uint64))
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01


def test_point_rows_layout_and_independence():
    """Entry (r, c) of a point's sketch rows is deviate c N + p of its stream; the
    rows of a point do not depend on which other points are asked for, and the
    far and fill streams differ."""
    pts = np.array([7, 3, 11])
    G = R.point_rows(4, 2, R.STREAM_FILL, pts, 20, 5)
    key = R.box_key(4, 2, R.STREAM_BASE + R.STREAM_FILL)
    for r, p in enumerate(pts):
        for c in (0, 3, 4):
            assert G[r, c] == R.gaussian(key, np.array([c * 20 + p], dtype=np.uint64))[0]
    G2 = R.point_rows(4, 2, R.STREAM_FILL, np.array([11, 7]), 20, 5)
    assert np.array_equal(G2, G[[2, 0]])
    F = R.point_rows(4, 2, R.STREAM_FAR, pts, 20, 5)
    assert not np.allclose(F, G)


# --- MLP -----------------------------------------------------------------------
def test_forward_identity_network_sums_relu_of_inputs():
    """W1 copies the 16 inputs, W2 = W3 = I, w4 sums the first 16 units: the
    network computes sum_i max(x_i, 0) + b4."""
    parts = {k: np.zeros(s) for k, s in R.SHAPES}
    parts["W1"][:16, :16] = np.eye(16)
    parts["W2"] = np.eye(64)
    parts["W3"] = np.eye(64)
    parts["w4"][:16] = 1.0
    parts["b4"][0] = 0.25
    th = R.pack(parts)
    X = np.random.default_rng(0).standard_normal((40, 16))
    y, _ = R.forward(th, X)
    assert np.allclose(y, np.maximum(X, 0).sum(axis=1) + 0.25, rtol=0, atol=1e-13)
    # a negative bias on the first layer switches those units off
    parts["b1"][:16] = -100.0
    y2, _ = R.forward(R.pack(parts), X)
    assert np.allclose(y2, 0.25)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    th = R.init_weights(5) + 0.01 * rng.standard_normal(R.NPARAM)
    X = rng.standard_normal((50, 16))
    t = rng.standard_normal(50)
    _, g = R.loss_and_grad(th, X, t)
    idx = np.concatenate([rng.choice(R.NPARAM, 300, replace=False), np.arange(R.NPARAM - 65, R.NPARAM)])
    h = 1e-6
    for j in idx:
        e = np.zeros(R.NPARAM)
        e[j] = h
        fd = (R.loss_and_grad(th + e, X, t)[0] - R.loss_and_grad(th - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_adam_first_step_closed_form():
    """With zero moments, the bias-corrected first step is lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    th = rng.standard_normal(R.NPARAM)
    g = rng.standard_normal(R.NPARAM) * 10.0 ** rng.uniform(-6, 2, R.NPARAM)
    th1, m, v = R.adam_step(th, np.zeros_like(th), np.zeros_like(th), g, 1, 1e-3)
    assert np.allclose(th1, th - 1e-3 * g / (np.abs(g) + R.ADAM_EPS), rtol=1e-12, atol=1e-15)


def test_training_fits_a_linear_target():
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (400, 16))
    t = X @ rng.uniform(-1, 1, 16) + 2.0
    th, hist = R.train(R.init_weights(7), X, t, 600, 3e-3)
    assert hist[-1] < 1e-2 * hist[0] and hist[-1] < 1e-2


def test_predicted_rank_and_sketch_size():
    assert R.predicted_rank(math.log2(1 + 40)) == 40
    assert R.predicted_rank(-3.0) == 0
    assert R.sketch_size(40, 8) == 58
    assert R.sketch_size(0, 8) == 8


# --- features --------------------------------------------------------------
def test_features_closed_form_on_a_segment():
    """Evenly spaced points on [0, a] along x: population variance
    a^2 (n + 1) / (12 (n - 1)), radius a / 2, so feature 9 is its root over a/2."""
    n, a = 256, 3.0
    X = np.zeros((n, 3))
    X[:, 0] = np.linspace(0, a, n)
    p = O.Params(leaf=64, tol=1e-6)
    tree = O.build_tree(X, p.leaf)
    near, far = O.build_lists(tree, p.eta)
    f = O.box_features(X, tree, near, far, 0, 0, n, 0, 0, p, 1.0)
    want = math.sqrt(a * a * (n + 1) / (12 * (n - 1))) / (a / 2)
    assert abs(f[9] - want) < 1e-6 and f[10] == 0 and f[11] == 0
    assert f[12] == 0.0 and f[2] == 0.0 and f[14] == 0.0
    leaf = O.box_features(X, tree, near, far, tree.L, 1, 64, 3, 100, p, 1.0)
    assert leaf[14] == 1.0 and leaf[2] == 1.0
    assert abs(leaf[0] - math.log2(65) / 12) < 1e-7 and abs(leaf[6] - math.log2(101) / 20) < 1e-7


def test_features_invariant_to_shift_and_scale():
    X = W.ellipsoid_points(2048, 3)
    p = O.Params(leaf=64, tol=1e-6)

    def feats(Y):
        tree = O.build_tree(Y, p.leaf)
        near, far = O.build_lists(tree, p.eta)
        return np.array([O.box_features(Y, tree, near, far, lev, i, 10, 2, 50, p, 0.5)
                         for lev in range(tree.L + 1) for i in range(1 << lev)])

    F = feats(X)
    assert np.allclose(feats(X * 4.0 + 1.5), F, rtol=0, atol=2e-6)


# --- sketched row ID -------------------------------------------------------
def _low_rank(m, n, r, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, n))


def test_sketch_row_id_exact_for_low_rank_matrix():
    """For an exactly rank-r matrix and a sketch of more than r columns, the
    skeleton rows span every row, so the interpolative decomposition is exact
    (randomized ID, Halko-Martinsson-Tropp 2011, Sec. 5.2)."""
    M = _low_rank(90, 400, 12, 4)
    Om = R.point_rows(3, 1, R.STREAM_FAR, np.arange(400), 400, 20 + O.SKETCH_PROBES)
    ok, k, piv, Wp, dg = O.sketch_row_id(M, 20, 1e-10, 90, Om)
    assert ok and k == 12
    assert np.linalg.norm(M - Wp @ M[piv[:k]]) <= 1e-9 * np.linalg.norm(M)
    assert np.array_equal(Wp[piv[:k]], np.eye(k))


def test_sketch_exhausted_is_rejected():
    M = _low_rank(90, 400, 30, 5)
    Om = R.point_rows(3, 1, R.STREAM_FAR, np.arange(400), 400, 16 + O.SKETCH_PROBES)
    ok, k, piv, Wp, dg = O.sketch_row_id(M, 16, 1e-10, 90, Om)
    assert not ok and k == 16


def test_predicted_mode_keeps_the_accuracy_class():
    """A model trained on the ranks of one factorization, used on another point
    set: sketched boxes are accepted and the error against dense LU stays in the
    class of the plain method."""
    p = O.Params(leaf=64, tol=1e-6)
    f0 = O.factorize(W.cube_points(2048, 21), p)
    F = np.concatenate([[b.feat for b in f0.levels[l]] for l in f0.levels])
    T = np.concatenate([[math.log2(1 + b.k) for b in f0.levels[l]] for l in f0.levels])
    th, hist = R.train(R.init_weights(1), F, T, 500, 3e-3)
    assert hist[-1] < 0.05
    X = W.cube_points(2048, 22)
    plain = O.factorize(X, p)
    pm = O.Params(leaf=64, tol=1e-6, rank_model=th.astype(np.float32), sketch_seed=5)
    fac = O.factorize(X, pm)
    states = [b.sketch for l in fac.levels for b in fac.levels[l]]
    assert states.count(1) >= 4
    b = W.gaussian_rhs(2048, 1, 8)[:, 0]
    xs = np.linalg.solve(O.dense_matrix(X, p), b)
    e_plain = np.linalg.norm(O.solve(plain, b) - xs) / np.linalg.norm(xs)
    e_pred = np.linalg.norm(O.solve(fac, b) - xs) / np.linalg.norm(xs)
    assert e_pred < max(1e-3, 5 * e_plain), (e_pred, e_plain)
    # every sketch is at most m - probes wide, wider than its predicted rank
    # unless that width is the cap, and an accepted one is wider than its rank
    for l in fac.levels:
        for bx in fac.levels[l]:
            if bx.sketch:
                assert 0 < bx.ell <= bx.m - O.SKETCH_PROBES
                assert bx.khat < bx.ell or bx.ell == bx.m - O.SKETCH_PROBES
            if bx.sketch in (1, 3):
                assert bx.k < bx.ell


def test_sketch_sized_by_prediction_saves_basis_work():
    """Where the predicted rank is well below m (leaf 256 of a sphere at tol
    1e-4: ranks about 50-60), a sketch sized by the prediction (k-hat = 60, 83
    columns) is accepted everywhere and costs fewer basis flops than the full QR;
    a prediction below some true leaf ranks (k-hat = 30, 46 columns) exhausts
    those sketches, which are retried at full width."""
    X = W.sphere_points(4096, 31)
    p = O.Params(leaf=256, tol=1e-4)
    plain = O.factorize(X, p)
    fac = O.factorize(X, O.Params(leaf=256, tol=1e-4, rank_model=_constant_mlp(60), sketch_seed=2))
    st = [b.sketch for l in fac.levels for b in fac.levels[l]]
    assert st.count(1) == len(st)
    assert fac.stats["flops"]["basis"] < 0.6 * plain.stats["flops"]["basis"]
    low = O.factorize(X, O.Params(leaf=256, tol=1e-4, rank_model=_constant_mlp(30), sketch_seed=2))
    L = low.tree.L
    leaves = low.levels[L]
    # exhausted first sketches are retried at full width (m - probes columns)
    retried = [b for b in leaves if b.sketch in (2, 3)]
    assert retried and all(b.ell == b.m - O.SKETCH_PROBES for b in retried)
    assert all(b.k < b.ell for b in leaves if b.sketch in (1, 3))


def _constant_mlp(k):
    parts = {name: np.zeros(s) for name, s in R.SHAPES}
    parts["b4"][0] = math.log2(1 + k)
    return R.pack(parts).astype(np.float32)


def test_rejected_sketch_without_fallback_reports_rank_check():
    """A model that predicts rank 10 everywhere with no oversampling exhausts
    every first sketch; boxes whose full-width retry fails too take the full
    pivoted QR by default, or stop the factorization with RANK_CHECK when the
    fallback is switched off."""
    parts = {name: np.zeros(s) for name, s in R.SHAPES}
    parts["b4"][0] = math.log2(1 + 10)
    th = R.pack(parts).astype(np.float32)
    X = W.cube_points(3000, 3901)
    kw = dict(leaf=64, tol=1e-6, rank_model=th, sketch_seed=77, oversample=0)
    f = O.factorize(X, O.Params(**kw))
    assert any(b.sketch == 2 for lev in f.levels.values() for b in lev)
    with pytest.raises(O.OracleError) as e:
        O.factorize(X, O.Params(sketch_fallback=False, **kw))
    assert e.value.status == O.ERR_RANK_CHECK


def test_sketch_min_level_keeps_the_top_levels_on_the_full_qr():
    """With sketch_min_level the levels above it take the full pivoted QR (no
    sketch) and the levels from it down are sketched; the threshold L + 1, one
    past the leaf level, sketches nothing and gives the plain factorization."""
    parts = {name: np.zeros(s) for name, s in R.SHAPES}
    parts["b4"][0] = math.log2(1 + 10000)
    th = R.pack(parts).astype(np.float32)
    X = W.cube_points(4096, 3907)
    kw = dict(leaf=128, tol=1e-6, rank_cap=32, rank_model=th, sketch_seed=77, oversample=8)
    plain = O.factorize(X, O.Params(leaf=128, tol=1e-6, rank_cap=32))
    L = plain.tree.L
    f = O.factorize(X, O.Params(sketch_min_level=L, **kw))
    for lev in range(1, L + 1):
        st = [b.sketch for b in f.levels[lev]]
        if lev < L:
            assert all(s_ == 0 for s_ in st) and all(b.ell == 0 for b in f.levels[lev])
        else:
            assert any(s_ in (1, 3) for s_ in st)
    none = O.factorize(X, O.Params(sketch_min_level=L + 1, **kw))
    b = W.gaussian_rhs(4096, 1, 2)
    assert all(bx.sketch == 0 for lev in none.levels.values() for bx in lev)
    for lev in range(1, L + 1):
        assert [bx.k for bx in none.levels[lev]] == [bx.k for bx in plain.levels[lev]]
    assert np.array_equal(O.solve(none, b), O.solve(plain, b))
    with pytest.raises(O.OracleError):
        O.factorize(X, O.Params(sketch_min_level=-1, **kw))
