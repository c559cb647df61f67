"""GPU parity: the HIP library (through the C-ABI) against the CPU oracle on the
same seeded inputs.

Bar (FP64 path): integer structure (ranks k, skeleton indices in pivot order)
identical; solution within 1e-10 relative of the oracle's; log|det| and the
algorithmic flop count equal to rounding.  Where the oracle cannot run the full
size, a sample of leaf boxes is checked box by box (the oracle restricted to the
boxes they depend on) and the solution is checked through its residual with the
exact matvec, a property that holds at any size.
"""
import numpy as np
import pytest

import workloads as W
from oracle import h2ulv_ref as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
H = pytest.importorskip("paper_2208_10907_amd.h2ulv")

X_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.lib()


def _params(op: O.Params, **kw):
    kw.setdefault("structure", op.structure)
    kw.setdefault("drift", op.drift)
    kw.setdefault("bases", op.bases)
    return H.make_params(kernel=op.kernel, alpha=op.alpha, diag=op.diag, eta=op.eta,
                         leaf=op.leaf, tol=op.tol, rank_cap=op.rank_cap,
                         far_sample=op.far_sample, **kw)


def _proj_bound(tol: float) -> float:
    """Bound on |U^S U^S^T - U_o^S U_o^S^T| for a box whose pivot order matches
    the oracle's: the bases then differ only through E = R11^-1 R12, whose
    rounding error is about eps cond(R11) <= eps |R_00| / |R_kk| <= eps / tol
    (every kept pivot has |R_tt| > tol |R_00|).  Measured differences stay
    below 0.15 eps / tol; the bound is 1.35 eps / tol, at least 1e-12."""
    return max(1e-12, 3e-16 / tol) if tol > 0 else 1e-12


def _compare_structure(fg, fo):
    L = fo.tree.L
    assert fg.levels() == L
    assert np.array_equal(fg.perm(), fo.tree.perm)
    for lev in sorted(fo.levels, reverse=True):
        m, k = fg.ranks(lev)
        assert np.array_equal(m, [b.m for b in fo.levels[lev]]), f"m differs at level {lev}"
        assert np.array_equal(k, [b.k for b in fo.levels[lev]]), f"k differs at level {lev}"
        for i in range(1 << lev):
            _compare_skeleton(fg.skeleton(lev, i), fo.levels[lev][i], (lev, i))


def _compare_skeleton(sk_gpu, bo, where):
    """Skeleton indices in pivot order must agree while the pivot norm is above
    rounding noise (1e-10 |R_00|); pivots below it are ties decided by rounding,
    so the tail is compared as a set."""
    k = bo.k
    dg = bo.absdiag
    nz = k
    if dg is not None and len(dg) and dg[0] > 0:
        nz = min(k, int(np.sum(dg[:k] > 1e-10 * dg[0])))
    assert np.array_equal(sk_gpu[:nz], bo.sk[:nz]), where
    assert sorted(sk_gpu[nz:].tolist()) == sorted(bo.sk[nz:].tolist()) or k < bo.m, where


def _parity(X, op, nrhs=1, rhs_seed=7, check_basis=True):
    fo = O.factorize(X, op)
    fg = H.factorize(X, _params(op))
    _compare_structure(fg, fo)
    if check_basis:
        lev = fo.tree.L
        for i in (0, (1 << lev) - 1) if lev else ():
            U = fg.basis(lev, i)
            Uo = fo.levels[lev][i].U
            k = fo.levels[lev][i].k
            assert np.abs(U.T @ U - np.eye(U.shape[0])).max() < 1e-13 * max(1, U.shape[0])
            if k:
                Pg = U[:, :k] @ U[:, :k].T
                Po = Uo[:, :k] @ Uo[:, :k].T
                assert np.abs(Pg - Po).max() < _proj_bound(op.tol)
    b = W.gaussian_rhs(X.shape[0], nrhs, rhs_seed)
    xo = O.solve(fo, b)
    xg = fg.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    assert rel < X_TOL, rel
    st = fg.stats()
    assert abs(st["logabsdet"] - O.logabsdet(fo)) <= 1e-10 * abs(O.logabsdet(fo))
    assert abs(st["flops"] - O.total_flops(fo)) <= 1e-9 * O.total_flops(fo)
    return fg, fo


def test_small_cube_fp64():
    """N=2048 unit cube, leaf 64, tol 1e-8, cap 32, one RHS (exact far field)."""
    prob = W.small_cube()
    _parity(prob.points, O.params_from_problem(prob), nrhs=1, rhs_seed=prob.rhs_seed)


@pytest.mark.parametrize("n,leaf,tol,cap,fs,nrhs", [
    (3000, 64, 1e-6, 0, 32, 3),      # ragged leaves, sampled far field, rank growth
    (4096, 128, 1e-8, 0, 32, 1),     # several 64-tiles per block, ranks > 256 above
    (1500, 40, 0.0, 0, 0, 2),        # tol 0: no truncation (k = m)
    (512, 64, 1e-8, 0, 0, 1),        # small cube, exact far field
    (1200, 64, 1e-3, 1, 16, 1),      # rank cap 1
    (2000, 64, 1e-7, 0, 32, 4),      # widest right-hand side of the vector-unit products
    (2000, 64, 1e-7, 0, 32, 5),      # one column more: the solve's products on MFMA tiles
])
def test_cube_variants(n, leaf, tol, cap, fs, nrhs):
    X = W.cube_points(n, n)
    _parity(X, O.Params(leaf=leaf, tol=tol, rank_cap=cap, far_sample=fs), nrhs=nrhs)


def test_yukawa_boxes():
    X = W.box_problem(0)[:2500]
    _parity(X, O.Params(kernel=O.YUKAWA, alpha=0.5, leaf=128, tol=1e-7, far_sample=32))


def test_hss_limit_and_sphere():
    _parity(W.sphere_points(2000, 4), O.Params(leaf=64, tol=1e-7, eta=0.0, far_sample=32))


@pytest.mark.parametrize("n", [1, 2, 50])
def test_root_only(n):
    X = W.cube_points(n, 11)
    _parity(X, O.Params(leaf=64, tol=1e-8, far_sample=0), nrhs=2, check_basis=False)


@pytest.mark.parametrize("kernel,n,nrhs", [(O.YUKAWA, 3000, 9), (O.LAPLACE, 3001, 4),
                                             (O.LAPLACE, 700, 1)])
def test_matvec_exact(kernel, n, nrhs):
    """Exact matvec (512-target workgroups with a ragged tail; blocks of 8 and 4
    columns on the matrix cores, single columns on the vector units) against
    the oracle, column by column."""
    X = W.sphere_points(n, 5)
    op = O.Params(kernel=kernel, alpha=0.5, leaf=128)
    fg = H.factorize(X, _params(op))
    x = W.gaussian_rhs(n, nrhs, 3)
    y = fg.matvec(torch.tensor(x, device="cuda")).cpu().numpy().reshape(n, nrhs)
    yo = O.matvec_exact(X, x, op).reshape(n, nrhs)
    for c in range(nrhs):
        assert np.linalg.norm(y[:, c] - yo[:, c]) / np.linalg.norm(yo[:, c]) < 1e-14, c


@pytest.mark.parametrize("kernel,n,nrhs", [(O.LAPLACE, 70001, 13), (O.YUKAWA, 66000, 1),
                                             (O.YUKAWA, 65537, 8), (O.LAPLACE, 300001, 9),
                                             (O.YUKAWA, 262657, 8), (O.LAPLACE, 300001, 1),
                                             (O.YUKAWA, 262657, 13)])
def test_matvec_split_sampled(kernel, n, nrhs):
    """Exact matvec at sizes where the sources are split over several
    workgroups (partial sums added in a fixed order) and, from 512 tiles of 512
    points on, in the pair forms (each unordered pair evaluated once, ragged
    last tile; blocks of 8 columns and single columns, 13 = 8 + 4 + 1): sampled
    rows against the oracle's kernel rows, and two calls give identical bits."""
    X = W.sphere_points(n, 8)
    op = O.Params(kernel=kernel, alpha=0.5, leaf=256, tol=1e-3)
    fg = H.factorize(X, _params(op))
    x = W.gaussian_rhs(n, nrhs, 4)
    xt = torch.tensor(x, device="cuda")
    y = fg.matvec(xt).cpu().numpy().reshape(n, nrhs)
    y2 = fg.matvec(xt).cpu().numpy().reshape(n, nrhs)
    assert np.array_equal(y, y2)
    rows = np.random.default_rng(3).choice(n, 48, replace=False)
    rows[0], rows[1] = 0, n - 1
    yo = O.kernel_block(X, rows, np.arange(n), op) @ x.reshape(n, nrhs)
    assert np.linalg.norm(y[rows] - yo) / np.linalg.norm(yo) < 1e-14


def test_refine_gmres_matches_refinement():
    """GMRES-accelerated refinement reaches the same 1e-10 residual in no more
    steps than classical refinement, with the same solution; a too small step
    budget reports NOT_CONVERGED."""
    X = W.cube_points(4000, 6)
    op = O.Params(leaf=64, tol=1e-4, far_sample=32)
    fg = H.factorize(X, _params(op))
    b = torch.tensor(W.gaussian_rhs(4000, 3, 8), device="cuda")
    x1, it1, rel1 = fg.refine(b, rtol=1e-10, max_iter=40)
    x2, it2, rel2 = fg.refine_gmres(b, rtol=1e-10, max_iter=40, restart=20)
    assert rel1 <= 1e-10 and rel2 <= 1e-10
    assert it2 <= it1
    assert torch.linalg.norm(x1 - x2) / torch.linalg.norm(x1) < 1e-8
    # against the oracle's matrix: the residual is a property of any size
    r = O.matvec_exact(X, x2.cpu().numpy(), op) - b.cpu().numpy()
    assert np.linalg.norm(r) / np.linalg.norm(b.cpu().numpy()) < 1e-9
    x3, it3, rel3 = fg.refine_gmres(b, rtol=1e-14, max_iter=2, raise_on_fail=False)
    assert it3 <= 3 and rel3 > 1e-14
    with pytest.raises(H.H2ULVError) as e:
        fg.refine_gmres(b, rtol=1e-14, max_iter=2)
    assert e.value.status == H.ERR_NOT_CONVERGED


def test_refine_and_not_converged():
    X = W.cube_points(4000, 6)
    op = O.Params(leaf=64, tol=1e-4, far_sample=32)
    fg = H.factorize(X, _params(op))
    b = torch.tensor(W.gaussian_rhs(4000, 4, 8), device="cuda")
    x, it, rel = fg.refine(b, rtol=1e-10, max_iter=20)
    assert rel <= 1e-10 and it >= 1
    r = b.cpu().numpy() - O.matvec_exact(X, x.cpu().numpy(), op)
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(b.cpu().numpy(), axis=0)) < 2e-10
    with pytest.raises(H.H2ULVError) as e:
        fg.refine(b, rtol=1e-15, max_iter=0)
    assert e.value.status == H.ERR_NOT_CONVERGED


def test_error_statuses():
    X = W.cube_points(300, 2)
    X[10] = X[200]
    with pytest.raises(H.H2ULVError) as e:
        H.factorize(X, H.make_params(leaf=64))
    assert e.value.status == H.ERR_DUPLICATE_POINTS
    with pytest.raises(H.H2ULVError) as e:
        H.factorize(W.cube_points(1, 1), H.make_params(leaf=64, diag=0.0))
    assert e.value.status == H.ERR_SINGULAR


def test_deterministic():
    X = W.cube_points(3000, 12)
    p = H.make_params(leaf=64, tol=1e-7)
    b = torch.tensor(W.gaussian_rhs(3000, 2, 1), device="cuda")
    x1 = H.factorize(X, p).solve(b)
    x2 = H.factorize(X, p).solve(b)
    assert torch.equal(x1, x2)


def test_batch_equals_single():
    probs = [W.cube_points(n, 40 + n) for n in (700, 1500, 2600)]
    p = H.make_params(kernel=H.YUKAWA, alpha=0.5, leaf=64, tol=1e-7)
    fb = H.factorize_batch(probs, p)
    for X, f in zip(probs, fb):
        b = torch.tensor(W.gaussian_rhs(X.shape[0], 1, 5), device="cuda")
        assert torch.allclose(f.solve(b), H.factorize(X, p).solve(b), rtol=0, atol=1e-13)


def _sampled_leaf_parity(prob, boxes, precision=H.FP64):
    op = O.params_from_problem(prob)
    fg = H.factorize(prob.points, H.params_from_problem(prob, precision=precision))
    L = fg.levels()
    fo = O.factorize(prob.points, op, level_stop=L, boxes=set(boxes))
    m, k = fg.ranks(L)
    for i in boxes:
        bo = fo.levels[L][i]
        assert k[i] == bo.k and m[i] == bo.m, (i, k[i], bo.k)
        _compare_skeleton(fg.skeleton(L, i), bo, (L, i))
        U = fg.basis(L, i)
        Pg = U[:, :bo.k] @ U[:, :bo.k].T
        Po = bo.U[:, :bo.k] @ bo.U[:, :bo.k].T
        assert np.abs(Pg - Po).max() < _proj_bound(op.tol)
    return fg


def test_sphere_65536_sampled():
    """N=65536 on the sphere, leaf 256, tol 1e-8, cap 128, 16 RHS: leaf boxes
    checked against the oracle one by one; the solve through its residual."""
    prob = W.sphere65k()
    fg = _sampled_leaf_parity(prob, [0, 77, 255])
    b = torch.tensor(prob.rhs(), device="cuda")
    x = fg.solve(b)
    r = b - fg.matvec(x)
    rel = (torch.linalg.norm(r, dim=0) / torch.linalg.norm(b, dim=0)).max().item()
    assert rel < 0.1  # rank cap 128 limits one solve's accuracy; refinement recovers it
    x2, it, rr = fg.refine(b, rtol=1e-10, max_iter=30)
    assert rr <= 1e-10
    # the refined residual with the oracle's matvec (two of the 16 columns)
    bn = b.cpu().numpy()[:, :2]
    r = bn - O.matvec_exact(prob.points, x2.cpu().numpy()[:, :2], O.params_from_problem(prob))
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bn, axis=0)) < 2e-10


def test_cube_1048576_full_size():
    """The benchmark's workload at its full size (N = 2^20 in the unit cube,
    leaf 256, tol 1e-6, cap 128, 8 right-hand sides), checked where the oracle
    can follow one output at a time: leaf boxes of the FP64 form against the
    oracle; the pair-form exact matvec (2048 tiles) on sampled rows against the
    oracle's kernel rows, twice with the same bits; and the benchmark's form
    (mixed precision, every box sketched at full width by a rank model that
    predicts above the cap, oversampling 88) refined to 1e-10 with block GMRES,
    its residual recomputed on sampled rows from the oracle's kernel rows."""
    import math
    from oracle import rank_model as R
    prob = W.cube1m()
    n = prob.n
    op = O.params_from_problem(prob)
    fg = _sampled_leaf_parity(prob, [0, 1777, 4095])
    b = torch.tensor(prob.rhs(), device="cuda")
    rows = np.random.default_rng(3).choice(n, 32, replace=False)
    rows[0], rows[1] = 0, n - 1
    Krows = O.kernel_block(prob.points, rows, np.arange(n), op)
    y = fg.matvec(b)
    y2 = fg.matvec(b)
    assert torch.equal(y, y2)
    yo = Krows @ prob.rhs()
    assert np.linalg.norm(y.cpu().numpy().reshape(n, -1)[rows] - yo) / np.linalg.norm(yo) < 1e-14
    del fg, y, y2
    parts = {name: np.zeros(s) for name, s in R.SHAPES}
    parts["b4"][0] = math.log2(1 + 10000)
    gm = H.RankModel()
    gm.set_params(R.pack(parts).astype(np.float32))
    fh = H.factorize(prob.points, H.params_from_problem(prob, precision=H.MIXED, rank_model=gm,
                                                        sketch_seed=5, oversample=88))
    for lev in range(1, fh.levels() + 1):
        m, _ = fh.ranks(lev)
        kh, ell, st = fh.sketch_info(lev)
        assert (st == 1).all() and np.array_equal(ell, m - 8), lev
    x, it, rel = fh.refine_block_gmres(b, rtol=1e-10, max_iter=100, restart=60)
    assert rel <= 1e-10 and it < 60, (rel, it)
    r = (b - fh.matvec(x)).cpu().numpy().reshape(n, -1)
    xn, bn = x.cpu().numpy().reshape(n, -1), prob.rhs()
    ro = bn[rows] - Krows @ xn
    # the sampled rows of the residual, recomputed from the oracle's kernel rows,
    # are as small as the whole; the GPU's agree with them to the rounding of
    # the two sums over 2^20 terms (|A_ij x_j| summed is ~1e3 |b_i|)
    assert np.linalg.norm(ro) / np.linalg.norm(bn[rows]) < 1e-9
    assert np.abs(r[rows] - ro).max() <= 1e-11 * np.abs(bn[rows]).max()


def test_ellipsoids_262144_full_size():
    """The learned-rank workload at its full size (N = 262144 on 12 ellipsoid
    surfaces, leaf 256, tol 1e-6, cap 128): leaf boxes of the plain FP64 form
    against the oracle box by box; a rank model trained on the GPU from the
    ranks of two 65536-point sets of the same family; the predicted form
    (mixed precision, the benchmark's oversampling 88) refined to 1e-10 with
    block GMRES in one cycle of up to 128 steps, with nearly every
    sketch accepted, and its residual recomputed on sampled rows from the
    oracle's kernel rows."""
    prob = W.ellipsoids()
    n = prob.n
    op = O.params_from_problem(prob)
    fg = _sampled_leaf_parity(prob, [0, 500, 1023])
    del fg
    F, T = [], []
    for seed in (501, 502):
        f = H.factorize(W.ellipsoid_points(65536, seed), H.params_from_problem(prob))
        for lev in range(1, f.levels() + 1):
            a, t = f.features(lev)
            F.append(a)
            T.append(t)
        del f
    gm = H.RankModel(seed=1)
    loss = gm.train(torch.tensor(np.concatenate(F), device="cuda"),
                    torch.tensor(np.concatenate(T), device="cuda"), 2000, 3e-3)
    assert loss < 0.05
    fh = H.factorize(prob.points, H.params_from_problem(prob, precision=H.MIXED, rank_model=gm,
                                                        sketch_seed=5, oversample=88))
    acc = tot = 0
    for lev in range(1, fh.levels() + 1):
        kh, ell, st = fh.sketch_info(lev)
        acc += int(((st == 1) | (st == 3)).sum())
        tot += int((st != 0).sum())
    assert tot > 0 and acc >= 0.9 * tot, (acc, tot)
    b = torch.tensor(prob.rhs(), device="cuda")
    # one right-hand side and a weak capped preconditioner: about 100 block steps,
    # which a restart after 60 would stall
    x, it, rel = fh.refine_block_gmres(b, rtol=1e-10, max_iter=200, restart=128)
    assert rel <= 1e-10, (rel, it)
    rows = np.random.default_rng(5).choice(n, 32, replace=False)
    rows[0], rows[1] = 0, n - 1
    xn, bn = x.cpu().numpy().reshape(n, -1), prob.rhs().reshape(n, -1)
    ro = bn[rows] - O.kernel_block(prob.points, rows, np.arange(n), op) @ xn
    assert np.linalg.norm(ro) / np.linalg.norm(bn[rows]) < 1e-9


def test_mixed_precision_refines_to_fp64_accuracy():
    """FP32 couplings, rotations and Schur updates with FP64 fill-in products
    (no rank cap), QR/ID, inverses, solve and residual: one solve is close to the
    FP64 factor's, and refinement with the exact FP64 matvec reaches 1e-10,
    rechecked with the oracle's matvec."""
    X = W.cube_points(6000, 21)
    prob_kw = dict(leaf=128, tol=1e-6, far_sample=32)
    f64 = H.factorize(X, H.make_params(**prob_kw))
    f32 = H.factorize(X, H.make_params(precision=H.MIXED, **prob_kw))
    b = torch.tensor(W.gaussian_rhs(6000, 3, 4), device="cuda")
    x64 = f64.solve(b)
    x32 = f32.solve(b)
    one_shot = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
    assert one_shot < 1e-3, one_shot
    y64, it64, r64 = f64.refine(b, rtol=1e-10, max_iter=40)
    y32, it32, r32 = f32.refine(b, rtol=1e-10, max_iter=40)
    assert r64 <= 1e-10 and r32 <= 1e-10
    bn = b.cpu().numpy()
    r = bn - O.matvec_exact(X, y32.cpu().numpy(), O.Params(**prob_kw))
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bn, axis=0)) < 2e-10
    assert (torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64)).item() < 1e-8
    assert it32 <= it64 + 3


def test_batch_matches_oracle_per_problem():
    """Several problems of different tree depths factorized in one batched pass
    (shared launches per height) each match the oracle run on its own: ranks and
    skeletons identical, solution within 1e-10 (Yukawa kernel, leaf 128, tol 1e-7,
    rank cap 64 as the batched workload)."""
    sizes = (900, 1700, 3300, 5000)  # 3, 4, 5 and 6 levels
    pts = [W.aspect_box_points(n, 3200 + n) for n in sizes]
    op = O.Params(kernel=O.YUKAWA, alpha=0.5, leaf=128, tol=1e-7, rank_cap=64, far_sample=32)
    fb = H.factorize_batch(pts, _params(op))
    depths = set()
    for X, fg in zip(pts, fb):
        fo = O.factorize(X, op)
        depths.add(fo.tree.L)
        _compare_structure(fg, fo)
        b = W.gaussian_rhs(X.shape[0], 1, 9)
        xo = O.solve(fo, b)
        xg = fg.solve(torch.tensor(b, device="cuda")).cpu().numpy()
        assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < X_TOL
    assert len(depths) == len(sizes)


def test_panels_beyond_4096_rows():
    """Leaf boxes of 4200 points: the LU of the diagonal blocks (fill-in step)
    and the Householder panels of the tall QR run their >4096-row kernels; the
    result still matches the oracle."""
    X = W.cube_points(8400, 31)
    op = O.Params(leaf=4200, tol=1e-6, far_sample=0)
    fg, fo = _parity(X, op, check_basis=False)
    m, k = fg.ranks(1)
    assert m.min() > 4096


def test_capped_mixed_precision_against_oracle_residual():
    """Mixed precision with a rank cap (FP32 fill-in products as well): refinement
    with the exact FP64 matvec reaches 1e-10, checked with the oracle's matvec,
    and the solution agrees with the refined FP64 one."""
    X = W.cube_points(6000, 22)
    kw = dict(leaf=128, tol=1e-6, rank_cap=64, far_sample=32)
    op = O.Params(**kw)
    f64 = H.factorize(X, H.make_params(**kw))
    f32 = H.factorize(X, H.make_params(precision=H.MIXED, **kw))
    b = torch.tensor(W.gaussian_rhs(6000, 2, 5), device="cuda")
    y64, _, r64 = f64.refine_gmres(b, rtol=1e-10, max_iter=60)
    y32, _, r32 = f32.refine_gmres(b, rtol=1e-10, max_iter=60)
    assert r64 <= 1e-10 and r32 <= 1e-10
    bn = b.cpu().numpy()
    for y in (y32, y64):
        r = bn - O.matvec_exact(X, y.cpu().numpy(), op)
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bn, axis=0)) < 2e-10
    assert (torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64)).item() < 1e-8


def test_tolerance_one_eliminates_every_box():
    """tol = 1: no pivot exceeds |R_00| strictly, so k = 0 in every leaf box, the
    boxes above the leaves are empty (m = 0) and the root is 0 x 0; the result is
    the leaf-level elimination alone, identical to the oracle's."""
    X = W.cube_points(2000, 33)
    op = O.Params(leaf=64, tol=1.0, far_sample=32)
    fg, fo = _parity(X, op, check_basis=False)
    L = fo.tree.L
    m, k = fg.ranks(L)
    assert k.max() == 0 and m.min() > 0
    for lev in range(L - 1, 0, -1):
        m, k = fg.ranks(lev)
        assert m.max() == 0 and k.max() == 0
    assert fg.stats()["root_size"] == 0


def test_caller_allocator_supplies_all_factor_memory():
    """h2ulv_allocator: every device block of the factorization and of later
    calls comes from the caller (here torch's caching allocator, counted) and
    goes back to it by h2ulv_destroy (a solve's temporaries right away, the
    recorded solve graphs' buffers with the factor); results equal those with
    the library's own cache.  A callback that returns NULL gives OOM at the first allocation,
    before any device work."""
    X = W.cube_points(3000, 41)
    p = H.make_params(leaf=64, tol=1e-7, rank_cap=32)
    live, calls = {}, {"alloc": 0, "free": 0}

    def alloc(nbytes, stream):
        ptr = torch.cuda.caching_allocator_alloc(nbytes, stream=stream or None)
        live[ptr] = nbytes
        calls["alloc"] += 1
        return ptr

    def free(ptr, stream):
        assert ptr in live
        del live[ptr]
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    al = H.make_allocator(alloc, free)
    b = torch.tensor(W.gaussian_rhs(3000, 2, 3), device="cuda")
    f = H.factorize(X, p, allocator=al)
    held = len(live)
    assert held > 0 and calls["alloc"] > held  # temporaries came and went
    x = f.solve(b)
    assert len(live) == held  # a solve's temporaries given back
    xr, _, rr = f.refine_gmres(b, rtol=1e-10)
    assert rr <= 1e-10
    # the refinement records its solves in HIP graphs whose buffers (from the
    # caller's allocator) the factor keeps; a second refinement replays them and
    # holds nothing more
    held_graphs = len(live)
    xr2, _, rr2 = f.refine_gmres(b, rtol=1e-10)
    assert len(live) == held_graphs and torch.equal(xr, xr2)
    g = H.factorize(X, p, allocator=None)
    assert torch.equal(x, g.solve(b))
    del f
    torch.cuda.synchronize()
    assert not live and calls["alloc"] == calls["free"]
    refused = {"n": 0}

    def no_memory(nbytes, stream):
        refused["n"] += 1
        return 0

    with pytest.raises(H.H2ULVError) as e:
        H.factorize(X, p, allocator=H.make_allocator(no_memory, lambda ptr, s: None))
    assert e.value.status == H.ERR_OOM
    assert refused["n"] == 1


def test_no_fill_in_ablation_matches_oracle():
    """The ablation with bases from the low-rank blocks alone (fill_in = 0)
    matches the oracle run the same way (ranks, skeletons, solution, flops)."""
    X = W.cube_points(3000, 44)
    op = O.Params(leaf=64, tol=1e-6, far_sample=32, fill_in=False)
    fg = H.factorize(X, _params(op, fill_in=False))
    fo = O.factorize(X, op)
    _compare_structure(fg, fo)
    b = W.gaussian_rhs(3000, 1, 2)
    xo = O.solve(fo, b)
    xg = fg.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < X_TOL
    assert abs(fg.stats()["flops"] - O.total_flops(fo)) <= 1e-9 * O.total_flops(fo)


def test_gemm_tile_autotuner():
    """The grouped GEMM's tile shapes are chosen from rates measured on the
    device the first time a precision is used; the rates are plausible for the
    matrix cores (below the FP64 / FP32 peaks of 78.6 / 157.3 TFLOP/s)."""
    X = W.cube_points(3000, 45)
    H.factorize(X, H.make_params(leaf=64, tol=1e-7, rank_cap=32, precision=H.MIXED))
    r = H.gemm_tile_rates()
    f64 = [r[k] for k in r if k.startswith("f64")]
    f32 = [r[k] for k in r if k.startswith("f32")]
    assert all(2.0 < v < 78.6 for v in f64), r
    assert all(4.0 < v < 157.3 for v in f32), r


def test_kmeans_partition_matches_oracle():
    """The balanced 2-means cluster tree (the k-means partition of Sec. V) on a
    surface point set: tree, ranks, skeletons and solution match the oracle."""
    X = W.ellipsoid_points(4000, 8)
    op = O.Params(leaf=64, tol=1e-6, rank_cap=32, far_sample=32, partition="kmeans")
    fg = H.factorize(X, _params(op, partition="kmeans"))
    fo = O.factorize(X, op)
    _compare_structure(fg, fo)
    b = W.gaussian_rhs(4000, 2, 6)
    xo = O.solve(fo, b)
    xg = fg.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < X_TOL


def test_block_gmres_refinement():
    """Block GMRES over all right-hand sides reaches the same 1e-10 residual
    (rechecked with the oracle's matvec) and the same solution as the lockstep
    GMRES, in no more block steps than the lockstep one takes steps; a too small
    step budget reports NOT_CONVERGED."""
    X = W.cube_points(5000, 46)
    op = O.Params(leaf=64, tol=1e-4, rank_cap=16, far_sample=32)
    fg = H.factorize(X, _params(op))
    b = torch.tensor(W.gaussian_rhs(5000, 6, 10), device="cuda")
    x1, it1, rel1 = fg.refine_gmres(b, rtol=1e-10, max_iter=200, restart=60)
    x2, it2, rel2 = fg.refine_block_gmres(b, rtol=1e-10, max_iter=200, restart=60)
    assert rel1 <= 1e-10 and rel2 <= 1e-10
    assert it2 <= it1
    assert torch.linalg.norm(x1 - x2) / torch.linalg.norm(x1) < 1e-8
    bn = b.cpu().numpy()
    r = bn - O.matvec_exact(X, x2.cpu().numpy(), op)
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bn, axis=0)) < 2e-10
    # one right-hand side: block GMRES is ordinary GMRES
    x3, it3, rel3 = fg.refine_block_gmres(b[:, :1], rtol=1e-10, max_iter=200, restart=60)
    assert rel3 <= 1e-10
    x4, it4, rel4 = fg.refine_block_gmres(b, rtol=1e-14, max_iter=2, raise_on_fail=False)
    assert it4 <= 2 and rel4 > 1e-14
    with pytest.raises(H.H2ULVError) as e:
        fg.refine_block_gmres(b, rtol=1e-14, max_iter=2)
    assert e.value.status == H.ERR_NOT_CONVERGED


@pytest.mark.parametrize("n,leaf,tol,eta,fs,kernel", [
    (2048, 64, 1e-8, 1.0, 0, O.LAPLACE), (3001, 100, 1e-6, 1.0, 16, O.YUKAWA),
    (1500, 64, 1e-6, 0.0, 0, O.LAPLACE)])
def test_flat_blr2_matches_oracle(n, leaf, tol, eta, fs, kernel):
    """Flat BLR^2 (Sec. II-B): one level of leaves, every pair classified
    directly, all skeletons in one root block.  Ranks and skeletons of the leaf
    level identical, the root as large as the sum of the leaf ranks, solution
    within 1e-10 of the oracle's; levels above the leaves hold nothing."""
    X = W.cube_points(n, 4)
    op = O.Params(kernel=kernel, alpha=0.5, leaf=leaf, tol=tol, eta=eta, far_sample=fs,
                  structure="blr2")
    fg, fo = _parity(X, op, nrhs=3)
    L = fo.tree.L
    assert fg.stats()["root_size"] == sum(b.k for b in fo.levels[L]) == fo.m_root
    if L > 1:
        with pytest.raises(H.H2ULVError):
            fg.ranks(L - 1)


class _ColumnSide:
    """The column side of an oracle box in the shape _compare_skeleton reads."""

    def __init__(self, bo):
        self.k, self.m, self.sk, self.absdiag = bo.k, bo.m, bo.skV, bo.absdiagV


ADV = dict(kernel=O.ADVECTION, alpha=1.0, drift=(0.6, -0.3, 0.5))


@pytest.mark.parametrize("n,leaf,tol,cap,fs,kw", [
    (2048, 64, 1e-8, 0, 0, ADV), (3000, 100, 1e-6, 0, 32, ADV), (1500, 64, 0.0, 0, 0, ADV),
    (2500, 64, 1e-7, 24, 16, ADV), (2048, 64, 1e-8, 0, 0, dict(bases="separate"))])
def test_separate_bases_match_oracle(n, leaf, tol, cap, fs, kw):
    """Separate row and column bases (Eq. fillu/fillv) on the nonsymmetric
    advection-diffusion kernel, and on Laplace when asked for: row and column
    ranks and skeletons identical to the oracle's, solution within 1e-10,
    log|det| and flops to rounding; the column bases are orthogonal and span the
    oracle's."""
    X = W.cube_points(n, 3)
    op = O.Params(leaf=leaf, tol=tol, rank_cap=cap, far_sample=fs, **kw)
    fg, fo = _parity(X, op, nrhs=2, check_basis=False)
    for lev in fo.levels:
        for i in range(1 << lev):
            _compare_skeleton(fg.column_skeleton(lev, i), _ColumnSide(fo.levels[lev][i]),
                              ("col", lev, i))
    lev = fo.tree.L
    for i in (0, (1 << lev) - 1):
        V = fg.column_basis(lev, i)
        bo = fo.levels[lev][i]
        assert np.abs(V.T @ V - np.eye(V.shape[0])).max() < 1e-13 * max(1, V.shape[0])
        if 0 < bo.k:
            Pg = V[:, :bo.k] @ V[:, :bo.k].T
            Po = bo.V[:, :bo.k] @ bo.V[:, :bo.k].T
            assert np.abs(Pg - Po).max() < _proj_bound(op.tol)


def test_advection_matvec_and_refinement():
    """The exact matvec of the nonsymmetric kernel against the oracle (8-, 4-
    and 1-column blocks), and block GMRES refinement to 1e-10 with the residual
    recomputed by the oracle."""
    n = 3001
    X = W.cube_points(n, 9)
    op = O.Params(leaf=128, tol=1e-5, far_sample=16, **ADV)
    fg = H.factorize(X, _params(op))
    x = W.gaussian_rhs(n, 13, 3)
    y = fg.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    yo = O.matvec_exact(X, x, op)
    for c in range(13):
        assert np.linalg.norm(y[:, c] - yo[:, c]) / np.linalg.norm(yo[:, c]) < 1e-14, c
    b = W.gaussian_rhs(n, 3, 4)
    xs, iters, rel = fg.refine_block_gmres(torch.tensor(b, device="cuda"), rtol=1e-10,
                                           max_iter=100, restart=30)
    xs = xs.cpu().numpy()
    r = b - O.matvec_exact(X, xs, op)
    assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)) < 1e-10
    assert iters > 0


@pytest.mark.parametrize("kw", [dict(kernel=O.ADVECTION, alpha=1.0, drift=(0.6, -0.3, 0.5)),
                                dict(kernel=O.LAPLACE, structure="blr2")])
def test_batch_separate_bases_and_flat(kw):
    """Batched factorization with separate row and column bases (each problem's
    column side in the same launches) and with the flat BLR^2 structure: every
    problem matches the oracle run on its own (row and column skeletons, solution
    within 1e-10)."""
    sizes = (700, 1500, 2600)
    pts = [W.cube_points(n, 4100 + n) for n in sizes]
    op = O.Params(leaf=64, tol=1e-7, far_sample=16, **kw)
    fb = H.factorize_batch(pts, _params(op))
    for X, fg in zip(pts, fb):
        fo = O.factorize(X, op)
        _compare_structure(fg, fo)
        if op.kernel == O.ADVECTION:
            for lev in fo.levels:
                for i in range(1 << lev):
                    _compare_skeleton(fg.column_skeleton(lev, i),
                                      _ColumnSide(fo.levels[lev][i]), ("col", lev, i))
        b = W.gaussian_rhs(X.shape[0], 2, 9)
        xo = O.solve(fo, b)
        xg = fg.solve(torch.tensor(b, device="cuda")).cpu().numpy()
        assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < X_TOL



@pytest.mark.parametrize("kw", [dict(), dict(kernel=O.ADVECTION, alpha=1.0, drift=(0.6, -0.3, 0.5)),
                                dict(structure="blr2")])
def test_solve_graph_replays_equal_eager_solves(kw):
    """The solve recorded in a HIP graph (h2ulv_solve_repeated, used by the
    refinement loops) gives the eager solve's bits on every replay: several
    right-hand-side counts, new right-hand sides each time, eager solves and
    matvecs between the replays."""
    n = 6000 if kw.get("structure") == "blr2" else 20000
    X = W.cube_points(n, 77)
    op = O.Params(leaf=128, tol=1e-6, far_sample=16, **kw)
    fg = H.factorize(X, _params(op))
    for nrhs in (1, 3, 8):
        for rep in range(4):
            b = torch.tensor(W.gaussian_rhs(n, nrhs, 100 * nrhs + rep), device="cuda")
            xe = fg.solve(b.clone())
            xg = fg.solve_repeated(b.clone())
            torch.cuda.synchronize()
            assert torch.equal(xe, xg), (nrhs, rep)
            fg.matvec(xg)  # eager work between replays
