"""Plain FP64 CPU oracle of the H^2-ULV factorization without trailing
sub-matrix dependencies (Ma, Deshmukh, Yokota; arXiv 2208.10907).

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this module.  The product path
(the HIP library) never calls it, and the two share no code: the only common
module is ``workloads`` (seeded point clouds and right-hand sides).

The oracle is deliberately plain: NumPy/SciPy in float64, one box at a time,
steps in the order the paper gives them.  LAPACK routines serve as single steps
(dgetrf/dgetrs for block LU, dgeqp3 for the column-pivoted QR, dgeqrf/dorgqr
for the orthogonal complement).

Method map (paper section / equation):
  tree + admissibility ........ Sec. I (strong admissibility), Sec. III-D (binary tree)
  dense / low-rank blocks ..... Sec. II-D: dense blocks only for inadmissible pairs
  fill-in pre-computation ..... Sec. III-B, Fig. "fill-in"
  shared basis [F A] .......... Sec. III-C, Eq. (fillu)/(fillv)
  QR / ID, skeleton split ..... Sec. II-A, Eq. (u)/(v)
  USV rotation ................ Sec. II-B, Eq. (rs) (dense) and Eq. (ss) (low-rank)
  RR elimination .............. Sec. II-B, Eq. (lu) and the two triangular solves
  Schur update of SS .......... Sec. II-B, the S^SS update equation
  merge into parent ........... Sec. II-C, the 2x2 merge of S^SS blocks
  root LU ..................... Sec. II-B, Eq. (BLR2final)
  solve ....................... Sec. II-B, the three-step forward/backward solve

Readings where the paper is silent (each is listed in the design notes):
  * kernel 1/r (Laplace) or exp(-alpha r)/r (Yukawa), diagonal entry ``diag``;
  * k-d tree: split along the widest bounding-box axis (lowest axis on ties),
    stable sort by (coordinate, original index), left child gets floor(n/2);
    L = smallest integer with leaf * 2^L >= N; or (partition="kmeans") a
    balanced 2-means bisection of every box (Sec. V);
  * admissible iff |c_i - c_j| > eta (r_i + r_j), centre = bounding-box
    midpoint, radius = half the bounding-box diagonal;
  * fill-in F_ij = sum over k in Near(i) cap Near(j), k not in {i,j}, of
    D_ik D_kk^-1 D_kj, into every reachable (i,j) (diagonal included);
  * the shared basis comes from a row interpolative decomposition of
    M'_i = [K(P_i, far) | T^-1 F_i+] (pivoted QR of M'^T), made orthogonal
    by a Householder QR of W = T W'; U = [U^S U^R] (skeleton columns first);
  * rank k = number of leading pivots with |R_tt| > tol |R_00|, capped (a
    configuration without a cap takes leaf/2: the rank stays independent of N,
    which the linear cost of Sec. I / IV-A presumes);
  * fill_in=False is the ablation without fill-ins in the basis (F = 0);
  * off-diagonal dense blocks keep only their S^SS quadrant after rotation;
  * symmetric kernels: V = U.  Nonsymmetric matrices (the advection-diffusion
    kernel exp(b.(x - y) - alpha r)/r, or bases="separate") take separate
    row and column bases (Eq. fillu/fillv): the column basis of box j is the
    row basis of A^T, whose fill-ins are F_ji^T; both interpolative
    decompositions of a box keep the same number of pivots,
    k = min(max(k_row, k_col), steps_row, steps_col), so that the redundant
    block S^RR stays square.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .rank_model import (STREAM_FAR, STREAM_FILL, forward as mlp_forward, point_rows,
                         predicted_rank, sketch_size)

# status codes (identical numbering to the C-ABI)
OK = 0
ERR_INVALID_ARG = -1
ERR_OOM = -2
ERR_HIP = -3
ERR_SINGULAR = -4
ERR_DUPLICATE_POINTS = -5
ERR_NOT_CONVERGED = -6
ERR_RANK_CHECK = -7

LAPLACE = 0
YUKAWA = 1
ADVECTION = 2   # exp(b.(x_i - x_j) - alpha r) / r: nonsymmetric for b != 0


class OracleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


@dataclass
class Params:
    kernel: int = LAPLACE
    alpha: float = 0.0
    diag: float = 1e3
    eta: float = 1.0
    leaf: int = 64
    tol: float = 1e-8
    rank_cap: int = 0          # 0 = no cap
    far_sample: int = 32       # 0 = exact far field, s > 0 = sampled
    rank_model: object = None  # MLP parameters (float32 array) or None
    sketch_seed: int = 0       # key of the Gaussian sketches
    oversample: int = 8        # sketch columns beyond 1.25 x the predicted rank
    fill_in: bool = True       # False: ablation, bases from the far field alone (F = 0)
    partition: str = "kd"      # "kd" median split of the widest axis, "kmeans" 2-means
    structure: str = "h2"      # "h2" the hierarchy; "blr2" one level of leaves (Sec. II-B)
    drift: tuple = (0.0, 0.0, 0.0)  # b of the advection-diffusion kernel
    bases: str = "auto"        # "auto": V = U for symmetric kernels; "separate": always U, V
    sketch_fallback: bool = True  # False: a sketch still rejected after its full-width
                                  # retry (if any) stops with ERR_RANK_CHECK
    sketch_min_level: int = 0  # levels above this one (lev < it) keep the full pivoted QR


def two_sided(p: Params) -> bool:
    """Separate row and column bases (Eq. fillu and fillv)."""
    return p.bases == "separate" or p.kernel == ADVECTION


def params_from_problem(prob, **kw) -> Params:
    return Params(prob.kernel, prob.alpha, prob.diag, prob.eta, prob.leaf,
                  prob.tol, prob.rank_cap, prob.far_sample, **kw)


def check_params(X: np.ndarray, p: Params) -> None:
    if X.ndim != 2 or X.shape[1] != 3 or X.shape[0] < 1:
        raise OracleError(ERR_INVALID_ARG, "points must be N x 3, N >= 1")
    if not np.all(np.isfinite(X)):
        raise OracleError(ERR_INVALID_ARG, "non-finite point coordinate")
    if p.leaf < 2 or p.eta < 0 or not math.isfinite(p.eta):
        raise OracleError(ERR_INVALID_ARG, "leaf >= 2 and eta >= 0 required")
    if p.tol < 0 or not math.isfinite(p.tol) or p.rank_cap < 0 or p.far_sample < 0:
        raise OracleError(ERR_INVALID_ARG, "tol, rank_cap, far_sample must be >= 0")
    if p.kernel not in (LAPLACE, YUKAWA, ADVECTION) or not math.isfinite(p.diag):
        raise OracleError(ERR_INVALID_ARG, "unknown kernel or bad diagonal")
    if len(p.drift) != 3 or not all(math.isfinite(float(v)) for v in p.drift):
        raise OracleError(ERR_INVALID_ARG, "drift must be three finite numbers")
    if p.kernel == ADVECTION and not math.sqrt(sum(float(v) ** 2 for v in p.drift)) <= p.alpha:
        # decay in every direction: b.(x - y) <= |b| r <= alpha r
        raise OracleError(ERR_INVALID_ARG, "the advection kernel needs alpha >= |drift|")
    if p.bases not in ("auto", "separate"):
        raise OracleError(ERR_INVALID_ARG, "bases must be auto or separate")
    if two_sided(p) and (p.rank_model is not None or p.structure != "h2"):
        raise OracleError(ERR_INVALID_ARG, "separate bases need structure h2 and no rank model")
    if p.oversample < 0:
        raise OracleError(ERR_INVALID_ARG, "oversample must be >= 0")
    if p.sketch_min_level < 0:
        raise OracleError(ERR_INVALID_ARG, "sketch_min_level must be >= 0")
    if p.structure not in ("h2", "blr2"):
        raise OracleError(ERR_INVALID_ARG, "structure must be h2 or blr2")
    if p.partition not in ("kd", "kmeans"):
        raise OracleError(ERR_INVALID_ARG, "partition must be kd or kmeans")
    if not p.fill_in and p.rank_model is not None:
        raise OracleError(ERR_INVALID_ARG, "fill_in = False is not combined with a rank model")


# ---------------------------------------------------------------------------
# Kernel matrix (Sec. IV: Laplace Green's function; Sec. V: Yukawa potential)
# ---------------------------------------------------------------------------
def kernel_block(X: np.ndarray, rows: np.ndarray, cols: np.ndarray, p: Params) -> np.ndarray:
    """K(X[rows], X[cols]); entry = diag where the row and column are the same
    point, kernel(|x_i - x_j|) otherwise.  Coincident distinct points raise
    DUPLICATE_POINTS."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.size == 0 or cols.size == 0:
        return np.zeros((rows.size, cols.size))
    xr, xc = X[rows], X[cols]
    r2 = np.zeros((rows.size, cols.size))
    for c in range(3):
        d = xr[:, c][:, None] - xc[:, c][None, :]
        r2 += d * d
    r = np.sqrt(r2)
    same = rows[:, None] == cols[None, :]
    if np.any((r == 0.0) & ~same):
        raise OracleError(ERR_DUPLICATE_POINTS, "two distinct points coincide")
    rs = np.where(same, 1.0, r)
    if p.kernel == LAPLACE:
        K = 1.0 / rs
    elif p.kernel == YUKAWA:
        K = np.exp(-p.alpha * rs) / rs
    else:
        # b.(x_row - x_col): the drift term that makes K(x, y) != K(y, x)
        bd = np.zeros((rows.size, cols.size))
        for c in range(3):
            bd += float(p.drift[c]) * (xr[:, c][:, None] - xc[:, c][None, :])
        K = np.exp(bd - p.alpha * rs) / rs
    return np.where(same, p.diag, K)


def dense_matrix(X: np.ndarray, p: Params) -> np.ndarray:
    idx = np.arange(X.shape[0])
    return kernel_block(X, idx, idx, p)


def matvec_exact(X: np.ndarray, x: np.ndarray, p: Params, chunk: int = 1024) -> np.ndarray:
    """y = A x with A generated on the fly: y_i = diag x_i + sum_{j != i} K(r_ij) x_j."""
    n = X.shape[0]
    x2 = x.reshape(n, -1)
    y = np.zeros_like(x2, dtype=np.float64)
    cols = np.arange(n)
    for s in range(0, n, chunk):
        rows = np.arange(s, min(n, s + chunk))
        y[rows] = kernel_block(X, rows, cols, p) @ x2
    return y.reshape(x.shape)


# ---------------------------------------------------------------------------
# Cluster tree (Sec. III-D: full binary tree over the point set)
# ---------------------------------------------------------------------------
@dataclass
class Tree:
    L: int
    perm: np.ndarray                 # tree position -> original point index
    start: list                      # start[l][i]
    end: list
    centre: list                     # centre[l]: (2^l, 3)
    radius: list                     # radius[l]: (2^l,)


def tree_depth(n: int, leaf: int) -> int:
    L = 0
    while leaf * (1 << L) < n:
        L += 1
    return L


def _seq_mean(X: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Mean of the points idx (ascending index order), each coordinate summed
    one point after another (a running sum), then divided by the count."""
    ids = np.sort(idx)
    return np.array([np.cumsum(X[ids, c])[-1] for c in range(3)]) / float(ids.size)


def kmeans_split(X: np.ndarray, pts: np.ndarray, axis: int) -> np.ndarray:
    """Balanced 2-means bisection of a box (Sec. V: k-means clusters with a
    power-of-two count).  Start from the k-d split along `axis`; then at most 10
    Lloyd steps: centroids of the two clusters, each point keyed by
    |x - c0|^2 - |x - c1|^2, the floor(n/2) smallest keys (ties: lower index)
    form cluster 0; stop once cluster 0 repeats.  Returns the points in the
    last (key, index) order."""
    n = pts.size
    half = n // 2
    order = pts[np.lexsort((pts, X[pts, axis]))]
    c0 = np.sort(order[:half])
    for _ in range(10):
        m0 = _seq_mean(X, c0)
        m1 = _seq_mean(X, order[half:])
        a = X[order] - m0
        b = X[order] - m1
        d0 = a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1] + a[:, 2] * a[:, 2]
        d1 = b[:, 0] * b[:, 0] + b[:, 1] * b[:, 1] + b[:, 2] * b[:, 2]
        order = order[np.lexsort((order, d0 - d1))]
        new0 = np.sort(order[:half])
        done = np.array_equal(new0, c0)
        c0 = new0
        if done:
            break
    return order


def build_tree(X: np.ndarray, leaf: int, partition: str = "kd") -> Tree:
    n = X.shape[0]
    L = tree_depth(n, leaf)
    perm = np.arange(n, dtype=np.int64)
    start, end, centre, radius = [], [], [], []
    ranges = [(0, n)]
    for lev in range(L + 1):
        st = np.array([a for a, _ in ranges], dtype=np.int64)
        en = np.array([b for _, b in ranges], dtype=np.int64)
        cen = np.zeros((len(ranges), 3))
        rad = np.zeros(len(ranges))
        nxt = []
        for bi, (a, b) in enumerate(ranges):
            pts = perm[a:b]
            lo = X[pts].min(axis=0)
            hi = X[pts].max(axis=0)
            cen[bi] = 0.5 * (lo + hi)
            d = hi - lo
            rad[bi] = 0.5 * math.sqrt(float(d[0]) * d[0] + float(d[1]) * d[1] + float(d[2]) * d[2])
            if lev < L:
                axis = int(np.argmax(hi - lo))
                if partition == "kmeans" and b - a >= 2:
                    perm[a:b] = kmeans_split(X, pts, axis)
                else:
                    order = np.lexsort((pts, X[pts, axis]))
                    perm[a:b] = pts[order]
                mid = a + (b - a) // 2
                nxt += [(a, mid), (mid, b)]
        start.append(st)
        end.append(en)
        centre.append(cen)
        radius.append(rad)
        ranges = nxt
    return Tree(L, perm, start, end, centre, radius)


# ---------------------------------------------------------------------------
# Near / far lists (strong admissibility, Sec. I and II-D)
# ---------------------------------------------------------------------------
def build_lists(tree: Tree, eta: float):
    near = [[[0]]]
    far = [[[]]]
    for lev in range(1, tree.L + 1):
        nb = 1 << lev
        nl = [[] for _ in range(nb)]
        fl = [[] for _ in range(nb)]
        c, r = tree.centre[lev], tree.radius[lev]
        for pbox in range(nb // 2):
            for q in near[lev - 1][pbox]:
                for i in (2 * pbox, 2 * pbox + 1):
                    for j in (2 * q, 2 * q + 1):
                        d = c[i] - c[j]
                        dist = math.sqrt(float(d[0]) * d[0] + float(d[1]) * d[1] + float(d[2]) * d[2])
                        if dist > eta * (float(r[i]) + float(r[j])):
                            fl[i].append(j)
                        else:
                            nl[i].append(j)
        near.append([sorted(x) for x in nl])
        far.append([sorted(x) for x in fl])
    return near, far


def build_flat_lists(tree: Tree, eta: float):
    """Lists of the flat BLR^2 structure (Sec. II-B): one level of boxes, the
    leaves of the tree, every pair classified directly by the admissibility
    rule (no hierarchy).  Returned in the per-level layout of build_lists, with
    only the leaf level filled in."""
    L = tree.L
    nb = 1 << L
    c, r = tree.centre[L], tree.radius[L]
    nl = [[] for _ in range(nb)]
    fl = [[] for _ in range(nb)]
    for i in range(nb):
        for j in range(nb):
            d = c[i] - c[j]
            dist = math.sqrt(float(d[0]) * d[0] + float(d[1]) * d[1] + float(d[2]) * d[2])
            (fl if dist > eta * (float(r[i]) + float(r[j])) else nl)[i].append(j)
    near = [[[0]]] + [[[] for _ in range(1 << lev)] for lev in range(1, L)] + [nl]
    far = [[[]]] + [[[] for _ in range(1 << lev)] for lev in range(1, L)] + [fl]
    return near, far


def fill_targets(near_l, i: int):
    """Column boxes j that receive a fill-in in block row i: every j that shares a
    near box k (k != i, k != j) with i.  Sorted ascending; includes i itself when
    i has a near neighbour."""
    js = set()
    for k in near_l[i]:
        if k == i:
            continue
        for j in near_l[k]:
            if j != k:
                js.add(j)
    return sorted(js)


def box_points(tree: Tree, lev: int, q: int) -> np.ndarray:
    return tree.perm[tree.start[lev][q]:tree.end[lev][q]]


def far_columns(tree: Tree, near, far, lev: int, i: int, P, s: int) -> np.ndarray:
    """Point indices that represent the far field of box i at level lev.
    s == 0: every point outside the near boxes of i (the literal A_{i,+}).
    s > 0: candidate rows P[lev][q] of every q in Far_lev(i), then for each
    ancestor level (nearest first) and each of its far boxes, all points if the
    box holds at most s points, else s evenly strided points."""
    if s == 0:
        mask = np.ones(tree.perm.size, dtype=bool)
        for j in near[lev][i]:
            mask[tree.start[lev][j]:tree.end[lev][j]] = False
        return tree.perm[mask]
    parts = [np.asarray(P[lev][q], dtype=np.int64) for q in far[lev][i]]
    a = i
    for la in range(lev - 1, 0, -1):
        a >>= 1
        for q in far[la][a]:
            pts = box_points(tree, la, q)
            nq = pts.size
            if nq <= s:
                parts.append(pts)
            else:
                t = np.arange(s)
                parts.append(pts[((t + 0.5) * nq / s).astype(np.int64)])
    if not parts:
        return np.zeros(0, dtype=np.int64)
    return np.concatenate(parts)


# ---------------------------------------------------------------------------
# Row interpolative decomposition and orthogonal complement
# (Sec. II-A Eq. (u): column-pivoted QR, Q kept; ID allowed; Sec. III-C)
# ---------------------------------------------------------------------------
def pivoted_qr(M: np.ndarray):
    """Column-pivoted Householder QR of M^T (LAPACK dgeqp3): M^T Pi = Q R.
    Returns (piv, R (steps x m), |diag R|), steps = min(m, n)."""
    m, n = M.shape
    qr, jpvt, tau, work, info = sla.lapack.dgeqp3(np.asfortranarray(M.T.copy()))
    piv = np.asarray(jpvt, dtype=np.int64) - 1
    steps = min(m, n)
    R = np.triu(qr[:steps, :])
    return piv, R, np.abs(np.diag(R))


def id_matrix(piv, R, m: int, k: int) -> np.ndarray:
    """W' (m x k) of the row ID that keeps the first k pivots: the identity on
    rows piv[:k], (R11^-1 R12)^T on rows piv[k:]."""
    Wp = np.zeros((m, k))
    if k > 0:
        Wp[piv[:k], np.arange(k)] = 1.0
        if k < m:
            E = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
            Wp[piv[k:], :] = E.T
    return Wp


def id_rank(dg, tol: float, cap: int, m: int, n: int) -> int:
    """Leading pivots with |R_tt| > tol |R_00|, at most the cap and min(m, n)."""
    steps = min(m, n)
    k = 0
    if steps > 0 and dg[0] > 0:
        thr = tol * dg[0]
        while k < steps and dg[k] > thr:
            k += 1
    cap_eff = steps if cap <= 0 else min(cap, steps)
    return min(k, cap_eff)


def row_id(M: np.ndarray, tol: float, cap: int):
    """Row ID of M (m x n): M ~= W' M[piv[:k], :].

    Column-pivoted Householder QR of M^T (LAPACK dgeqp3): M^T Pi = Q R.
    k = number of leading t with |R_tt| > tol |R_00| (then capped).
    W' has the identity on rows piv[:k] and (R11^-1 R12)^T on rows piv[k:].
    Returns (k, piv, Wp, absdiag)."""
    m, n = M.shape
    if m == 0:
        return 0, np.zeros(0, dtype=np.int64), np.zeros((0, 0)), np.zeros(0)
    if n == 0:
        return 0, np.arange(m), np.zeros((m, 0)), np.zeros(0)
    piv, R, dg = pivoted_qr(M)
    k = id_rank(dg, tol, cap, m, n)
    return k, piv, id_matrix(piv, R, m, k), dg


def complement_basis(W: np.ndarray):
    """Householder QR of W (m x k), LAPACK convention: W = Q [T; 0].
    Returns U = Q (m x m, orthogonal, skeleton columns first) and T (k x k)."""
    m, k = W.shape
    if k == 0:
        return np.eye(m), np.zeros((0, 0))
    Q, Rw = np.linalg.qr(W, mode="complete")
    return Q, Rw[:k, :k]


# ---------------------------------------------------------------------------
# Learned-rank variant of the basis step: box features, and the row ID taken
# from a Gaussian sketch of M' sized by the predicted rank, accepted or
# rejected by a randomized probe of its error (falls back to the full pivoted QR).
# ---------------------------------------------------------------------------
SKETCH_PROBES = 8       # probe columns of the error check
SKETCH_SLACK = 10.0     # allowed factor over the pivoted-QR error bound


def box_features(X, tree: Tree, near, far, lev: int, i: int, m: int, ntargets: int,
                 ncols: int, p: Params, child_ratio: float) -> np.ndarray:
    """The 16 rank-model features of box i at level lev (float32):
      0 log2(1+m)/12          candidate rows
      1 log2(1+n_pts)/20      points of the box's subtree
      2 lev / L
      3 log2(1+|Near|)/6,  4 log2(1+|Far|)/6,  5 log2(1+|fill targets|)/8
      6 log2(1+ncols)/20      columns of M'
      7 -log10(tol)/16        (1 for tol = 0)
      8 alpha r (Yukawa), else 0
      9-11 sqrt of the covariance eigenvalues of the box's points (descending) / r
      12 log2(max(r / r_root, 2^-30))/16   (0 when r_root = 0)
      13 children's compression (k_c1 + k_c2)/(m_c1 + m_c2) above the leaves, 1 at the leaves
      14 1 at the leaves, else 0
      15 eta / 2
    r is the box radius (half the bounding-box diagonal)."""
    pts = X[box_points(tree, lev, i)]
    n = pts.shape[0]
    mu = pts.mean(axis=0)
    dev = pts - mu
    C = dev.T @ dev / n
    lam = np.sort(np.clip(np.linalg.eigvalsh(C), 0.0, None))[::-1]
    r = float(tree.radius[lev][i])
    r0 = float(tree.radius[0][0])
    f = np.zeros(16)
    f[0] = math.log2(1 + m) / 12
    f[1] = math.log2(1 + n) / 20
    f[2] = lev / max(tree.L, 1)
    f[3] = math.log2(1 + len(near[lev][i])) / 6
    f[4] = math.log2(1 + len(far[lev][i])) / 6
    f[5] = math.log2(1 + ntargets) / 8
    f[6] = math.log2(1 + ncols) / 20
    f[7] = -math.log10(p.tol) / 16 if p.tol > 0 else 1.0
    f[8] = p.alpha * r if p.kernel == YUKAWA else 0.0
    if r > 0:
        f[9:12] = np.sqrt(lam) / r
    f[12] = math.log2(max(r / r0, 2.0 ** -30)) / 16 if r0 > 0 else 0.0
    f[13] = child_ratio
    f[14] = 1.0 if lev == tree.L else 0.0
    f[15] = p.eta / 2
    return f.astype(np.float32)


def sketch_matrix(p: Params, lev: int, fcols, targets, P, npts: int, cols: int) -> np.ndarray:
    """Omega of one box (columns of M' x cols): the far-stream rows of its far-field
    points, then the fill-stream rows of the candidate points of every fill target
    (the order of M''s columns)."""
    parts = [point_rows(p.sketch_seed, lev, STREAM_FAR, fcols, npts, cols)]
    for j in targets:
        parts.append(point_rows(p.sketch_seed, lev, STREAM_FILL, P[lev][j], npts, cols))
    return np.concatenate(parts, axis=0)


def sketch_row_id(M: np.ndarray, ell: int, tol: float, cap_eff: int, Om: np.ndarray,
                  rank_cap: int = 0):
    """Row ID of M (m x n) from Y = M Omega, Omega (n x (ell + q)) Gaussian with
    rows keyed by point: column-pivoted QR of the first ell columns of Y (as rows of
    Y^T), k = leading pivots with |R_tt| > tol |R_00| (at most cap_eff and ell).
    The last q columns G of Omega probe the error: with Z = M G,
      res = Z[piv[k:]] - E^T Z[piv[:k]],  E = R11^-1 R12,
    and the result is accepted iff k < ell (the sketch was not exhausted) and
      ||res||_F <= SLACK sqrt(m - k) tol max_j ||Z[j]||,
    the pivoted-QR bound ||M - W' M[sk]||_F <= sqrt(m - k) tol |R_00| with the
    row norms of M estimated by those of Z.  When the rank cap ends the pivot loop
    (k == rank_cap) the full pivoted QR misses tol as well; the sketch is then
    accepted without the tol test if it keeps at least q columns of oversampling
    beyond k (ell - k >= q), the randomized ID's usual margin.
    Returns (accepted, k, piv, Wp, absdiag)."""
    m, n = M.shape
    Yt = Om[:, :ell + SKETCH_PROBES].T @ M.T
    Ys, Zt = Yt[:ell], Yt[ell:]
    qr, jpvt, tau, work, info = sla.lapack.dgeqp3(np.asfortranarray(Ys.copy()))
    piv = np.asarray(jpvt, dtype=np.int64) - 1
    steps = min(ell, m)
    R = np.triu(qr[:steps, :])
    dg = np.abs(np.diag(R))
    k = 0
    if steps > 0 and dg[0] > 0:
        thr = tol * dg[0]
        while k < steps and dg[k] > thr:
            k += 1
    k = min(k, cap_eff, ell)
    E = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False) if k else np.zeros((0, m))
    res = Zt[:, piv[k:]] - Zt[:, piv[:k]] @ E
    zmax = float(np.max(np.linalg.norm(Zt, axis=0))) if m else 0.0
    capped = rank_cap > 0 and k == rank_cap and ell - k >= SKETCH_PROBES
    ok = k < ell and (capped or
                      float(np.linalg.norm(res)) <= SKETCH_SLACK * math.sqrt(m - k) * tol * zmax)
    Wp = np.zeros((m, k))
    if k > 0:
        Wp[piv[:k], np.arange(k)] = 1.0
        if k < m:
            Wp[piv[k:], :] = E.T
    return ok, k, piv, Wp, dg


# ---------------------------------------------------------------------------
# Block LU helpers (Sec. II-B Eq. (lu); partial pivoting, LAPACK dgetrf)
# ---------------------------------------------------------------------------
def lu(A: np.ndarray):
    if A.shape[0] == 0:
        return (A.copy(), np.zeros(0, dtype=np.int32))
    lu_, piv = sla.lu_factor(A, check_finite=False)
    d = np.diag(lu_)
    if np.any(d == 0) or not np.all(np.isfinite(lu_)):
        raise OracleError(ERR_SINGULAR, "zero or non-finite pivot")
    return lu_, piv


def apply_pinv(piv, B):
    """P^T B for LAPACK row interchanges (sequential swaps)."""
    B = np.array(B, dtype=np.float64, copy=True)
    for t, pt in enumerate(piv):
        if pt != t:
            B[[t, pt]] = B[[pt, t]]
    return B


def lower_solve(lu_, B):
    return sla.solve_triangular(lu_, B, lower=True, unit_diagonal=True, check_finite=False)


def upper_solve(lu_, B):
    return sla.solve_triangular(lu_, B, lower=False, check_finite=False)


# ---------------------------------------------------------------------------
# Factorization
# ---------------------------------------------------------------------------
@dataclass
class BoxFactor:
    m: int
    k: int
    U: np.ndarray          # m x m, [U^S U^R]
    T: np.ndarray          # k x k
    sk: np.ndarray         # skeleton point indices (pivot order)
    piv: np.ndarray        # row-ID pivots (indices into the box's candidate rows)
    lu: np.ndarray = None  # LU of S^RR (r x r)
    lupiv: np.ndarray = None
    URS: np.ndarray = None  # L^-1 P^T S^RS   (r x k)
    LSR: np.ndarray = None  # S^SR U^-1       (k x r)
    absdiag: np.ndarray = None
    feat: np.ndarray = None  # rank-model features (float32, 16)
    khat: int = -1           # predicted rank (-1: no model)
    ell: int = 0             # sketch columns (0: full pivoted QR)
    sketch: int = 0          # 0 not sketched, 1 sketch accepted, 2 fell back to the
                             # full QR, 3 accepted on the full-width retry
    # separate column basis (nonsymmetric matrices; None: V = U)
    V: np.ndarray = None     # m x m, [V^S V^R]
    TV: np.ndarray = None    # k x k
    skV: np.ndarray = None   # column skeleton point indices (pivot order)
    pivV: np.ndarray = None
    absdiagV: np.ndarray = None


def right_basis(f: BoxFactor) -> np.ndarray:
    """The column basis [V^S V^R] of a box (U itself for shared bases)."""
    return f.U if f.V is None else f.V


@dataclass
class Factor:
    X: np.ndarray
    params: Params
    tree: Tree
    near: list
    far: list
    levels: dict = field(default_factory=dict)   # lev -> list[BoxFactor]
    cand: dict = field(default_factory=dict)     # lev -> list of candidate point arrays
    cand_col: dict = field(default_factory=dict) # lev -> column candidates (separate bases)
    root_lu: tuple = None
    m_root: int = 0
    stats: dict = field(default_factory=dict)


def _offdiag_dropped(U_i, D, U_j, k_i, k_j):
    """Norm of the dropped (non-SS) quadrants of a rotated off-diagonal block."""
    S = U_i.T @ D @ U_j
    tot = np.linalg.norm(D)
    S[:k_i, :k_j] = 0.0
    return np.linalg.norm(S), tot


def factorize(X: np.ndarray, p: Params, diagnostics: bool = False,
              level_stop: int | None = None, boxes: set | None = None) -> Factor:
    """H^2-ULV factorization without trailing sub-matrix dependencies.

    Level loop from the leaves up (Sec. III-B..III-C, then Sec. II-B/II-C):
      (a) dense blocks D_ij for j in Near(i)      (leaf: kernel; upper: merged S)
      (b) fill-ins F_ij = sum_k D_ik D_kk^-1 D_kj  (Sec. III-B)
      (c) shared basis from [K(P_i, far) | T^-1 F_i+] by row ID + QR (Eq. fillu)
      (d) low-rank couplings S^SS_ij = T_i K(sk_i, sk_j) T_j^T   (Eq. ss)
      (e) rotation S_ii = U_i^T D_ii U_i, near S^SS_ij = U^S_i^T D_ij U^S_j (Eq. rs)
      (f) LU of S^RR, triangular solves, Schur update of S^SS    (Eq. lu ff.)
      merge children's S^SS into the parent's dense blocks       (Sec. II-C)
    then the root LU (Eq. BLR2final).  With ``structure="blr2"`` (the flat BLR^2
    of Sec. II-B) only the leaf level is factorized, with lists that classify
    every pair of leaves directly, and the root is the dense block of all leaves'
    S^SS blocks (Eq. BLR2final).

    ``level_stop``/``boxes``: stop after the basis step of that level, for the
    given boxes only (used to time or check a sample of one level).

    Flop counts (``stats["flops"]``) follow the operations a device forms:
    LU 2/3 m^3 per diagonal block; for a box whose M' is formed, the products
    D_ik D_kk^-1 (2 m_i m_k^2 each) and the fill-ins (2 m_i m_k m_j per term);
    for a sketched box, per attempt the far part 2 |far| m_i c and the fill part
    2 c m_k m_i per near k, plus per pass the shared Q'_k (2 m_k^2 C + 2 m_k m_j C);
    QR 2 n m^2 - 2/3 m^3; GEMM 2 m n k."""
    X = np.asarray(X, dtype=np.float64)
    check_params(X, p)
    tree = build_tree(X, p.leaf, p.partition)
    flat = p.structure == "blr2"
    near, far = build_flat_lists(tree, p.eta) if flat else build_lists(tree, p.eta)
    fac = Factor(X, p, tree, near, far)
    L = tree.L
    flops = {"fill": 0.0, "basis": 0.0, "rotate": 0.0, "couple": 0.0, "elim": 0.0, "root": 0.0}
    dropped = []
    kevals = 0

    if L == 0:
        idx = tree.perm.copy()
        D0 = kernel_block(X, idx, idx, p)
        fac.root_lu = lu(D0)
        fac.m_root = D0.shape[0]
        flops["root"] += 2.0 / 3.0 * fac.m_root ** 3
        fac.stats = {"flops": flops, "kevals": D0.size}
        return fac
    if two_sided(p):
        return _factorize_two_sided(fac, flops)

    # candidate rows and T-hat blocks of the current level
    P = {L: [box_points(tree, L, i) for i in range(1 << L)]}
    prev_bf = None
    That = None                    # per box: list of triangular blocks (upper levels)
    Sblk = None                    # previous level's S^SS blocks: dict (c, d) -> array
    for lev in range(L, (L - 1) if flat else 0, -1):
        nb = 1 << lev
        Pl = P[lev]
        m = [len(Pl[i]) for i in range(nb)]
        # rows needed when only a sample of boxes of the stopping level is wanted:
        # the sample, their near boxes (whose LU and solves feed the fill-ins)
        need = None
        if level_stop is not None and lev == level_stop and boxes is not None:
            need = set(boxes)
            for i in boxes:
                need.update(near[lev][i])
        # (a) dense blocks
        D = {}
        for i in range(nb):
            if need is not None and i not in need:
                continue
            for j in near[lev][i]:
                if lev == L:
                    D[i, j] = kernel_block(X, Pl[i], Pl[j], p)
                    kevals += m[i] * m[j]
                else:
                    c1, c2 = 2 * i, 2 * i + 1
                    d1, d2 = 2 * j, 2 * j + 1
                    D[i, j] = np.block([[Sblk[c1, d1], Sblk[c1, d2]],
                                        [Sblk[c2, d1], Sblk[c2, d2]]])
        # (b) fill-ins: one LU per diagonal block, one solve per near block
        dlu = {}
        Y = {}
        for k in range(nb):
            # the ablation without fill-ins in the basis has no fill-in step
            if not p.fill_in or m[k] == 0 or (need is not None and k not in need):
                continue
            dlu[k] = lu(D[k, k])
            flops["fill"] += 2.0 / 3.0 * m[k] ** 3
            # Y_kj = D_kk^-1 D_kj; the flops are counted per box below as the
            # products D_ik D_kk^-1 of the boxes whose M' is formed
            for j in near[lev][k]:
                if j != k:
                    Y[k, j] = sla.lu_solve(dlu[k], D[k, j], check_finite=False)
        fac.cand[lev] = Pl
        bf = [None] * nb
        first_attempts, retries = [], []
        todo = range(nb) if (level_stop is None or lev != level_stop or boxes is None) else sorted(boxes)
        for i in todo:
            # F_ij for every reachable j (its flops are counted below, unless the
            # basis comes from a sketch, which forms M' Omega without F)
            Fcols = []
            fl_F = 0.0
            # without fill-ins in the basis (the ablation) no block receives one
            targets = fill_targets(near[lev], i) if p.fill_in else []
            for j in targets:
                F = np.zeros((m[i], m[j]))
                for k in near[lev][i]:
                    # an empty box (both children fully eliminated) has no blocks
                    if k == i or k == j or m[k] == 0 or j not in near[lev][k]:
                        continue
                    F += D[i, k] @ Y[k, j]
                    fl_F += 2.0 * m[i] * m[k] * m[j]
                Fcols.append(F)
            Fi = np.concatenate(Fcols, axis=1) if Fcols else np.zeros((m[i], 0))
            if lev < L and m[i] > 0:
                # map fill-ins to point-row coordinates: T-hat^-1 F
                Fi = Fi.copy()
                off = 0
                for Tc in That[i]:
                    kc = Tc.shape[0]
                    if kc:
                        Fi[off:off + kc] = sla.solve_triangular(Tc, Fi[off:off + kc], lower=False)
                    off += kc
            fcols = far_columns(tree, near, far, lev, i, P, p.far_sample)
            Kf = kernel_block(X, Pl[i], fcols, p)
            kevals += Kf.size
            M = np.concatenate([Kf, Fi], axis=1)
            ncol = M.shape[1]
            # (c) row ID + orthogonal complement; with a rank model, the row ID of
            # a Gaussian sketch sized by the predicted rank when it is accepted
            if lev == L:
                ratio = 1.0
            else:
                c1, c2 = prev_bf[2 * i], prev_bf[2 * i + 1]
                ratio = (c1.k + c2.k) / (c1.m + c2.m) if c1.m + c2.m > 0 else 0.0
            feat = box_features(X, tree, near, far, lev, i, m[i], len(targets), ncol, p, ratio)
            khat, ell, state = -1, 0, 0

            def attempt(width):
                # M' Omega as formed without F: the far part K(P_i, far) Omega_far
                # (basis) and the fill part T-hat^-1 sum_k D_ik Q'_k (fill; the
                # Q'_k are shared by the level and counted after the loop)
                cols = width + SKETCH_PROBES
                flops["basis"] += 2.0 * len(fcols) * m[i] * cols
                for k in near[lev][i]:
                    if k != i and m[k] > 0:
                        flops["fill"] += 2.0 * cols * m[k] * m[i]
                Om = sketch_matrix(p, lev, fcols, targets, P, X.shape[0], cols)
                return sketch_row_id(M, width, p.tol, cap_eff, Om, p.rank_cap)

            if p.rank_model is not None:
                y = mlp_forward(np.asarray(p.rank_model, dtype=np.float32), feat[None, :],
                                dtype=np.float32)[0][0]
                khat = predicted_rank(y)
                # the sketch never exceeds m - probes columns: a box whose
                # predicted rank leaves no room (k-hat >= m - probes included) is
                # still sketched at full width, accepted when its rank is below it;
                # with a rank cap the sketch is sized for min(k-hat, cap)
                kh = min(khat, p.rank_cap) if p.rank_cap > 0 else khat
                ell = min(sketch_size(kh, p.oversample), m[i] - SKETCH_PROBES)
                if 0 < ell < ncol and lev >= p.sketch_min_level:
                    cap_eff = min(m[i], ncol) if p.rank_cap <= 0 else min(p.rank_cap, m[i], ncol)
                    first_attempts.append((i, ell))
                    ok, k_i, piv, Wp, dg = attempt(ell)
                    state = 1 if ok else 2
                    # a rejected sketch is retried once at full width (m - probes
                    # columns) before the full pivoted QR
                    full = m[i] - SKETCH_PROBES
                    if not ok and ell < full < ncol:
                        ell = full
                        retries.append((i, ell))
                        ok, k_i, piv, Wp, dg = attempt(ell)
                        state = 3 if ok else 2
                else:
                    ell = 0
            if state == 2 and not p.sketch_fallback:
                raise OracleError(ERR_RANK_CHECK, "a sketched row ID failed its check")
            if state not in (1, 3):
                # M' formed: the products D_ik D_kk^-1, then the fill-ins
                if p.fill_in:
                    flops["fill"] += sum(2.0 * m[i] * m[k] ** 2 for k in near[lev][i] if k != i)
                flops["fill"] += fl_F
                k_i, piv, Wp, dg = row_id(M, p.tol, p.rank_cap)
                flops["basis"] += 2.0 * ncol * m[i] ** 2 - 2.0 / 3.0 * min(ncol, m[i]) ** 3 if ncol >= m[i] else 2.0 * m[i] * ncol ** 2 - 2.0 / 3.0 * ncol ** 3
            if lev < L and m[i] > 0:
                W = np.zeros_like(Wp)
                off = 0
                for Tc in That[i]:
                    kc = Tc.shape[0]
                    W[off:off + kc] = Tc @ Wp[off:off + kc]
                    off += kc
            else:
                W = Wp
            U, T = complement_basis(W)
            flops["basis"] += 4.0 * m[i] * k_i * k_i + 4.0 * m[i] ** 2 * k_i
            bf[i] = BoxFactor(m[i], k_i, U, T, np.asarray(Pl[i])[piv[:k_i]], piv, absdiag=dg,
                              feat=feat, khat=khat, ell=ell, sketch=state)
        # shared sketch blocks Q'_k = D_kk^-1 sum_{j in Near(k), j != k} D_kj Omega_fill[P_j]
        # for every box k next to a sketched box, as wide as the widest sketch of
        # the pass (first attempts, then full-width retries)
        for att in (first_attempts, retries):
            if not att:
                continue
            cols = max(w for _, w in att) + SKETCH_PROBES
            ks = {k for i, _ in att for k in near[lev][i] if k != i and m[k] > 0}
            for k in ks:
                flops["fill"] += 2.0 * m[k] ** 2 * cols
                for j in near[lev][k]:
                    if j != k and m[j] > 0:
                        flops["fill"] += 2.0 * m[k] * m[j] * cols
        if level_stop is not None and lev == level_stop:
            fac.levels[lev] = bf
            fac.stats = {"flops": flops, "kevals": kevals}
            return fac
        # (d) low-rank couplings
        Snew = {}
        for i in range(nb):
            for j in far[lev][i]:
                Kc = kernel_block(X, bf[i].sk, bf[j].sk, p)
                kevals += Kc.size
                Snew[i, j] = bf[i].T @ Kc @ bf[j].T.T
                ki, kj = bf[i].k, bf[j].k
                flops["couple"] += 2.0 * ki * ki * kj + 2.0 * ki * kj * kj
        # (e) rotation + (f) elimination
        for i in range(nb):
            Ui, ki = bf[i].U, bf[i].k
            for j in near[lev][i]:
                if j == i:
                    continue
                Uj, kj = bf[j].U, bf[j].k
                Snew[i, j] = Ui[:, :ki].T @ D[i, j] @ Uj[:, :kj]
                # an empty S^SS block (k_i or k_j = 0) costs nothing
                if ki and kj:
                    flops["rotate"] += 2.0 * m[i] * m[j] * kj + 2.0 * ki * m[i] * kj
                if diagnostics:
                    dropped.append(_offdiag_dropped(Ui, D[i, j], Uj, ki, kj))
            S = Ui.T @ D[i, i] @ Ui
            flops["rotate"] += 4.0 * m[i] ** 3
            r = m[i] - ki
            if r > 0:
                lu_, lp = lu(S[ki:, ki:])
                URS = lower_solve(lu_, apply_pinv(lp, S[ki:, :ki]))
                # L^SR = S^SR U^-1  <=>  U^T L^SR^T = S^SR^T
                LSR = sla.solve_triangular(lu_, S[:ki, ki:].T, trans="T", lower=False,
                                           check_finite=False).T if ki else np.zeros((0, r))
                Snew[i, i] = S[:ki, :ki] - LSR @ URS
                bf[i].lu, bf[i].lupiv, bf[i].URS, bf[i].LSR = lu_, lp, URS, LSR
                flops["elim"] += 2.0 / 3.0 * r ** 3 + 2.0 * r * r * ki + 2.0 * ki * ki * r
            else:
                Snew[i, i] = S[:ki, :ki].copy()
        fac.levels[lev] = bf
        prev_bf = bf
        # merge: next level's candidate rows and T-hat
        if lev > 1 and not flat:
            P[lev - 1] = [np.concatenate([bf[2 * q].sk, bf[2 * q + 1].sk]) for q in range(nb // 2)]
            That = [[bf[2 * q].T, bf[2 * q + 1].T] for q in range(nb // 2)]
        Sblk = Snew
    # root: the two children of the root box, or (flat) every leaf
    kids = list(range(1 << L)) if flat else [0, 1]
    D0 = np.block([[Sblk[a, b] for b in kids] for a in kids])
    fac.m_root = D0.shape[0]
    fac.root_lu = lu(D0) if fac.m_root > 0 else (D0, np.zeros(0, dtype=np.int32))
    flops["root"] += 2.0 / 3.0 * fac.m_root ** 3
    fac.stats = {"flops": flops, "kevals": kevals}
    if diagnostics:
        fac.stats["dropped"] = dropped
    return fac


def _block_tri_solve(Th, F):
    """T-hat^-1 F for the block-diagonal upper-triangular T-hat (children's T)."""
    F = F.copy()
    off = 0
    for Tc in Th:
        kc = Tc.shape[0]
        if kc:
            F[off:off + kc] = sla.solve_triangular(Tc, F[off:off + kc], lower=False)
        off += kc
    return F


def _block_tri_mul(Th, Wp):
    """T-hat W' for the block-diagonal T-hat."""
    W = np.zeros_like(Wp)
    off = 0
    for Tc in Th:
        kc = Tc.shape[0]
        W[off:off + kc] = Tc @ Wp[off:off + kc]
        off += kc
    return W


def _factorize_two_sided(fac: Factor, flops: dict) -> Factor:
    """H^2-ULV with separate row and column bases (Sec. III-C, Eq. fillu and
    fillv), for matrices that are not symmetric.

    Per level, with row candidates P^U and column candidates P^V of each box:
      (a) D_ij = A(P^U_i, P^V_j) for j in Near(i) (upper levels: merged S^SS);
      (b) one LU per diagonal block; the row fill-ins F_ij = sum_k D_ik D_kk^-1 D_kj
          and, for the columns, the fill-ins of A^T, F_ji^T = sum_k D_ki^T D_kk^-T D_jk^T;
      (c) row basis of box i from [K(P^U_i, far) | T-hat_U^-1 F_i+] and column
          basis from [K(far, P^V_i)^T | T-hat_V^-1 F_+i^T]: the far-field samples
          of own-level far boxes are their candidates of the other side (the
          columns, resp. rows, of the far blocks); both pivoted QRs keep
          k = min(max(k_U, k_V), steps_U, steps_V) pivots;
      (d) S^SS_ij = T_U,i K(sk^U_i, sk^V_j) T_V,j^T for far pairs;
      (e) S_ii = U_i^T D_ii V_i, near S^SS_ij = U^S_i^T D_ij V^S_j;
      (f) LU of S^RR, triangular solves, Schur update (as for shared bases);
      parents take the children's row skeletons as row candidates and their
      column skeletons as column candidates.
    Flop counts as for shared bases, the basis step (fill products, QR, ID,
    complement) once per side; one LU per diagonal block serves both."""
    X, p, tree, near, far = fac.X, fac.params, fac.tree, fac.near, fac.far
    L = tree.L
    kevals = 0
    PU = {L: [box_points(tree, L, i) for i in range(1 << L)]}
    PV = {L: [box_points(tree, L, i) for i in range(1 << L)]}
    ThU = ThV = None
    Sblk = None
    fac.cand_col = {}
    for lev in range(L, 0, -1):
        nb = 1 << lev
        m = [len(PU[lev][i]) for i in range(nb)]
        # (a) dense blocks
        D = {}
        for i in range(nb):
            for j in near[lev][i]:
                if lev == L:
                    D[i, j] = kernel_block(X, PU[lev][i], PV[lev][j], p)
                    kevals += m[i] * m[j]
                else:
                    D[i, j] = np.block([[Sblk[2 * i, 2 * j], Sblk[2 * i, 2 * j + 1]],
                                        [Sblk[2 * i + 1, 2 * j], Sblk[2 * i + 1, 2 * j + 1]]])
        # (b) LU of the diagonal blocks; Y_kj = D_kk^-1 D_kj, Yt_kj = D_kk^-T D_jk^T
        dlu, Y, Yt = {}, {}, {}
        for k in range(nb):
            if not p.fill_in or m[k] == 0:
                continue
            dlu[k] = lu(D[k, k])
            flops["fill"] += 2.0 / 3.0 * m[k] ** 3
            for j in near[lev][k]:
                if j != k:
                    Y[k, j] = sla.lu_solve(dlu[k], D[k, j], check_finite=False)
                    Yt[k, j] = sla.lu_solve(dlu[k], D[j, k].T, trans=1, check_finite=False)
        fac.cand[lev] = PU[lev]
        fac.cand_col[lev] = PV[lev]
        bf = [None] * nb
        for i in range(nb):
            targets = fill_targets(near[lev], i) if p.fill_in else []
            side = []
            for s_ in (0, 1):
                # s_ = 0: rows of A (U basis); s_ = 1: rows of A^T (V basis)
                Fcols = []
                for j in targets:
                    F = np.zeros((m[i], m[j]))
                    for k in near[lev][i]:
                        if k == i or k == j or m[k] == 0 or j not in near[lev][k]:
                            continue
                        F += D[i, k] @ Y[k, j] if s_ == 0 else D[k, i].T @ Yt[k, j]
                        flops["fill"] += 2.0 * m[i] * m[k] * m[j]
                    Fcols.append(F)
                if p.fill_in:
                    flops["fill"] += sum(2.0 * m[i] * m[k] ** 2 for k in near[lev][i] if k != i)
                Fi = np.concatenate(Fcols, axis=1) if Fcols else np.zeros((m[i], 0))
                Th = ThU if s_ == 0 else ThV
                if lev < L and m[i] > 0:
                    Fi = _block_tri_solve(Th[i], Fi)
                Pown = (PU if s_ == 0 else PV)[lev]
                fcols = far_columns(tree, near, far, lev, i, PV if s_ == 0 else PU, p.far_sample)
                if s_ == 0:
                    Kf = kernel_block(X, Pown[i], fcols, p)
                else:
                    Kf = kernel_block(X, fcols, Pown[i], p).T
                kevals += Kf.size
                M = np.concatenate([Kf, Fi], axis=1)
                ncol = M.shape[1]
                steps = min(m[i], ncol)
                if steps > 0:
                    piv, R, dg = pivoted_qr(M)
                    flops["basis"] += (2.0 * ncol * m[i] ** 2 - 2.0 / 3.0 * m[i] ** 3
                                       if ncol >= m[i] else
                                       2.0 * m[i] * ncol ** 2 - 2.0 / 3.0 * ncol ** 3)
                else:
                    piv, R, dg = np.arange(m[i], dtype=np.int64), None, np.zeros(0)
                side.append((piv, R, dg, ncol, steps, Pown[i], Th))
            kU = id_rank(side[0][2], p.tol, p.rank_cap, m[i], side[0][3])
            kV = id_rank(side[1][2], p.tol, p.rank_cap, m[i], side[1][3])
            k = min(max(kU, kV), side[0][4], side[1][4])
            out = []
            for piv, R, dg, ncol, steps, Pown, Th in side:
                Wp = id_matrix(piv, R, m[i], k) if k else np.zeros((m[i], 0))
                W = _block_tri_mul(Th[i], Wp) if (lev < L and m[i] > 0) else Wp
                B, T = complement_basis(W)
                flops["basis"] += 4.0 * m[i] * k * k + 4.0 * m[i] ** 2 * k
                out.append((B, T, np.asarray(Pown)[piv[:k]], piv, dg))
            (U, TU, skU, pU, dU), (V, TV, skV, pV, dV) = out
            bf[i] = BoxFactor(m[i], k, U, TU, skU, pU, absdiag=dU, V=V, TV=TV, skV=skV, pivV=pV,
                              absdiagV=dV)
        # (d) low-rank couplings
        Snew = {}
        for i in range(nb):
            for j in far[lev][i]:
                Kc = kernel_block(X, bf[i].sk, bf[j].skV, p)
                kevals += Kc.size
                Snew[i, j] = bf[i].T @ Kc @ bf[j].TV.T
                ki, kj = bf[i].k, bf[j].k
                flops["couple"] += 2.0 * ki * ki * kj + 2.0 * ki * kj * kj
        # (e) rotation + (f) elimination
        for i in range(nb):
            Ui, Vi, ki = bf[i].U, bf[i].V, bf[i].k
            for j in near[lev][i]:
                if j == i:
                    continue
                kj = bf[j].k
                Snew[i, j] = Ui[:, :ki].T @ D[i, j] @ bf[j].V[:, :kj]
                if ki and kj:
                    flops["rotate"] += 2.0 * m[i] * m[j] * kj + 2.0 * ki * m[i] * kj
            S = Ui.T @ D[i, i] @ Vi
            flops["rotate"] += 4.0 * m[i] ** 3
            r = m[i] - ki
            if r > 0:
                lu_, lp = lu(S[ki:, ki:])
                URS = lower_solve(lu_, apply_pinv(lp, S[ki:, :ki]))
                LSR = sla.solve_triangular(lu_, S[:ki, ki:].T, trans="T", lower=False,
                                           check_finite=False).T if ki else np.zeros((0, r))
                Snew[i, i] = S[:ki, :ki] - LSR @ URS
                bf[i].lu, bf[i].lupiv, bf[i].URS, bf[i].LSR = lu_, lp, URS, LSR
                flops["elim"] += 2.0 / 3.0 * r ** 3 + 2.0 * r * r * ki + 2.0 * ki * ki * r
            else:
                Snew[i, i] = S[:ki, :ki].copy()
        fac.levels[lev] = bf
        if lev > 1:
            PU[lev - 1] = [np.concatenate([bf[2 * q].sk, bf[2 * q + 1].sk]) for q in range(nb // 2)]
            PV[lev - 1] = [np.concatenate([bf[2 * q].skV, bf[2 * q + 1].skV])
                           for q in range(nb // 2)]
            ThU = [[bf[2 * q].T, bf[2 * q + 1].T] for q in range(nb // 2)]
            ThV = [[bf[2 * q].TV, bf[2 * q + 1].TV] for q in range(nb // 2)]
        Sblk = Snew
    D0 = np.block([[Sblk[0, 0], Sblk[0, 1]], [Sblk[1, 0], Sblk[1, 1]]])
    fac.m_root = D0.shape[0]
    fac.root_lu = lu(D0) if fac.m_root > 0 else (D0, np.zeros(0, dtype=np.int32))
    flops["root"] += 2.0 / 3.0 * fac.m_root ** 3
    fac.stats = {"flops": flops, "kevals": kevals}
    return fac


# ---------------------------------------------------------------------------
# Solve (Sec. II-B: L z = U^T b, U y = z, x = V^T y, applied level by level)
# ---------------------------------------------------------------------------
def solve(fac: Factor, B: np.ndarray) -> np.ndarray:
    tree = fac.tree
    L = tree.L
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    B2 = B.reshape(B.shape[0], -1)
    bt = B2[tree.perm]
    if L == 0:
        lu_, lp = fac.root_lu
        x = sla.lu_solve((lu_, lp), bt, check_finite=False)
        out = np.empty_like(x)
        out[tree.perm] = x
        return out.reshape(B.shape)
    # forward (the flat BLR^2 structure has the leaf level only, and its root
    # gathers the skeleton parts of every leaf)
    flat = fac.params.structure == "blr2"
    rhs = [bt[tree.start[L][i]:tree.end[L][i]] for i in range(1 << L)]
    saved = {}
    for lev in range(L, (L - 1) if flat else 0, -1):
        bf = fac.levels[lev]
        cs = []
        for i, f in enumerate(bf):
            c = f.U.T @ rhs[i]
            k = f.k
            cS, cR = c[:k].copy(), c[k:]
            yR = None
            if f.m - k > 0:
                yR = lower_solve(f.lu, apply_pinv(f.lupiv, cR))
                if k:
                    cS -= f.LSR @ yR
            saved[lev, i] = yR
            cs.append(cS)
        if flat:
            rhs = [np.concatenate(cs)]
        else:
            rhs = [np.concatenate([cs[2 * q], cs[2 * q + 1]]) for q in range(len(bf) // 2)]
    b0 = rhs[0]
    x0 = sla.lu_solve(fac.root_lu, b0, check_finite=False) if fac.m_root else b0
    xs = [x0]
    if flat:
        # skeleton parts of every leaf from the root, in leaf order
        parts, off = [], 0
        for f in fac.levels[L]:
            parts.append(x0[off:off + f.k])
            off += f.k
        nxt = []
        for i, (f, xS) in enumerate(zip(fac.levels[L], parts)):
            if f.m - f.k > 0:
                xR = upper_solve(f.lu, saved[L, i] - f.URS @ xS)
                nxt.append(right_basis(f) @ np.concatenate([xS, xR]))
            else:
                nxt.append(right_basis(f) @ xS)
        xs = nxt
    # backward
    for lev in ([] if flat else range(1, L + 1)):
        bf = fac.levels[lev]
        nxt = []
        for q in range(len(bf) // 2):
            xp = xs[q]
            k1 = bf[2 * q].k
            for i, xS in ((2 * q, xp[:k1]), (2 * q + 1, xp[k1:])):
                f = bf[i]
                if f.m - f.k > 0:
                    xR = upper_solve(f.lu, saved[lev, i] - f.URS @ xS)
                    nxt.append(right_basis(f) @ np.concatenate([xS, xR]))
                else:
                    nxt.append(right_basis(f) @ xS)
        xs = nxt
    xt = np.concatenate(xs)
    out = np.empty_like(xt)
    out[tree.perm] = xt
    return out[:, 0] if vec else out


def logabsdet(fac: Factor) -> float:
    """log|det A~| = sum log|diag U^RR| over all boxes + log|det D_root|
    (U and V are orthogonal)."""
    s = 0.0
    for lev, bf in fac.levels.items():
        for f in bf:
            if f.lu is not None:
                s += float(np.sum(np.log(np.abs(np.diag(f.lu)))))
    if fac.m_root:
        s += float(np.sum(np.log(np.abs(np.diag(fac.root_lu[0])))))
    return s


def refine(fac: Factor, B: np.ndarray, rtol: float = 1e-10, max_iter: int = 20):
    """Classical iterative refinement with the exact FP64 matvec:
    x = solve(b); repeat r = b - A x, stop when max_c |r_c|/|b_c| <= rtol,
    else x += solve(r).  Returns (x, iterations, relres)."""
    X, p = fac.X, fac.params
    x = solve(fac, B)
    bn = np.linalg.norm(B.reshape(B.shape[0], -1), axis=0)
    bn[bn == 0] = 1.0
    for it in range(max_iter + 1):
        r = B - matvec_exact(X, x, p)
        rel = float(np.max(np.linalg.norm(r.reshape(r.shape[0], -1), axis=0) / bn))
        if rel <= rtol:
            return x, it, rel
        if it == max_iter:
            break
        x = x + solve(fac, r)
    raise OracleError(ERR_NOT_CONVERGED, f"refinement stalled at {rel:.3e}")


def assemble_dense(fac: Factor) -> np.ndarray:
    """The matrix A~ that the factorization represents exactly, assembled densely
    in the original point order: at each level
      A~_l = U_l [[blkdiag S^RR, blkdiag S^RS], [blkdiag S^SR, A~_{l-1} + blkdiag S^SR S^RR^-1 S^RS]] V_l^T
    (rows of each box ordered [S; R]; V = U for shared bases, the right factor
    is V^T for separate ones); the flat BLR^2 structure has the leaf
    level alone, its root holding every leaf's skeleton.  Small N only."""
    tree = fac.tree
    L = tree.L
    flat = fac.params.structure == "blr2"
    lu_, lp = fac.root_lu
    if fac.m_root:
        Lm = np.tril(lu_, -1) + np.eye(fac.m_root)
        Um = np.triu(lu_)
        A = apply_pinv_inverse(lp, Lm @ Um)
    else:
        A = np.zeros((0, 0))
    for lev in ([L] if flat else range(1, L + 1)):
        bf = fac.levels[lev]
        ks = [f.k for f in bf]
        ms = [f.m for f in bf]
        ntot = sum(ms)
        ktot = sum(ks)
        # per-box ordering: all S parts first (box order), then R parts (box order)
        G = np.zeros((ntot, ntot))
        G[:ktot, :ktot] = A
        roff = ktot
        soff = 0
        pos = []  # (S range, R range) per box in G coordinates
        for f in bf:
            k, r = f.k, f.m - f.k
            sR = slice(roff, roff + r)
            sS = slice(soff, soff + k)
            if r > 0:
                Lm = np.tril(f.lu, -1) + np.eye(r)
                Um = np.triu(f.lu)
                SRR = apply_pinv_inverse(f.lupiv, Lm @ Um)
                SRS = apply_pinv_inverse(f.lupiv, Lm @ f.URS)
                SSR = f.LSR @ Um
                G[sR, sR] = SRR
                G[sR, sS] = SRS
                G[sS, sR] = SSR
                G[sS, sS] += SSR @ np.linalg.solve(SRR, SRS)
            pos.append((sS, sR))
            roff += r
            soff += k
        # map G coordinates to per-box [S;R] rotated coordinates, then apply U
        order = np.concatenate([np.r_[s.start:s.stop, r.start:r.stop] for s, r in pos]).astype(np.int64)
        Gb = G[np.ix_(order, order)]
        Ubig = sla.block_diag(*[f.U for f in bf]) if bf else np.zeros((0, 0))
        Vbig = sla.block_diag(*[right_basis(f) for f in bf]) if bf else np.zeros((0, 0))
        A = Ubig @ Gb @ Vbig.T
    out = np.empty_like(A)
    out[np.ix_(tree.perm, tree.perm)] = A
    return out


def apply_pinv_inverse(piv, B):
    """P B for LAPACK row interchanges (undo of apply_pinv)."""
    B = np.array(B, dtype=np.float64, copy=True)
    for t in range(len(piv) - 1, -1, -1):
        pt = piv[t]
        if pt != t:
            B[[t, pt]] = B[[pt, t]]
    return B


def total_flops(fac: Factor) -> float:
    return float(sum(fac.stats["flops"].values()))
