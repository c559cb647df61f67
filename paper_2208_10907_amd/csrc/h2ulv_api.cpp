// H^2-ULV library: solve sweeps, exact matvec, iterative refinement and the
// C-ABI entry points.  The factorization itself is the batched level driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <memory>

#include "h2ulv_factor.h"
#include "h2ulv_learned.h"

struct h2ulv_structure {
  h2ulv::Tree tree;
  h2ulv::Lists lists;
};

namespace h2ulv {

h2ulv_rankmodel* rankmodel_create(uint64_t seed);
void rankmodel_gradient(const h2ulv_rankmodel& M, const float* feat, const float* target,
                        int64_t n, float* grad, float* loss_host, hipStream_t s);
void rankmodel_adam(h2ulv_rankmodel& M, const float* grad, float lr, hipStream_t s);
void rankmodel_train(h2ulv_rankmodel& M, const float* feat, const float* target, int64_t n,
                     int steps, float lr, float* loss_host, hipStream_t s);

static thread_local std::string g_last_error;

// ---------------------------------------------------------------------------
// solve: forward sweep over levels, root, backward sweep (Sec. II-B)
// ---------------------------------------------------------------------------
static void solve_body(const h2ulv_factor& F, double* b, int nrhs, int64_t ldb, Stage& st) {
  hipStream_t s = st.s;
  const Tree& T = F.tree;
  const int L = T.L;
  const int64_t n = F.n;
  double* bt = st.scratch<double>(n * nrhs);
  launch_permute_rows(b, ldb, bt, n, F.perm.as<int64_t>(), n, nrhs, 0, s);
  H2ULV_HIP(hipGetLastError());
  if (L == 0) {
    double* x = st.scratch<double>(n * nrhs);
    GemmBatch<double> g;
    g.one(x, n, (int)n, nrhs, (int)n, F.root_inv.as<double>(), n, false, bt, n, false);
    g.run(st, "solve");
    launch_permute_rows(x, n, b, ldb, F.perm.as<int64_t>(), n, nrhs, 1, s);
    return;
  }
  // per-level RHS blocks: rhs[lev] holds m_i x nrhs per box (ld m_i); the leaf
  // level reads bt directly.  The top factored level is 1 (its two boxes meet
  // at the root), or the leaf level for the flat structure (every leaf meets
  // at the root).
  const int top = F.p.structure == 1 ? L : 1;
  std::vector<std::vector<int64_t>> moff(L + 1), woff(L + 1);
  std::vector<double*> rhs(L + 1, nullptr), cbuf(L + 1, nullptr), wbuf(L + 1, nullptr),
      xbuf(L + 1, nullptr);
  for (int lev = top; lev <= L; ++lev) {
    const LevelFactor& lf = F.levels[lev];
    moff[lev].assign(lf.nb + 1, 0);
    woff[lev].assign(lf.nb + 1, 0);
    for (int i = 0; i < lf.nb; ++i) {
      moff[lev][i + 1] = moff[lev][i] + (int64_t)lf.m[i] * nrhs;
      woff[lev][i + 1] = woff[lev][i] + (int64_t)(lf.m[i] - lf.k[i]) * nrhs;
    }
    cbuf[lev] = st.scratch<double>(std::max<int64_t>(moff[lev].back(), 1));
    wbuf[lev] = st.scratch<double>(std::max<int64_t>(woff[lev].back(), 1));
    xbuf[lev] = st.scratch<double>(std::max<int64_t>(moff[lev].back(), 1));
    if (lev < L) rhs[lev] = st.scratch<double>(std::max<int64_t>(moff[lev].back(), 1));
  }
  auto in_ptr = [&](int lev, int i, int64_t* ld) -> double* {
    if (lev == L) {
      *ld = n;
      return bt + T.start[L][i];
    }
    *ld = std::max(1, F.levels[lev].m[i]);
    return rhs[lev] + moff[lev][i];
  };
  // forward
  for (int lev = L; lev >= top; --lev) {
    const LevelFactor& lf = F.levels[lev];
    GemmBatch<double> g1, g2, g3;
    for (int i = 0; i < lf.nb; ++i) {
      int mi = lf.m[i], ki = lf.k[i], r = mi - ki;
      if (mi == 0) continue;
      int64_t ld;
      double* bi = in_ptr(lev, i, &ld);
      double* ci = cbuf[lev] + moff[lev][i];
      g1.one(ci, mi, mi, nrhs, mi, lf.U.as<double>() + lf.offU[i], mi, true, bi, ld, false);
      if (r > 0) {
        double* wi = wbuf[lev] + woff[lev][i];
        g2.one(wi, r, r, nrhs, r, lf.Sinv.as<double>() + lf.offR[i], r, false, ci + ki, mi,
               false);
        if (ki > 0)
          g3.one(ci, mi, ki, nrhs, r, lf.SSR.as<double>() + lf.offX[i], ki, false, wi, r, false,
                 -1.0, 1.0);
      }
    }
    g1.run(st, "solve");
    g2.run(st, "solve");
    g3.run(st, "solve");
    // gather c^S of both children into the parent's rhs
    CopyBatch cb;
    if (lev > top) {
      const LevelFactor& pa = F.levels[lev - 1];
      for (int p = 0; p < pa.nb; ++p) {
        int k1 = lf.k[2 * p], k2 = lf.k[2 * p + 1];
        double* dst = rhs[lev - 1] + moff[lev - 1][p];
        int mp = pa.m[p];
        cb.add(cbuf[lev] + moff[lev][2 * p], lf.m[2 * p], dst, mp, k1, nrhs);
        cb.add(cbuf[lev] + moff[lev][2 * p + 1], lf.m[2 * p + 1], dst + k1, mp, k2, nrhs);
      }
      cb.run(st);
    }
  }
  // root: the skeleton parts of the top level's boxes, in box order
  const LevelFactor& lt = F.levels[top];
  const int m0 = F.m_root;
  std::vector<int> koff(lt.nb + 1, 0);
  for (int a = 0; a < lt.nb; ++a) koff[a + 1] = koff[a] + lt.k[a];
  double* b0 = st.scratch<double>(std::max<int64_t>((int64_t)m0 * nrhs, 1));
  double* x0 = st.scratch<double>(std::max<int64_t>((int64_t)m0 * nrhs, 1));
  {
    CopyBatch cb;
    for (int a = 0; a < lt.nb; ++a)
      if (lt.k[a] > 0)
        cb.add(cbuf[top] + moff[top][a], lt.m[a], b0 + koff[a], m0, lt.k[a], nrhs);
    cb.run(st);
    GemmBatch<double> g;
    g.one(x0, m0, m0, nrhs, m0, F.root_inv.as<double>(), m0, false, b0, m0, false);
    g.run(st, "solve");
  }
  // backward: x = V [x^S; x^R] with the column bases (V = U for shared bases)
  for (int lev = top; lev <= L; ++lev) {
    const LevelFactor& lf = F.levels[lev];
    const LevelFactor& rv = F.colview ? F.colview->levels[lev] : lf;
    GemmBatch<double> g1, g2;
    for (int i = 0; i < lf.nb; ++i) {
      int mi = lf.m[i], ki = lf.k[i], r = mi - ki;
      if (mi == 0) continue;
      // skeleton part of the solution from the parent
      const double* xs;
      int64_t ldxs;
      if (lev == top) {
        xs = x0 + koff[i];
        ldxs = std::max(m0, 1);
      } else {
        int p = i / 2;
        const LevelFactor& pa = F.levels[lev - 1];
        xs = xbuf[lev - 1] + moff[lev - 1][p] + ((i & 1) ? lf.k[i - 1] : 0);
        ldxs = std::max(pa.m[p], 1);
      }
      double* wi = wbuf[lev] + woff[lev][i];
      if (r > 0 && ki > 0)
        g1.one(wi, r, r, nrhs, ki, lf.Xs.as<double>() + lf.offX[i], r, false, xs, ldxs, false,
               -1.0, 1.0);
      double* xo;
      int64_t ldo;
      if (lev == L) {
        xo = bt + T.start[L][i];
        ldo = n;
      } else {
        xo = xbuf[lev] + moff[lev][i];
        ldo = mi;
      }
      g2.item(xo, ldo, mi, nrhs);
      if (ki > 0) g2.term(rv.U.as<double>() + rv.offU[i], mi, false, xs, ldxs, false, ki);
      if (r > 0)
        g2.term(rv.U.as<double>() + rv.offU[i] + (int64_t)ki * mi, mi, false, wi, r, false, r);
    }
    g1.run(st, "solve");
    g2.run(st, "solve");
  }
  launch_permute_rows(bt, n, b, ldb, F.perm.as<int64_t>(), n, nrhs, 1, s);
  H2ULV_HIP(hipGetLastError());
}


static void solve_impl(const h2ulv_factor& F, double* b, int nrhs, int64_t ldb, hipStream_t s) {
  Stage st(s);
  solve_body(F, b, nrhs, ldb, st);
  st.sync();
}

// A solve recorded in a HIP graph for one right-hand-side count: the launches
// of solve_body on fixed buffers (an n x nrhs staging block in and out), its
// scratch and descriptor uploads kept for the graph's lifetime.  Recorded on a
// stream of its own after a first eager pass that allocated everything, so the
// capture allocates nothing; replays on the caller's stream.
struct SolveGraph {
  int nrhs = 0;
  hipStream_t cs = nullptr;
  std::unique_ptr<Stage> st;
  DBuf io;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  hipEvent_t done = nullptr;  // the last replay's copy-out (the staging block is free after it)
  ~SolveGraph() {
    if (cs) (void)hipStreamSynchronize(cs);
    if (done) (void)hipEventSynchronize(done);
    if (ex) (void)hipGraphExecDestroy(ex);
    if (g) (void)hipGraphDestroy(g);
    st.reset();
    if (done) (void)hipEventDestroy(done);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

static std::shared_ptr<SolveGraph> solve_graph_for(const h2ulv_factor& F, int nrhs) {
  std::lock_guard<std::mutex> lk(F.graph_mu);
  for (auto& gp : F.solve_graphs)
    if (gp->nrhs == nrhs) return gp;
  auto gp = std::make_shared<SolveGraph>();
  gp->nrhs = nrhs;
  // the GEMM tile rates are measured outside the capture (a factorization has
  // normally done it already)
  (void)gemm_tile_rates(true, nullptr);
  H2ULV_HIP(hipStreamCreateWithFlags(&gp->cs, hipStreamNonBlocking));
  H2ULV_HIP(hipEventCreateWithFlags(&gp->done, hipEventDisableTiming));
  gp->io.alloc((size_t)F.n * nrhs * sizeof(double));
  H2ULV_HIP(hipMemsetAsync(gp->io.p, 0, (size_t)F.n * nrhs * sizeof(double), gp->cs));
  gp->st = std::make_unique<Stage>(gp->cs);
  solve_body(F, gp->io.as<double>(), nrhs, F.n, *gp->st);  // first pass: allocates
  H2ULV_HIP(hipStreamSynchronize(gp->cs));
  gp->st->begin_replay();
  H2ULV_HIP(hipStreamBeginCapture(gp->cs, hipStreamCaptureModeRelaxed));
  try {
    solve_body(F, gp->io.as<double>(), nrhs, F.n, *gp->st);
  } catch (...) {
    hipGraph_t junk = nullptr;
    (void)hipStreamEndCapture(gp->cs, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    throw;
  }
  H2ULV_HIP(hipStreamEndCapture(gp->cs, &gp->g));
  H2ULV_HIP(hipGraphInstantiate(&gp->ex, gp->g, nullptr, nullptr, 0));
  F.solve_graphs.push_back(gp);
  return gp;
}

// solve_impl through the recorded graph of this right-hand-side count: copy b
// into the staging block, replay, copy back.  Solves of one factor are
// serialised on the staging block by an event (a replay waits for the previous
// replay's copy-out).
static void solve_graph(const h2ulv_factor& F, double* b, int nrhs, int64_t ldb, hipStream_t s) {
  std::shared_ptr<SolveGraph> gp = solve_graph_for(F, nrhs);
  const int64_t n = F.n;
  H2ULV_HIP(hipStreamWaitEvent(s, gp->done, 0));
  H2ULV_HIP(hipMemcpy2DAsync(gp->io.p, n * sizeof(double), b, ldb * sizeof(double),
                             n * sizeof(double), nrhs, hipMemcpyDeviceToDevice, s));
  {
    ProfScope ps("solve_graph", 0, 0, s);
    H2ULV_HIP(hipGraphLaunch(gp->ex, s));
  }
  H2ULV_HIP(hipMemcpy2DAsync(b, ldb * sizeof(double), gp->io.p, n * sizeof(double),
                             n * sizeof(double), nrhs, hipMemcpyDeviceToDevice, s));
  H2ULV_HIP(hipEventRecord(gp->done, s));
}

static h2ulv_factor* factorize_impl(const double* pts, int64_t n, const h2ulv_params* params,
                                    hipStream_t s) {
  validate_params(params);
  return factorize_many({pts}, {n}, *params, s)[0];
}

static void matvec_impl(const h2ulv_factor& F, const double* x, int64_t ldx, double* y,
                        int64_t ldy, int nrhs, hipStream_t s) {
  // partial sums of the source ranges; the stream is drained before the
  // buffer goes back to the cache, which other streams may draw from
  const int64_t words = matvec_work_words(F.n, nrhs);
  DBuf work(std::max<int64_t>(words, 1) * sizeof(double));
  {
    // algorithmic work of a dense y = A x: 2 flops per matrix entry and column;
    // bytes: the points, x and y
    const double nn = (double)F.n;
    ProfScope ps("matvec", 2.0 * nn * nn * nrhs, 8.0 * nn * (3.0 + 2.0 * nrhs), s);
    launch_matvec(F.pts.as<double>(), F.n, kfn(F.p), x, ldx, y, ldy, nrhs,
                  words > 0 ? work.as<double>() : nullptr, s);
  }
  H2ULV_HIP(hipGetLastError());
  if (words > 0) H2ULV_HIP(hipStreamSynchronize(s));
}

static h2ulv_status refine_impl(const h2ulv_factor& F, const double* b, int64_t ldb, double* x,
                                int64_t ldx, int nrhs, double rtol, int max_iter, int32_t* iters,
                                double* relres, hipStream_t s) {
  const int64_t n = F.n;
  DBuf ax(n * nrhs * sizeof(double)), r(n * nrhs * sizeof(double)),
      nr(2 * nrhs * sizeof(double));
  // x = solve(b)
  CopyBatch cb;
  Stage st(s);
  cb.add(b, ldb, x, ldx, (int)n, nrhs);
  cb.run(st);
  st.sync();
  solve_graph(F, x, nrhs, ldx, s);
  double rel = 0;
  std::vector<double> h(2 * nrhs);
  for (int it = 0; it <= max_iter; ++it) {
    matvec_impl(F, x, ldx, ax.as<double>(), n, nrhs, s);
    launch_resid_norms(b, ldb, ax.as<double>(), n, r.as<double>(), n, n, nrhs, nr.as<double>(),
                       nr.as<double>() + nrhs, s);
    H2ULV_HIP(hipMemcpyAsync(h.data(), nr.p, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost,
                             s));
    H2ULV_HIP(hipStreamSynchronize(s));
    rel = 0;
    for (int c = 0; c < nrhs; ++c) {
      double bn = std::sqrt(h[nrhs + c]);
      double rn = std::sqrt(h[c]);
      rel = std::max(rel, bn > 0 ? rn / bn : rn);
    }
    if (relres) *relres = rel;
    if (iters) *iters = it;
    if (rel <= rtol) return H2ULV_OK;
    if (it == max_iter) break;
    solve_graph(F, r.as<double>(), nrhs, n, s);
    launch_axpy_cols(x, ldx, r.as<double>(), n, n, nrhs, s);
    H2ULV_HIP(hipGetLastError());
  }
  g_last_error = "refinement did not reach the tolerance";
  return H2ULV_ERR_NOT_CONVERGED;
}

// Restarted GMRES on A x = b, right-preconditioned by the ULV solve (the
// correction equation of iterative refinement solved in a Krylov space): the
// same two operations per step as classical refinement (one exact matvec, one
// solve), but the correction is the best one in the space they span.  The
// right-hand sides run in lockstep: each has its own Krylov basis, Hessenberg
// matrix and stopping test, while the solve and the exact matvec of a step act
// on all of them at once (the matvec evaluates each kernel entry once for all
// columns).  Arnoldi with classical Gram-Schmidt applied twice; Givens
// rotations give the residual estimate; every restart recomputes the true
// residuals with the exact matvec.
static h2ulv_status gmres_impl(const h2ulv_factor& F, const double* b, int64_t ldb, double* x,
                               int64_t ldx, int nrhs, double rtol, int max_iter, int restart,
                               int32_t* iters, double* relres, hipStream_t s) {
  const int64_t n = F.n;
  constexpr int MAXM = 128;  // longest Krylov cycle
  const int m = std::max(1, std::min(restart, MAXM));
  constexpr int NBLK = 256;
  constexpr int HS = 2 * MAXM + 32;  // per column: two Gram-Schmidt passes and the norm
  // Krylov blocks: block j holds column u's j-th vector at offset u * n
  DBuf Vb((int64_t)(m + 1) * n * nrhs * sizeof(double)),
      Zb((int64_t)m * n * nrhs * sizeof(double)), wb(n * nrhs * sizeof(double)),
      rb(n * nrhs * sizeof(double)), part((int64_t)NBLK * 32 * sizeof(double)),
      hd((int64_t)nrhs * HS * sizeof(double)), ys((int64_t)nrhs * MAXM * sizeof(double)),
      nr(2 * nrhs * sizeof(double));
  double* V = Vb.as<double>();
  double* Z = Zb.as<double>();
  double* w = wb.as<double>();
  double* r = rb.as<double>();
  double* h = hd.as<double>();
  {
    // x0 = M^-1 b
    CopyBatch cb;
    Stage st(s);
    cb.add(b, ldb, x, ldx, (int)n, nrhs);
    cb.run(st);
    st.sync();
  }
  solve_graph(F, x, nrhs, ldx, s);
  std::vector<int> steps(nrhs, 0);
  std::vector<double> rel(nrhs, 0.0), bnorm(nrhs, 0.0), beta(nrhs, 0.0);
  std::vector<char> done(nrhs, 0);
  std::vector<double> hv(2 * nrhs), hh((size_t)nrhs * HS);
  for (;;) {
    // true residuals r = b - A x of every column
    matvec_impl(F, x, ldx, w, n, nrhs, s);
    launch_resid_norms(b, ldb, w, n, r, n, n, nrhs, nr.as<double>(), nr.as<double>() + nrhs, s);
    H2ULV_HIP(hipMemcpyAsync(hv.data(), nr.p, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost,
                             s));
    H2ULV_HIP(hipStreamSynchronize(s));
    std::vector<int> act;  // columns that take another cycle
    for (int c = 0; c < nrhs; ++c) {
      bnorm[c] = std::sqrt(hv[nrhs + c]);
      beta[c] = std::sqrt(hv[c]);
      rel[c] = bnorm[c] > 0 ? beta[c] / bnorm[c] : beta[c];
      done[c] = rel[c] <= rtol;
      if (!done[c] && steps[c] < max_iter) act.push_back(c);
    }
    if (act.empty()) break;
    const int na = (int)act.size();
    const int64_t ldk = n * na;  // stride between a column's Krylov vectors
    // v0 = r / |r| per column
    for (int u = 0; u < na; ++u)
      launch_scale_inv_norm(V + (int64_t)u * n, r + (int64_t)act[u] * n,
                            nr.as<double>() + act[u], n, s);
    H2ULV_HIP(hipGetLastError());
    std::vector<std::vector<double>> H(na, std::vector<double>((size_t)(m + 1) * m, 0.0)),
        g(na, std::vector<double>(m + 1, 0.0)), cs(na, std::vector<double>(m, 0.0)),
        sn(na, std::vector<double>(m, 0.0));
    std::vector<int> jc(na, 0);
    std::vector<char> run(na, 1);
    for (int u = 0; u < na; ++u) g[u][0] = beta[act[u]];
    for (int j = 0; j < m; ++j) {
      std::vector<int> live;
      for (int u = 0; u < na; ++u)
        if (run[u]) live.push_back(u);
      if (live.empty()) break;
      double* Vj = V + (int64_t)j * ldk;
      double* Zj = Z + (int64_t)j * ldk;
      // z = M^-1 v and w = A z for all columns of the block at once
      H2ULV_HIP(hipMemcpyAsync(Zj, Vj, ldk * sizeof(double), hipMemcpyDeviceToDevice, s));
      solve_graph(F, Zj, na, n, s);
      matvec_impl(F, Zj, n, w, n, na, s);
      // w_u -= V_u h_u, twice (classical Gram-Schmidt with re-orthogonalisation)
      for (int pass = 0; pass < 2; ++pass) {
        // the dot products 32 basis vectors per launch
        for (int u : live)
          for (int c0 = 0; c0 <= j; c0 += 32)
            launch_multidot(V + (int64_t)c0 * ldk + (int64_t)u * n, ldk,
                            std::min(32, j + 1 - c0), w + (int64_t)u * n, n, part.as<double>(),
                            NBLK, h + (int64_t)u * HS + MAXM * pass + c0, s);
        Stage st(s);
        GemmBatch<double> gb;
        for (int u : live)
          gb.one(w + (int64_t)u * n, n, (int)n, 1, j + 1, V + (int64_t)u * n, ldk, false,
                 h + (int64_t)u * HS + MAXM * pass, j + 1, false, -1.0, 1.0);
        gb.run(st, "gmres");
        st.sync();
      }
      for (int u : live) {
        launch_multidot(w + (int64_t)u * n, n, 1, w + (int64_t)u * n, n, part.as<double>(), NBLK,
                        h + (int64_t)u * HS + 2 * MAXM, s);
        launch_scale_inv_norm(V + (int64_t)(j + 1) * ldk + (int64_t)u * n, w + (int64_t)u * n,
                              h + (int64_t)u * HS + 2 * MAXM, n, s);
      }
      H2ULV_HIP(hipGetLastError());
      H2ULV_HIP(hipMemcpyAsync(hh.data(), h, (size_t)na * HS * sizeof(double),
                               hipMemcpyDeviceToHost, s));
      H2ULV_HIP(hipStreamSynchronize(s));
      for (int u : live) {
        const int c = act[u];
        ++steps[c];
        const double* hu = hh.data() + (size_t)u * HS;
        // column j of the Hessenberg matrix
        double* col = H[u].data() + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = hu[i] + hu[MAXM + i];
        col[j + 1] = std::sqrt(std::max(hu[2 * MAXM], 0.0));
        for (int i = 0; i < j; ++i) {
          const double a0 = col[i], a1 = col[i + 1];
          col[i] = cs[u][i] * a0 + sn[u][i] * a1;
          col[i + 1] = -sn[u][i] * a0 + cs[u][i] * a1;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        cs[u][j] = den > 0 ? col[j] / den : 1.0;
        sn[u][j] = den > 0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        g[u][j + 1] = -sn[u][j] * g[u][j];
        g[u][j] = cs[u][j] * g[u][j];
        jc[u] = j + 1;
        // stop early when the estimate is well below the target, on breakdown,
        // or at the step limit
        if (std::fabs(g[u][j + 1]) <= 0.5 * rtol * bnorm[c] || hu[2 * MAXM] <= 0.0 ||
            steps[c] >= max_iter)
          run[u] = 0;
      }
    }
    // y = R^-1 g, x += Z y per column
    std::vector<double> y((size_t)na * MAXM, 0.0);
    for (int u = 0; u < na; ++u) {
      const int jj = jc[u];
      double* yu = y.data() + (size_t)u * MAXM;
      for (int i = jj - 1; i >= 0; --i) {
        double sacc = g[u][i];
        for (int l = i + 1; l < jj; ++l) sacc -= H[u][(size_t)l * (m + 1) + i] * yu[l];
        const double d = H[u][(size_t)i * (m + 1) + i];
        yu[i] = d != 0.0 ? sacc / d : 0.0;
      }
    }
    H2ULV_HIP(hipMemcpyAsync(ys.p, y.data(), y.size() * sizeof(double), hipMemcpyHostToDevice,
                             s));
    {
      Stage st(s);
      GemmBatch<double> gb;
      for (int u = 0; u < na; ++u)
        if (jc[u] > 0)
          gb.one(x + (int64_t)act[u] * ldx, ldx, (int)n, 1, jc[u], Z + (int64_t)u * n, ldk, false,
                 ys.as<double>() + (int64_t)u * MAXM, jc[u], false, 1.0, 1.0);
      gb.run(st, "gmres");
      st.sync();
    }
  }
  int worst_it = 0;
  double worst_rel = 0.0;
  bool converged_all = true;
  for (int c = 0; c < nrhs; ++c) {
    worst_it = std::max(worst_it, steps[c]);
    worst_rel = std::max(worst_rel, rel[c]);
    converged_all = converged_all && done[c];
  }
  if (iters) *iters = worst_it;
  if (relres) *relres = worst_rel;
  if (converged_all) return H2ULV_OK;
  g_last_error = "GMRES refinement did not reach the tolerance";
  return H2ULV_ERR_NOT_CONVERGED;
}

namespace {
// Small dense host helpers of the block GMRES (matrices column-major).

// Eigenpairs of a symmetric q x q matrix by cyclic Jacobi rotations:
// A = E diag(lam) E^T.
void sym_eig(std::vector<double> A, int q, std::vector<double>& lam, std::vector<double>& E) {
  E.assign((size_t)q * q, 0.0);
  for (int i = 0; i < q; ++i) E[i + (size_t)i * q] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i)
        (i == j ? dia : off) += A[i + (size_t)j * q] * A[i + (size_t)j * q];
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int p = 0; p < q; ++p)
      for (int r = p + 1; r < q; ++r) {
        const double apr = A[p + (size_t)r * q];
        if (apr == 0.0) continue;
        const double app = A[p + (size_t)p * q], arr = A[r + (size_t)r * q];
        const double th = 0.5 * (arr - app) / apr;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < q; ++k) {  // columns p, r
          const double akp = A[k + (size_t)p * q], akr = A[k + (size_t)r * q];
          A[k + (size_t)p * q] = c * akp - s * akr;
          A[k + (size_t)r * q] = s * akp + c * akr;
        }
        for (int k = 0; k < q; ++k) {  // rows p, r
          const double apk = A[p + (size_t)k * q], ark = A[r + (size_t)k * q];
          A[p + (size_t)k * q] = c * apk - s * ark;
          A[r + (size_t)k * q] = s * apk + c * ark;
        }
        for (int k = 0; k < q; ++k) {
          const double ekp = E[k + (size_t)p * q], ekr = E[k + (size_t)r * q];
          E[k + (size_t)p * q] = c * ekp - s * ekr;
          E[k + (size_t)r * q] = s * ekp + c * ekr;
        }
      }
  }
  lam.resize(q);
  for (int i = 0; i < q; ++i) lam[i] = A[i + (size_t)i * q];
}

// Upper Cholesky factor of a symmetric positive definite q x q matrix (G = R^T R);
// false when a pivot is not positive.
bool chol_upper(const std::vector<double>& G, int q, std::vector<double>& R) {
  R.assign((size_t)q * q, 0.0);
  for (int j = 0; j < q; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = G[i + (size_t)j * q];
      for (int k = 0; k < i; ++k) s -= R[k + (size_t)i * q] * R[k + (size_t)j * q];
      if (i == j) {
        if (!(s > 0.0)) return false;
        R[j + (size_t)j * q] = std::sqrt(s);
      } else {
        R[i + (size_t)j * q] = s / R[i + (size_t)i * q];
      }
    }
  }
  return true;
}

// min_Y |E - H Y|_F column by column for H (rows x cols, rows > cols) by
// Householder QR; Y is cols x p, res[c] the residual norm of column c.
void least_squares(std::vector<double> Hm, int rows, int cols, std::vector<double> E, int p,
                   std::vector<double>& Y, std::vector<double>& res) {
  for (int j = 0; j < cols; ++j) {
    double nrm = 0.0;
    for (int i = j; i < rows; ++i) nrm += Hm[i + (size_t)j * rows] * Hm[i + (size_t)j * rows];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double a = Hm[j + (size_t)j * rows];
    const double beta = a >= 0 ? -nrm : nrm;
    std::vector<double> v(rows - j);
    v[0] = a - beta;
    for (int i = j + 1; i < rows; ++i) v[i - j] = Hm[i + (size_t)j * rows];
    double vv = 0.0;
    for (double x : v) vv += x * x;
    if (vv == 0.0) continue;
    auto reflect = [&](double* col) {
      double d = 0.0;
      for (int i = j; i < rows; ++i) d += v[i - j] * col[i];
      d = 2.0 * d / vv;
      for (int i = j; i < rows; ++i) col[i] -= d * v[i - j];
    };
    for (int k = j; k < cols; ++k) reflect(Hm.data() + (size_t)k * rows);
    for (int k = 0; k < p; ++k) reflect(E.data() + (size_t)k * rows);
  }
  Y.assign((size_t)cols * p, 0.0);
  res.assign(p, 0.0);
  for (int k = 0; k < p; ++k) {
    const double* e = E.data() + (size_t)k * rows;
    double* y = Y.data() + (size_t)k * cols;
    for (int i = cols - 1; i >= 0; --i) {
      double s = e[i];
      for (int l = i + 1; l < cols; ++l) s -= Hm[i + (size_t)l * rows] * y[l];
      const double d = Hm[i + (size_t)i * rows];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
    double r = 0.0;
    for (int i = cols; i < rows; ++i) r += e[i] * e[i];
    res[k] = std::sqrt(r);
  }
}
}  // namespace

// Block GMRES for several right-hand sides (restarted, right-preconditioned by
// the ULV solve).  All residuals span one Krylov space: every step applies the
// solve and the exact matvec to a block of up to p vectors, and the outlying
// eigenvalues of the preconditioned operator, the same for every right-hand
// side, are found once for all of them.  The residual columns are scaled by
// 1/|b_c|, so each column's least-squares residual is its relative residual.
// Block orthonormalisation: the Gram matrix of the block (one GEMM), its
// eigenvectors on the host with directions below 1e-12 of the largest (or, for
// the starting block, below 1e-3 rtol) dropped (deflation), then a second pass
// with the Cholesky factor of the new Gram matrix.  Block classical Gram-Schmidt
// against all earlier blocks, applied twice, as GEMMs.
static h2ulv_status block_gmres_impl(const h2ulv_factor& F, const double* b, int64_t ldb,
                                     double* x, int64_t ldx, int p, double rtol, int max_iter,
                                     int restart, int32_t* iters, double* relres, hipStream_t s) {
  const int64_t n = F.n;
  const int m = std::max(1, std::min(restart, 128));
  const int QMAX = p * (m + 1);
  DBuf Vb((int64_t)QMAX * n * sizeof(double)), Zb((int64_t)p * m * n * sizeof(double)),
      Wb((int64_t)p * n * sizeof(double)), Rb((int64_t)p * n * sizeof(double)),
      nr(2 * p * sizeof(double)), hd((int64_t)QMAX * p * sizeof(double)),
      td((int64_t)p * p * sizeof(double)), yd((int64_t)QMAX * p * sizeof(double));
  double* V = Vb.as<double>();
  double* Z = Zb.as<double>();
  double* Wm = Wb.as<double>();
  double* R = Rb.as<double>();
  double* hdev = hd.as<double>();
  double* tdev = td.as<double>();
  auto gemm = [&](double* C, int64_t ldc, int M, int N, int K, const double* A, int64_t lda,
                  bool ta, const double* B, int64_t ldB, double alpha, double beta) {
    if (M <= 0 || N <= 0) return;
    Stage st(s);
    GemmBatch<double> g;
    g.one(C, ldc, M, N, K, A, lda, ta, B, ldB, false, alpha, beta);
    g.run(st, "bgmres");
    st.sync();
  };
  // C (M x N) = A^T B over the n rows (inner products with the basis): row
  // chunks in parallel, summed in a fixed order, 8 columns of B at a time
  DBuf gpart((int64_t)GRAM_CHUNKS * QMAX * 8 * sizeof(double));
  auto inner = [&](double* C, int64_t ldc, int M, int N, const double* A, const double* B) {
    for (int j0 = 0; j0 < N; j0 += 8) {
      launch_gram(A, n, M, B + (int64_t)j0 * n, n, std::min(8, N - j0), n,
                  C + (int64_t)j0 * ldc, ldc, gpart.as<double>(), s);
      H2ULV_HIP(hipGetLastError());
    }
  };
  auto download = [&](const double* src, int64_t cnt) {
    std::vector<double> h(cnt);
    H2ULV_HIP(hipMemcpyAsync(h.data(), src, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    H2ULV_HIP(hipStreamSynchronize(s));
    return h;
  };
  auto upload = [&](double* dst, const std::vector<double>& h) {
    H2ULV_HIP(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
  };
  // Orthonormal basis of the columns of A (n x q, column scales sc), written to
  // out; returns its width q' and Rf (q' x q) with A diag(sc) = out Rf.
  auto block_qr = [&](const double* A, int q, const std::vector<double>& sc, double floor_abs,
                      double* out, std::vector<double>& Rf) -> int {
    inner(tdev, q, q, q, A, A);
    std::vector<double> G = download(tdev, (int64_t)q * q);
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) G[i + (size_t)j * q] *= sc[i] * sc[j];
    std::vector<double> lam, E;
    sym_eig(G, q, lam, E);
    double lmax = 0.0;
    for (double l : lam) lmax = std::max(lmax, l);
    std::vector<int> keep;
    for (int i = 0; i < q; ++i)
      if (lam[i] > 1e-24 * lmax && lam[i] > floor_abs * floor_abs) keep.push_back(i);
    const int qk = (int)keep.size();
    Rf.assign((size_t)qk * q, 0.0);
    if (qk == 0) return 0;
    // T = diag(sc) E_keep Lambda^-1/2 (q x qk); out = A T
    std::vector<double> T((size_t)q * qk);
    for (int c = 0; c < qk; ++c)
      for (int i = 0; i < q; ++i)
        T[i + (size_t)c * q] = sc[i] * E[i + (size_t)keep[c] * q] / std::sqrt(lam[keep[c]]);
    upload(tdev, T);
    gemm(out, n, (int)n, qk, q, A, n, false, tdev, q, 1.0, 0.0);
    // second pass: out^T out = C^T C, out <- out C^-1
    inner(tdev, qk, qk, qk, out, out);
    std::vector<double> G2 = download(tdev, (int64_t)qk * qk), Cu;
    if (!chol_upper(G2, qk, Cu)) fail(H2ULV_ERR_HIP, "block GMRES: orthonormalisation failed");
    std::vector<double> Ci((size_t)qk * qk, 0.0);  // C^-1 (upper)
    for (int j = 0; j < qk; ++j) {
      Ci[j + (size_t)j * qk] = 1.0 / Cu[j + (size_t)j * qk];
      for (int i = j - 1; i >= 0; --i) {
        double acc = 0.0;
        for (int k = i + 1; k <= j; ++k) acc += Cu[i + (size_t)k * qk] * Ci[k + (size_t)j * qk];
        Ci[i + (size_t)j * qk] = -acc / Cu[i + (size_t)i * qk];
      }
    }
    upload(tdev, Ci);
    gemm(Wm, n, (int)n, qk, qk, out, n, false, tdev, qk, 1.0, 0.0);
    H2ULV_HIP(hipMemcpyAsync(out, Wm, (size_t)qk * n * sizeof(double), hipMemcpyDeviceToDevice,
                             s));
    // Rf = C Lambda^1/2 E_keep^T
    for (int j = 0; j < q; ++j)
      for (int r = 0; r < qk; ++r) {
        double acc = 0.0;
        for (int k = r; k < qk; ++k)
          acc += Cu[r + (size_t)k * qk] * std::sqrt(lam[keep[k]]) * E[j + (size_t)keep[k] * q];
        Rf[r + (size_t)j * qk] = acc;
      }
    return qk;
  };
  {
    CopyBatch cb;
    Stage st(s);
    cb.add(b, ldb, x, ldx, (int)n, p);
    cb.run(st);
    st.sync();
  }
  solve_graph(F, x, p, ldx, s);
  int steps = 0;
  std::vector<double> rel(p, 0.0), bn(p, 1.0);
  for (;;) {
    matvec_impl(F, x, ldx, Wm, n, p, s);
    launch_resid_norms(b, ldb, Wm, n, R, n, n, p, nr.as<double>(), nr.as<double>() + p, s);
    std::vector<double> hv = download(nr.as<double>(), 2 * p);
    bool done = true;
    for (int c = 0; c < p; ++c) {
      bn[c] = std::sqrt(hv[p + c]);
      if (bn[c] == 0.0) bn[c] = 1.0;
      rel[c] = std::sqrt(hv[c]) / bn[c];
      done = done && rel[c] <= rtol;
    }
    if (done || steps >= max_iter) break;
    std::vector<double> sc(p);
    for (int c = 0; c < p; ++c) sc[c] = 1.0 / bn[c];
    std::vector<double> S0;
    const int q0 = block_qr(R, p, sc, 1e-3 * rtol, V, S0);
    if (q0 == 0) break;
    std::vector<int> qs{q0};
    std::vector<int64_t> qoff{0, q0};
    std::vector<std::vector<double>> Hcol;  // per step: (qoff[j+1] + q_{j+1}) x q_j
    std::vector<double> Y, res;
    int Qz = 0;  // columns of Z
    for (int j = 0; j < m && steps < max_iter; ++j) {
      const int qj = qs[j];
      double* Vj = V + qoff[j] * n;
      double* Zj = Z + (int64_t)Qz * n;
      H2ULV_HIP(hipMemcpyAsync(Zj, Vj, (size_t)qj * n * sizeof(double), hipMemcpyDeviceToDevice,
                               s));
      solve_graph(F, Zj, qj, n, s);
      matvec_impl(F, Zj, n, Wm, n, qj, s);
      ++steps;
      Qz += qj;
      const int Qj = (int)qoff[j + 1];
      std::vector<double> h((size_t)Qj * qj, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        inner(hdev, Qj, Qj, qj, V, Wm);
        std::vector<double> hp = download(hdev, (int64_t)Qj * qj);
        for (size_t e = 0; e < hp.size(); ++e) h[e] += hp[e];
        gemm(Wm, n, (int)n, qj, Qj, V, n, false, hdev, Qj, -1.0, 1.0);
      }
      std::vector<double> ones(qj, 1.0), Rn;
      const int qn = block_qr(Wm, qj, ones, 0.0, V + (int64_t)Qj * n, Rn);
      qs.push_back(qn);
      qoff.push_back(Qj + qn);
      std::vector<double> colblk((size_t)(Qj + qn) * qj, 0.0);
      for (int c = 0; c < qj; ++c) {
        for (int i = 0; i < Qj; ++i) colblk[i + (size_t)c * (Qj + qn)] = h[i + (size_t)c * Qj];
        for (int i = 0; i < qn; ++i) colblk[Qj + i + (size_t)c * (Qj + qn)] = Rn[i + (size_t)c * qn];
      }
      Hcol.push_back(std::move(colblk));
      // least squares over the block Hessenberg matrix
      const int rows = Qj + qn, cols = Qz;
      std::vector<double> Hm((size_t)rows * cols, 0.0);
      int c0 = 0;
      for (size_t jj = 0; jj < Hcol.size(); ++jj) {
        const int rj = (int)qoff[jj + 1] + qs[jj + 1];
        for (int c = 0; c < qs[jj]; ++c)
          for (int i = 0; i < rj; ++i)
            Hm[i + (size_t)(c0 + c) * rows] = Hcol[jj][i + (size_t)c * rj];
        c0 += qs[jj];
      }
      std::vector<double> E1((size_t)rows * p, 0.0);
      for (int c = 0; c < p; ++c)
        for (int i = 0; i < q0; ++i) E1[i + (size_t)c * rows] = S0[i + (size_t)c * q0];
      least_squares(Hm, rows, cols, E1, p, Y, res);
      double worst = 0.0;
      for (double r : res) worst = std::max(worst, r);
      if (worst <= 0.5 * rtol || qn == 0) break;
    }
    if (Qz == 0) break;
    // x_c += |b_c| (Z Y)_c
    for (int c = 0; c < p; ++c)
      for (int i = 0; i < Qz; ++i) Y[i + (size_t)c * Qz] *= bn[c];
    upload(yd.as<double>(), Y);
    gemm(x, ldx, (int)n, p, Qz, Z, n, false, yd.as<double>(), Qz, 1.0, 1.0);
  }
  double worst = 0.0;
  bool ok = true;
  for (int c = 0; c < p; ++c) {
    worst = std::max(worst, rel[c]);
    ok = ok && rel[c] <= rtol;
  }
  if (iters) *iters = steps;
  if (relres) *relres = worst;
  if (ok) return H2ULV_OK;
  g_last_error = "block GMRES refinement did not reach the tolerance";
  return H2ULV_ERR_NOT_CONVERGED;
}

template <class Fn>
static h2ulv_status guarded(Fn&& fn) {
  try {
    fn();
    return H2ULV_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return H2ULV_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return H2ULV_ERR_HIP;
  }
}

}  // namespace h2ulv

using namespace h2ulv;

extern "C" {

h2ulv_status h2ulv_params_default(h2ulv_params* p) {
  if (!p) {
    g_last_error = "params is NULL";
    return H2ULV_ERR_INVALID_ARG;
  }
  std::memset(p, 0, sizeof(*p));
  p->struct_size = (int32_t)sizeof(h2ulv_params);
  p->kernel = H2ULV_LAPLACE;
  p->alpha = 0.0;
  p->diag = 1e3;
  p->eta = 1.0;
  p->leaf_size = 256;
  p->rank_cap = 0;
  p->tol = 1e-8;
  p->far_sample = 32;
  p->precision = H2ULV_FP64;
  p->verbose = 0;
  p->oversample = 8;
  p->rank_model = nullptr;
  p->sketch_seed = 0;
  p->fill_in = 1;
  p->partition = 0;
  p->structure = 0;
  p->bases = 0;
  p->sketch_fallback = 1;
  p->sketch_min_level = 0;
  p->drift[0] = p->drift[1] = p->drift[2] = 0.0;
  return H2ULV_OK;
}

static bool bad_allocator(const h2ulv_allocator* a) {
  return a && (!a->alloc || !a->free);
}

// the factors remember the caller's allocator for the temporaries of later calls
static void keep_allocator(h2ulv_factor* f, const h2ulv_allocator* a) {
  if (f && a) {
    f->alloc = *a;
    f->has_alloc = true;
  }
}

h2ulv_status h2ulv_factorize(const double* pts, int64_t n, const h2ulv_params* params,
                             const h2ulv_allocator* alloc, void* stream, h2ulv_factor** out) {
  if (!out || bad_allocator(alloc)) {
    g_last_error = !out ? "out is NULL" : "allocator with a NULL function";
    return H2ULV_ERR_INVALID_ARG;
  }
  *out = nullptr;
  return guarded([&] {
    CacheScope cs;
    AllocScope as(alloc, stream);
    *out = factorize_impl(pts, n, params, (hipStream_t)stream);
    keep_allocator(*out, alloc);
  });
}

h2ulv_status h2ulv_factorize_batch(int32_t nprob, const double* const* pts, const int64_t* n,
                                   const h2ulv_params* params, const h2ulv_allocator* alloc,
                                   void* stream, h2ulv_factor** out) {
  if (nprob < 1 || !pts || !n || !out || bad_allocator(alloc)) {
    g_last_error = "bad batch arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  for (int p = 0; p < nprob; ++p) out[p] = nullptr;
  h2ulv_status st = guarded([&] {
    CacheScope cs;
    AllocScope as(alloc, stream);
    if (!params) fail(H2ULV_ERR_INVALID_ARG, "params is NULL");
    validate_params(params);
    std::vector<const double*> pv(pts, pts + nprob);
    std::vector<int64_t> nv(n, n + nprob);
    std::vector<h2ulv_factor*> fs = factorize_many(pv, nv, *params, (hipStream_t)stream);
    for (int p = 0; p < nprob; ++p) {
      out[p] = fs[p];
      keep_allocator(out[p], alloc);
    }
  });
  if (st != H2ULV_OK)
    for (int p = 0; p < nprob; ++p) {
      delete out[p];
      out[p] = nullptr;
    }
  return st;
}

h2ulv_status h2ulv_solve(const h2ulv_factor* f, double* b, int32_t nrhs, int64_t ldb,
                         void* stream) {
  if (!f || !b || nrhs < 1 || ldb < f->n) {
    g_last_error = "bad solve arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    CacheScope cs;
    AllocScope as(f->has_alloc ? &f->alloc : nullptr, stream);
    solve_impl(*f, b, nrhs, ldb, (hipStream_t)stream);
  });
}

h2ulv_status h2ulv_solve_repeated(const h2ulv_factor* f, double* b, int32_t nrhs, int64_t ldb,
                                  void* stream) {
  if (!f || !b || nrhs < 1 || ldb < f->n) {
    g_last_error = "bad solve arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    CacheScope cs;
    AllocScope as(f->has_alloc ? &f->alloc : nullptr, stream);
    solve_graph(*f, b, nrhs, ldb, (hipStream_t)stream);
  });
}

h2ulv_status h2ulv_matvec_exact(const h2ulv_factor* f, const double* x, int64_t ldx, double* y,
                                int64_t ldy, int32_t nrhs, void* stream) {
  if (!f || !x || !y || nrhs < 1 || ldx < f->n || ldy < f->n) {
    g_last_error = "bad matvec arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    AllocScope as(f->has_alloc ? &f->alloc : nullptr, stream);
    matvec_impl(*f, x, ldx, y, ldy, nrhs, (hipStream_t)stream);
  });
}

h2ulv_status h2ulv_matvec_exact_noalloc(const h2ulv_factor* f, const double* x, int64_t ldx,
                                        double* y, int64_t ldy, int32_t nrhs, void* stream) {
  if (!f || !x || !y || nrhs < 1 || ldx < f->n || ldy < f->n) {
    g_last_error = "bad matvec arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] { matvec_noalloc(*f, x, ldx, y, ldy, nrhs, (hipStream_t)stream); });
}

h2ulv_status h2ulv_refine(const h2ulv_factor* f, const double* b, int64_t ldb, double* x,
                          int64_t ldx, int32_t nrhs, double rtol, int32_t max_iter,
                          int32_t* iters, double* relres, void* stream) {
  if (!f || !b || !x || nrhs < 1 || ldb < f->n || ldx < f->n || !(rtol >= 0) || max_iter < 0) {
    g_last_error = "bad refine arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  h2ulv_status out = H2ULV_OK;
  h2ulv_status st = guarded([&] {
    CacheScope cs;
    AllocScope as(f->has_alloc ? &f->alloc : nullptr, stream);
    out = refine_impl(*f, b, ldb, x, ldx, nrhs, rtol, max_iter, iters, relres,
                      (hipStream_t)stream);
  });
  return st != H2ULV_OK ? st : out;
}

h2ulv_status h2ulv_refine_gmres(const h2ulv_factor* f, const double* b, int64_t ldb, double* x,
                                int64_t ldx, int32_t nrhs, double rtol, int32_t max_iter,
                                int32_t restart, int32_t* iters, double* relres, void* stream) {
  if (!f || !b || !x || nrhs < 1 || ldb < f->n || ldx < f->n || !(rtol >= 0) || max_iter < 0 ||
      restart < 1) {
    g_last_error = "bad GMRES arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  h2ulv_status out = H2ULV_OK;
  h2ulv_status st = guarded([&] {
    CacheScope cs;
    AllocScope as(f->has_alloc ? &f->alloc : nullptr, stream);
    out = gmres_impl(*f, b, ldb, x, ldx, nrhs, rtol, max_iter, restart, iters, relres,
                     (hipStream_t)stream);
  });
  return st != H2ULV_OK ? st : out;
}

h2ulv_status h2ulv_refine_block_gmres(const h2ulv_factor* f, const double* b, int64_t ldb,
                                      double* x, int64_t ldx, int32_t nrhs, double rtol,
                                      int32_t max_iter, int32_t restart, int32_t* iters,
                                      double* relres, void* stream) {
  if (!f || !b || !x || nrhs < 1 || ldb < f->n || ldx < f->n || !(rtol >= 0) || max_iter < 0 ||
      restart < 1) {
    g_last_error = "bad GMRES arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  h2ulv_status out = H2ULV_OK;
  h2ulv_status st = guarded([&] {
    CacheScope cs;
    AllocScope as(f->has_alloc ? &f->alloc : nullptr, stream);
    out = block_gmres_impl(*f, b, ldb, x, ldx, nrhs, rtol, max_iter, restart, iters, relres,
                           (hipStream_t)stream);
  });
  return st != H2ULV_OK ? st : out;
}

h2ulv_status h2ulv_get_stats(const h2ulv_factor* f, h2ulv_stats* s) {
  if (!f || !s) {
    g_last_error = "NULL argument";
    return H2ULV_ERR_INVALID_ARG;
  }
  *s = f->stats;
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_levels(const h2ulv_factor* f, int32_t* L) {
  if (!f || !L) return H2ULV_ERR_INVALID_ARG;
  *L = f->tree.L;
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_perm(const h2ulv_factor* f, int64_t* perm) {
  if (!f || !perm) return H2ULV_ERR_INVALID_ARG;
  std::memcpy(perm, f->tree.perm.data(), f->n * sizeof(int64_t));
  return H2ULV_OK;
}

// levels that hold a factorization: 1..L, or only L for the flat structure
static bool factored_level(const h2ulv_factor* f, int32_t lev) {
  return f && lev >= 1 && lev <= f->tree.L && (f->p.structure == 0 || lev == f->tree.L);
}

h2ulv_status h2ulv_get_ranks(const h2ulv_factor* f, int32_t lev, int32_t* m, int32_t* k) {
  if (!factored_level(f, lev)) {
    g_last_error = "bad level";
    return H2ULV_ERR_INVALID_ARG;
  }
  const LevelFactor& lf = f->levels[lev];
  for (int i = 0; i < lf.nb; ++i) {
    if (m) m[i] = lf.m[i];
    if (k) k[i] = lf.k[i];
  }
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_skeleton(const h2ulv_factor* f, int32_t lev, int32_t box, int64_t* sk) {
  if (!sk || !factored_level(f, lev) || box < 0 || box >= (1 << lev)) {
    g_last_error = "bad level or box";
    return H2ULV_ERR_INVALID_ARG;
  }
  const auto& v = f->levels[lev].sk[box];
  std::copy(v.begin(), v.end(), sk);
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_column_skeleton(const h2ulv_factor* f, int32_t lev, int32_t box,
                                        int64_t* sk) {
  if (f && !f->colview) return h2ulv_get_skeleton(f, lev, box, sk);
  if (!sk || !factored_level(f, lev) || box < 0 || box >= (1 << lev)) {
    g_last_error = "bad level or box";
    return H2ULV_ERR_INVALID_ARG;
  }
  const auto& v = f->colview->levels[lev].sk[box];
  std::copy(v.begin(), v.end(), sk);
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_column_basis(const h2ulv_factor* f, int32_t lev, int32_t box, double* V) {
  if (f && !f->colview) return h2ulv_get_basis(f, lev, box, V);
  if (!V || !factored_level(f, lev) || box < 0 || box >= (1 << lev)) {
    g_last_error = "bad level or box";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    const LevelFactor& lf = f->colview->levels[lev];
    int64_t mm = (int64_t)lf.m[box] * lf.m[box];
    if (mm == 0) return;
    H2ULV_HIP(hipMemcpy(V, lf.U.as<double>() + lf.offU[box], mm * sizeof(double),
                        hipMemcpyDeviceToHost));
  });
}

h2ulv_status h2ulv_get_basis(const h2ulv_factor* f, int32_t lev, int32_t box, double* U) {
  if (!U || !factored_level(f, lev) || box < 0 || box >= (1 << lev)) {
    g_last_error = "bad level or box";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    const LevelFactor& lf = f->levels[lev];
    int64_t mm = (int64_t)lf.m[box] * lf.m[box];
    if (mm == 0) return;
    H2ULV_HIP(hipMemcpy(U, lf.U.as<double>() + lf.offU[box], mm * sizeof(double),
                        hipMemcpyDeviceToHost));
  });
}

void h2ulv_destroy(h2ulv_factor* f) { delete f; }

h2ulv_status h2ulv_structure_create(const double* pts, int64_t n, const h2ulv_params* params,
                                    h2ulv_structure** out) {
  if (!out) return H2ULV_ERR_INVALID_ARG;
  *out = nullptr;
  return guarded([&] {
    validate_params(params);
    if (!pts || n < 1) fail(H2ULV_ERR_INVALID_ARG, "bad points");
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(pts[i])) fail(H2ULV_ERR_INVALID_ARG, "non-finite point coordinate");
    auto s = std::make_unique<h2ulv_structure>();
    s->tree = build_tree(pts, n, params->leaf_size, params->partition);
    s->lists = build_structure_lists(s->tree, *params);
    *out = s.release();
  });
}

h2ulv_status h2ulv_structure_levels(const h2ulv_structure* s, int32_t* L) {
  if (!s || !L) return H2ULV_ERR_INVALID_ARG;
  *L = s->tree.L;
  return H2ULV_OK;
}

h2ulv_status h2ulv_structure_perm(const h2ulv_structure* s, int64_t* perm) {
  if (!s || !perm) return H2ULV_ERR_INVALID_ARG;
  std::memcpy(perm, s->tree.perm.data(), s->tree.n * sizeof(int64_t));
  return H2ULV_OK;
}

h2ulv_status h2ulv_structure_lists(const h2ulv_structure* s, int32_t lev, int64_t* near_ptr,
                                   int32_t* near_idx, int64_t* far_ptr, int32_t* far_idx) {
  if (!s || lev < 0 || lev > s->tree.L) return H2ULV_ERR_INVALID_ARG;
  const Lists& ls = s->lists;
  if (near_ptr) std::copy(ls.near_ptr[lev].begin(), ls.near_ptr[lev].end(), near_ptr);
  if (far_ptr) std::copy(ls.far_ptr[lev].begin(), ls.far_ptr[lev].end(), far_ptr);
  if (near_idx) std::copy(ls.near_idx[lev].begin(), ls.near_idx[lev].end(), near_idx);
  if (far_idx) std::copy(ls.far_idx[lev].begin(), ls.far_idx[lev].end(), far_idx);
  return H2ULV_OK;
}

h2ulv_status h2ulv_structure_geometry(const h2ulv_structure* s, int32_t lev, double* centre,
                                      double* radius) {
  if (!s || lev < 0 || lev > s->tree.L) return H2ULV_ERR_INVALID_ARG;
  if (centre) std::copy(s->tree.centre[lev].begin(), s->tree.centre[lev].end(), centre);
  if (radius) std::copy(s->tree.radius[lev].begin(), s->tree.radius[lev].end(), radius);
  return H2ULV_OK;
}

void h2ulv_structure_destroy(h2ulv_structure* s) { delete s; }

h2ulv_status h2ulv_rankmodel_create(uint64_t seed, h2ulv_rankmodel** out) {
  if (!out) {
    g_last_error = "out is NULL";
    return H2ULV_ERR_INVALID_ARG;
  }
  *out = nullptr;
  return guarded([&] { *out = rankmodel_create(seed); });
}

void h2ulv_rankmodel_destroy(h2ulv_rankmodel* m) { delete m; }

h2ulv_status h2ulv_rankmodel_set_params(h2ulv_rankmodel* m, const float* host) {
  if (!m || !host) {
    g_last_error = "NULL argument";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    H2ULV_HIP(hipMemcpy(m->theta.p, host, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  });
}

h2ulv_status h2ulv_rankmodel_get_params(const h2ulv_rankmodel* m, float* host) {
  if (!m || !host) {
    g_last_error = "NULL argument";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    H2ULV_HIP(hipMemcpy(host, m->theta.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  });
}

// Rank model file: the 4 bytes "H2RM", the format version and the parameter
// count (uint32 each), the Adam step count (int64), then the parameters and
// the two Adam moments (H2ULV_MLP_NPARAM float32 each), in host byte order.
namespace {
constexpr char RM_MAGIC[4] = {'H', '2', 'R', 'M'};
constexpr uint32_t RM_VERSION = 1;
using FileHandle = std::unique_ptr<FILE, int (*)(FILE*)>;
}  // namespace

h2ulv_status h2ulv_rankmodel_save(const h2ulv_rankmodel* m, const char* path) {
  if (!m || !path) {
    g_last_error = "NULL argument";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    const size_t np = MLP_NPARAM;
    std::vector<float> buf(3 * np);
    H2ULV_HIP(hipMemcpy(buf.data(), m->theta.p, np * sizeof(float), hipMemcpyDeviceToHost));
    H2ULV_HIP(hipMemcpy(buf.data() + np, m->m.p, np * sizeof(float), hipMemcpyDeviceToHost));
    H2ULV_HIP(hipMemcpy(buf.data() + 2 * np, m->v.p, np * sizeof(float), hipMemcpyDeviceToHost));
    FileHandle f(std::fopen(path, "wb"), &std::fclose);
    if (!f) fail(H2ULV_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
    const uint32_t head[2] = {RM_VERSION, (uint32_t)np};
    const int64_t step = m->step;
    bool ok = std::fwrite(RM_MAGIC, 1, 4, f.get()) == 4 &&
              std::fwrite(head, sizeof(uint32_t), 2, f.get()) == 2 &&
              std::fwrite(&step, sizeof(int64_t), 1, f.get()) == 1 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f.get()) == buf.size();
    ok = (std::fclose(f.release()) == 0) && ok;
    if (!ok) fail(H2ULV_ERR_INVALID_ARG, std::string("writing ") + path + " failed");
  });
}

h2ulv_status h2ulv_rankmodel_load(const char* path, h2ulv_rankmodel** out) {
  if (!path || !out) {
    g_last_error = "NULL argument";
    return H2ULV_ERR_INVALID_ARG;
  }
  *out = nullptr;
  return guarded([&] {
    FileHandle f(std::fopen(path, "rb"), &std::fclose);
    if (!f) fail(H2ULV_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char magic[4];
    uint32_t head[2];
    int64_t step = 0;
    const size_t np = MLP_NPARAM;
    if (std::fread(magic, 1, 4, f.get()) != 4 || std::memcmp(magic, RM_MAGIC, 4) != 0)
      fail(H2ULV_ERR_INVALID_ARG, std::string(path) + " is not a rank model file");
    if (std::fread(head, sizeof(uint32_t), 2, f.get()) != 2 || head[0] != RM_VERSION ||
        head[1] != (uint32_t)np)
      fail(H2ULV_ERR_INVALID_ARG, std::string(path) + ": unsupported version or parameter count");
    std::vector<float> buf(3 * np);
    if (std::fread(&step, sizeof(int64_t), 1, f.get()) != 1 || step < 0 ||
        std::fread(buf.data(), sizeof(float), buf.size(), f.get()) != buf.size() ||
        std::fgetc(f.get()) != EOF)
      fail(H2ULV_ERR_INVALID_ARG, std::string(path) + ": truncated or oversized rank model file");
    std::unique_ptr<h2ulv_rankmodel> M(rankmodel_create(0));
    H2ULV_HIP(hipMemcpy(M->theta.p, buf.data(), np * sizeof(float), hipMemcpyHostToDevice));
    H2ULV_HIP(hipMemcpy(M->m.p, buf.data() + np, np * sizeof(float), hipMemcpyHostToDevice));
    H2ULV_HIP(hipMemcpy(M->v.p, buf.data() + 2 * np, np * sizeof(float), hipMemcpyHostToDevice));
    M->step = step;
    *out = M.release();
  });
}

h2ulv_status h2ulv_rankmodel_forward(const h2ulv_rankmodel* m, const float* feat, int64_t n,
                                     float* y, void* stream) {
  if (!m || n < 0 || (n > 0 && (!feat || !y))) {
    g_last_error = "bad forward arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    launch_mlp_forward(m->theta.as<float>(), feat, n, y, (hipStream_t)stream);
    H2ULV_HIP(hipGetLastError());
  });
}

h2ulv_status h2ulv_rankmodel_gradient(const h2ulv_rankmodel* m, const float* feat,
                                      const float* target, int64_t n, float* grad, float* loss,
                                      void* stream) {
  if (!m || n < 1 || !feat || !target || !grad) {
    g_last_error = "bad gradient arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    CacheScope cs;
    rankmodel_gradient(*m, feat, target, n, grad, loss, (hipStream_t)stream);
  });
}

h2ulv_status h2ulv_rankmodel_adam_step(h2ulv_rankmodel* m, const float* grad, float lr,
                                       void* stream) {
  if (!m || !grad || !(lr >= 0.0f)) {
    g_last_error = "bad Adam arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] { rankmodel_adam(*m, grad, lr, (hipStream_t)stream); });
}

h2ulv_status h2ulv_rankmodel_train(h2ulv_rankmodel* m, const float* feat, const float* target,
                                   int64_t n, int32_t steps, float lr, float* loss, void* stream) {
  if (!m || n < 1 || !feat || !target || steps < 0 || !(lr >= 0.0f)) {
    g_last_error = "bad training arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    CacheScope cs;
    rankmodel_train(*m, feat, target, n, steps, lr, loss, (hipStream_t)stream);
  });
}

h2ulv_status h2ulv_get_features(const h2ulv_factor* f, int32_t lev, float* feat, float* target) {
  if (!factored_level(f, lev)) {
    g_last_error = "bad level";
    return H2ULV_ERR_INVALID_ARG;
  }
  const LevelFactor& lf = f->levels[lev];
  if (feat) std::copy(lf.feat.begin(), lf.feat.end(), feat);
  if (target)
    for (int i = 0; i < lf.nb; ++i) target[i] = (float)std::log2(1.0 + lf.k[i]);
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_sketch_info(const h2ulv_factor* f, int32_t lev, int32_t* khat,
                                   int32_t* ell, int32_t* state) {
  if (!factored_level(f, lev)) {
    g_last_error = "bad level";
    return H2ULV_ERR_INVALID_ARG;
  }
  const LevelFactor& lf = f->levels[lev];
  for (int i = 0; i < lf.nb; ++i) {
    if (khat) khat[i] = lf.khat[i];
    if (ell) ell[i] = lf.ell[i];
    if (state) state[i] = lf.sk_state[i];
  }
  return H2ULV_OK;
}

h2ulv_status h2ulv_release_cache(void) {
  return guarded([&] {
    H2ULV_HIP(hipDeviceSynchronize());
    cache_release();
  });
}

const char* h2ulv_status_string(h2ulv_status s) {
  switch (s) {
    case H2ULV_OK: return "ok";
    case H2ULV_ERR_INVALID_ARG: return "invalid argument";
    case H2ULV_ERR_OOM: return "out of memory";
    case H2ULV_ERR_HIP: return "HIP runtime error";
    case H2ULV_ERR_SINGULAR: return "singular block";
    case H2ULV_ERR_DUPLICATE_POINTS: return "duplicate points";
    case H2ULV_ERR_NOT_CONVERGED: return "refinement not converged";
    case H2ULV_ERR_RANK_CHECK: return "sketched basis rejected (no fallback)";
  }
  return "unknown status";
}

const char* h2ulv_last_error(void) { return g_last_error.c_str(); }

h2ulv_status h2ulv_profile_enable(int32_t on) {
  return guarded([&] {
    Profiler& p = profiler();
    for (auto& r : p.recs) {
      p.pool.push_back(r.a);
      p.pool.push_back(r.b);
    }
    p.recs.clear();
    p.on = on != 0;
    // create the events up front: hipEventCreate inside the measured work would
    // add its own cost to every recorded launch
    if (p.on)
      while (p.pool.size() < 65536) {
        hipEvent_t e;
        H2ULV_HIP(hipEventCreate(&e));
        p.pool.push_back(e);
      }
  });
}

h2ulv_status h2ulv_gemm_tile_rates(double* out) {
  if (!out) {
    g_last_error = "out is NULL";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] { (void)gemm_tile_rates_known(out); });
}

h2ulv_status h2ulv_profile_read(h2ulv_kernel_profile* out, int32_t max, int32_t* count) {
  if (!count || (max > 0 && !out)) {
    g_last_error = "bad profile arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] {
    Profiler& p = profiler();
    std::vector<std::string> names;
    std::map<std::string, h2ulv_kernel_profile> agg;
    for (auto& r : p.recs) {
      H2ULV_HIP(hipEventSynchronize(r.b));
      float ms = 0;
      H2ULV_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      auto it = agg.find(r.name);
      if (it == agg.end()) {
        h2ulv_kernel_profile z{};
        std::snprintf(z.name, sizeof(z.name), "%s", r.name);
        it = agg.emplace(r.name, z).first;
        names.push_back(r.name);
      }
      it->second.launches += 1;
      it->second.time_ms += ms;
      it->second.flops += r.flops;
      it->second.bytes += r.bytes;
      p.pool.push_back(r.a);
      p.pool.push_back(r.b);
    }
    p.recs.clear();
    int c = 0;
    for (auto& nm : names) {
      if (c < max) out[c] = agg[nm];
      ++c;
    }
    *count = c;
  });
}

}  // extern "C"
