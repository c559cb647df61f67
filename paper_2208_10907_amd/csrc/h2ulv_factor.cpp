// H^2-ULV factorization without trailing sub-matrix dependencies: the batched
// level driver.  Each level of the tree is one batched pass over all of its
// boxes (Sec. III of Ma, Deshmukh, Yokota, arXiv 2208.10907), and several
// independent problems go through the same launches: problems are aligned by
// height above their leaves, and every phase of a level gathers the work items
// of all problems of the group before it launches.
//   (a) dense blocks of the inadmissible pairs (leaf: kernel evaluation; upper
//       levels: the children's skeleton blocks merged 2 x 2, Sec. II-C);
//   (b) fill-ins F_ij = sum_k D_ik D_kk^-1 D_kj into every reachable (i, j),
//       from one inverse per diagonal block (Sec. III-B);
//   (c) shared basis from M'_i = [K(P_i, far) | T^-1 F_i+] (Sec. III-C,
//       Eq. fillu): tall Householder QR, column-pivoted QR of its triangle,
//       row ID W', and the orthogonal factor of W = T W' (Sec. II-A);
//   (d) low-rank couplings S_ij = T_i K(sk_i, sk_j) T_j^T (Eq. ss);
//   (e) rotation S_ii = U_i^T D_ii U_i and S^SS_ij = U^S_i^T D_ij U^S_j (Eq. rs);
//   (f) elimination of the redundant part: inverse of S^RR, S^RR^-1 S^RS and
//       the Schur update S^SS - S^SR S^RR^-1 S^RS (Sec. II-B, Eq. lu ff.);
// then the root blocks are inverted (Eq. BLR2final).  Ranks are read back once
// per level to size the next level.
#include "h2ulv_factor.h"
#include "h2ulv_learned.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <numeric>

namespace h2ulv {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

KernelFn kfn(const h2ulv_params& p) {
  return KernelFn{p.kernel, p.alpha, p.diag, {p.drift[0], p.drift[1], p.drift[2]}};
}

namespace {

// float copy of a device array (mixed precision: operands of the FP32 products)
DBuf to_f32(const double* src, int64_t count, hipStream_t s) {
  DBuf b(std::max<int64_t>(count, 1) * sizeof(float));
  launch_convert_d2f(src, b.as<float>(), count, s);
  H2ULV_HIP(hipGetLastError());
  return b;
}

// far-field column indices of box i at level lev: exact = every point outside
// the near boxes; sampled = all candidate rows of the own-level far boxes +
// strided samples of the ancestors' far boxes (all points of a box holding at
// most s points).
std::vector<int64_t> far_columns(const Tree& t, const Lists& ls, int lev, int i,
                                 const std::vector<std::vector<int64_t>>& cand, int s) {
  std::vector<int64_t> out;
  if (s == 0) {
    std::vector<char> mask(t.n, 1);
    for (int64_t e = ls.near_ptr[lev][i]; e < ls.near_ptr[lev][i + 1]; ++e) {
      int j = ls.near_idx[lev][e];
      for (int64_t a = t.start[lev][j]; a < t.end[lev][j]; ++a) mask[a] = 0;
    }
    for (int64_t a = 0; a < t.n; ++a)
      if (mask[a]) out.push_back(t.perm[a]);
    return out;
  }
  for (int64_t e = ls.far_ptr[lev][i]; e < ls.far_ptr[lev][i + 1]; ++e) {
    int q = ls.far_idx[lev][e];
    out.insert(out.end(), cand[q].begin(), cand[q].end());
  }
  int a = i;
  for (int la = lev - 1; la >= 1; --la) {
    a >>= 1;
    for (int64_t e = ls.far_ptr[la][a]; e < ls.far_ptr[la][a + 1]; ++e) {
      int q = ls.far_idx[la][e];
      int64_t s0 = t.start[la][q], nq = t.end[la][q] - s0;
      if (nq <= s) {
        for (int64_t u = 0; u < nq; ++u) out.push_back(t.perm[s0 + u]);
      } else {
        for (int u = 0; u < s; ++u) out.push_back(t.perm[s0 + (int64_t)((u + 0.5) * nq / s)]);
      }
    }
  }
  return out;
}

std::vector<int> fill_targets(const Lists& ls, int lev, int i) {
  std::vector<int> js;
  for (int64_t e = ls.near_ptr[lev][i]; e < ls.near_ptr[lev][i + 1]; ++e) {
    int k = ls.near_idx[lev][e];
    if (k == i) continue;
    for (int64_t f = ls.near_ptr[lev][k]; f < ls.near_ptr[lev][k + 1]; ++f) {
      int j = ls.near_idx[lev][f];
      if (j != k) js.push_back(j);
    }
  }
  std::sort(js.begin(), js.end());
  js.erase(std::unique(js.begin(), js.end()), js.end());
  return js;
}

int64_t csr_find(const std::vector<int64_t>& ptr, const std::vector<int32_t>& idx, int i, int j) {
  auto b = idx.begin() + ptr[i], e = idx.begin() + ptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it != e && *it == j) return it - idx.begin();
  return -1;
}

void check_info(const int32_t* dinfo, size_t n, hipStream_t s, const char* what) {
  if (!dinfo || n == 0) return;
  std::vector<int32_t> h(n);
  H2ULV_HIP(hipMemcpyAsync(h.data(), dinfo, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i)
    if (h[i] != 0)
      fail(H2ULV_ERR_SINGULAR, std::string("zero or non-finite pivot in ") + what);
}

// One problem of the batch: its factor, its place in the shared point buffer
// and the state of the level being factored.
struct Prob {
  h2ulv_factor* F = nullptr;
  // separate bases: the row side (colside false) and the column side (the
  // transposed matrix, colside true) of one problem point at each other
  Prob* partner = nullptr;
  bool colside = false;
  int64_t poff = 0;  // offset of its points in the shared point buffer
  double fl_fill = 0, fl_basis = 0, fl_couple = 0, fl_rotate = 0, fl_elim = 0, fl_root = 0,
         kevals = 0;

  // skeleton blocks of the level just finished, keyed by CSR position (near
  // pairs, then far pairs)
  DBuf Shat;
  std::vector<int64_t> shat_near_off, shat_far_off;

  // level state
  int lev = 0, nb = 0;
  std::vector<int64_t> cand_all, cand_off;
  DBuf dcand;
  std::vector<int64_t> Doff, offSq, offTinv, offW, ncols;
  DBuf D, Dinv, Tinv, Z, D32, Z32, PQ, pivd, kd, S;
  std::vector<std::vector<int>> targets;
  std::vector<std::vector<int64_t>> farcols;
  std::vector<int64_t> far_off;  // box i's far columns at dfar + far_off[i]
  DBuf dfar;
  double* PQ0 = nullptr;  // separate bases: copy of PQ before pivoting (row_ids only)
  std::vector<const double*> Eptr;  // E = R11^-1 R12 of each box and its leading dimension
  std::vector<int64_t> ldE;
  std::vector<DBuf> Ebufs;

  int L() const { return F->tree.L; }
  LevelFactor& lf() { return F->levels[lev]; }
  // the level factor holding the right-hand (column) bases of this level
  LevelFactor& rlf() { return partner && !colside ? partner->lf() : lf(); }
  const std::vector<int64_t>& np() const { return F->lists.near_ptr[lev]; }
  const std::vector<int32_t>& ni() const { return F->lists.near_idx[lev]; }
  const std::vector<int64_t>& fp() const { return F->lists.far_ptr[lev]; }
  const std::vector<int32_t>& fi() const { return F->lists.far_idx[lev]; }
  int64_t nnear() const { return np()[nb]; }
  int64_t nfar() const { return fp()[nb]; }
  const int64_t* candp(int i) const { return dcand.as<int64_t>() + cand_off[i]; }
  const int64_t* farp(int i) const { return dfar.as<int64_t>() + far_off[i]; }
  double* Dblk(int i, int j) { return D.as<double>() + Doff[csr_find(np(), ni(), i, j)]; }

  const double* shat_block(int clev, int c, int d, int64_t* ld) {
    const Lists& ls = F->lists;
    *ld = F->levels[clev].k[c];
    int64_t e = csr_find(ls.near_ptr[clev], ls.near_idx[clev], c, d);
    if (e >= 0) return Shat.as<double>() + shat_near_off[e];
    e = csr_find(ls.far_ptr[clev], ls.far_idx[clev], c, d);
    if (e < 0) fail(H2ULV_ERR_HIP, "internal: child pair is neither near nor far");
    return Shat.as<double>() + shat_far_off[e];
  }

  // device bytes the level's transient buffers need at their peak (dense
  // blocks, their fill-in products and the per-box square workspaces)
  double level_bytes(bool mixed) const {
    const auto& m = F->levels[lev].cand;
    double dw = 0, sq = 0;
    for (int i = 0; i < nb; ++i) {
      double mi = (double)m[i].size();
      sq += mi * mi;
      for (int64_t e = np()[i]; e < np()[i + 1]; ++e) dw += mi * (double)m[ni()[e]].size();
    }
    return 8.0 * (3.0 * dw + 4.0 * sq) + (mixed ? 8.0 * dw : 0.0);
  }

  void end_level() {
    cand_all.clear();
    cand_off.clear();
    Doff.clear();
    offSq.clear();
    offTinv.clear();
    offW.clear();
    ncols.clear();
    targets.clear();
    farcols.clear();
    far_off.clear();
    Eptr.clear();
    ldE.clear();
    Ebufs.clear();
    for (DBuf* b : {&dcand, &dfar, &D, &Dinv, &Tinv, &Z, &D32, &Z32, &PQ, &pivd, &kd, &S})
      b->reset();
  }
};

struct Box {
  Prob* P;
  int i;
};

struct Driver {
  hipStream_t s;
  h2ulv_params p;
  KernelFn kf;
  bool mixed;
  // mixed precision with a rank cap: the fill-in products run in FP32 as well
  // (the cap bounds the basis, so FP32 rounding of M' cannot inflate ranks)
  bool fill32;
  const double* pts = nullptr;  // shared points of all problems (n x 3 each)
  DBuf dupbuf;
  int* dup = nullptr;

  // per-step wall times (verbose mode synchronises at each step)
  std::map<std::string, double> step_time;
  double t_last = 0;

  Driver(hipStream_t st, const h2ulv_params& pr)
      : s(st),
        p(pr),
        kf(kfn(pr)),
        mixed(pr.precision == H2ULV_MIXED),
        fill32(pr.precision == H2ULV_MIXED && pr.rank_cap > 0) {
    dupbuf.alloc(sizeof(int));
    dup = dupbuf.as<int>();
    H2ULV_HIP(hipMemsetAsync(dup, 0, sizeof(int), s));
  }

  // host-only time of a section (verbose mode)
  void htime(const char* name, double t0) {
    if (p.verbose) step_time[name] += now_s() - t0;
  }

  void tick(const char* name) {
    if (!p.verbose) return;
    H2ULV_HIP(hipStreamSynchronize(s));
    double t = now_s();
    if (name) step_time[name] += t - t_last;
    t_last = t;
  }

  void check_dup() {
    int h = 0;
    H2ULV_HIP(hipMemcpyAsync(&h, dup, sizeof(int), hipMemcpyDeviceToHost, s));
    H2ULV_HIP(hipStreamSynchronize(s));
    if (h) fail(H2ULV_ERR_DUPLICATE_POINTS, "two distinct points coincide");
  }

  void level(const std::vector<Prob*>& G);
  void roots(const std::vector<Prob*>& G);

 private:
  void dense_blocks(Stage& st, const std::vector<Prob*>& G);
  void fill_products(Stage& st, const std::vector<Prob*>& G);
  void basis_prepare(Stage& st, const std::vector<Prob*>& G);
  void fill_z(Stage& st, const std::vector<Box>& boxes);
  // rebuild: boxes whose sketch was rejected, sketched again at full width or
  // given their M' (kernel entries are not counted again)
  void build_triangles(Stage& st, const std::vector<Box>& boxes, bool rebuild = false);
  void build_sketch(Stage& st, const std::vector<Box>& boxes, bool rebuild);
  // force: per box of `boxes`, keep exactly that many pivots (tol 0, cap = it)
  void pivot_boxes(Stage& st, const std::vector<Box>& boxes,
                   const std::vector<int>* force = nullptr);
  void couple_ranks(Stage& st, const std::vector<Prob*>& G);
  std::vector<Box> check_sketches(Stage& st, const std::vector<Box>& boxes);
  void row_ids(Stage& st, const std::vector<Prob*>& G);
  void bases(Stage& st, const std::vector<Prob*>& G);
  void couplings(Stage& st, const std::vector<Prob*>& G);
  void rotations(Stage& st, const std::vector<Prob*>& G);
  void elimination(Stage& st, const std::vector<Prob*>& G);
};

// ---- (a) dense blocks ---------------------------------------------------------
void Driver::dense_blocks(Stage& st, const std::vector<Prob*>& G) {
  KgenBatch kb;
  CopyBatch cb;
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const int nb = P->nb;
    const std::vector<int>& m = lf.m;
    const auto& np = P->np();
    const auto& ni = P->ni();
    const int64_t nnear = P->nnear();
    P->Doff.assign(nnear + 1, 0);
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e)
        P->Doff[e + 1] = P->Doff[e] + (int64_t)m[i] * m[ni[e]];
    P->D.alloc(std::max<int64_t>(P->Doff[nnear], 1) * sizeof(double));
    double* Dp = P->D.as<double>();
    if (P->colside) continue;  // transposed copies of the row side's blocks, below
    if (P->lev == P->L()) {
      for (int i = 0; i < nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e) {
          int j = ni[e];
          kb.add(P->candp(i), m[i], P->candp(j), m[j], Dp + P->Doff[e], m[i]);
          P->kevals += (double)m[i] * m[j];
        }
    } else {
      const std::vector<int>& kc = P->F->levels[P->lev + 1].k;
      for (int i = 0; i < nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e) {
          int j = ni[e];
          double* out = Dp + P->Doff[e];
          int rows[2] = {2 * i, 2 * i + 1}, cols[2] = {2 * j, 2 * j + 1};
          int ro = 0;
          for (int a = 0; a < 2; ++a) {
            int co = 0;
            for (int b = 0; b < 2; ++b) {
              int64_t ld;
              const double* src = P->shat_block(P->lev + 1, rows[a], cols[b], &ld);
              cb.add(src, std::max<int64_t>(ld, 1), out + ro + (int64_t)co * m[i], m[i],
                     kc[rows[a]], kc[cols[b]]);
              co += kc[cols[b]];
            }
            ro += kc[rows[a]];
          }
        }
    }
  }
  kb.run(st, pts, kf, dup);
  cb.run(st);
  // the column side works on A^T: D'_ij = D_ji^T, i.e. the leaf blocks of the
  // row side transposed, and above the leaves the children's S^SS blocks of
  // the row side transposed
  CopyBatch ct;
  for (Prob* P : G) {
    if (!P->colside) continue;
    Prob* R = P->partner;
    const std::vector<int>& m = P->lf().m;
    const auto& np = P->np();
    const auto& ni = P->ni();
    double* Dp = P->D.as<double>();
    for (int i = 0; i < P->nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        const int j = ni[e];
        if (P->lev == P->L()) {
          ct.add(R->Dblk(j, i), std::max(m[j], 1), Dp + P->Doff[e], std::max(m[i], 1), m[i],
                 m[j], true);
          continue;
        }
        const std::vector<int>& kc = P->F->levels[P->lev + 1].k;
        int ro = 0;
        for (int a = 0; a < 2; ++a) {
          const int c = 2 * i + a;
          int co = 0;
          for (int b = 0; b < 2; ++b) {
            const int d = 2 * j + b;
            if (kc[c] > 0 && kc[d] > 0) {
              int64_t ld;
              const double* src = R->shat_block(P->lev + 1, d, c, &ld);
              ct.add(src, std::max<int64_t>(ld, 1), Dp + P->Doff[e] + ro + (int64_t)co * m[i],
                     std::max(m[i], 1), kc[c], kc[d], true);
            }
            co += kc[d];
          }
          ro += kc[c];
        }
      }
  }
  ct.run(st);
  st.sync();
  for (Prob* P : G) P->Shat.reset();  // children's skeleton blocks are merged now
}

// ---- (b) fill-ins: inverses of the diagonal blocks and Z'_ik = T^-1 D_ik D_kk^-1
void Driver::fill_products(Stage& st, const std::vector<Prob*>& G) {
  // the ablation without fill-ins in the basis has no fill-in step
  if (!p.fill_in) return;
  {
    std::vector<DBuf> LUw;
    CopyBatch cb;
    std::vector<SqMat> mats;
    for (Prob* P : G) {
      const int nb = P->nb;
      const std::vector<int>& m = P->lf().m;
      P->Dinv.alloc(std::max<int64_t>(P->offSq[nb], 1) * sizeof(double));
      LUw.emplace_back(std::max<int64_t>(P->offSq[nb], 1) * sizeof(double));
      double* W = LUw.back().as<double>();
      if (P->colside) continue;  // (D_ii^T)^-1 = (D_ii^-1)^T, copied below
      for (int i = 0; i < nb; ++i) {
        if (m[i] == 0) continue;
        cb.add(P->Dblk(i, i), m[i], W + P->offSq[i], m[i], m[i], m[i]);
        mats.push_back(SqMat{W + P->offSq[i], m[i], m[i], P->Dinv.as<double>() + P->offSq[i], m[i]});
        P->fl_fill += 2.0 / 3.0 * std::pow((double)m[i], 3);
      }
    }
    cb.run(st);
    int32_t* info = nullptr;
    batched_inverse(st, mats, &info, nullptr, nullptr);
    check_info(info, mats.size(), s, "a diagonal block (fill-in step)");
    CopyBatch ct;
    for (Prob* P : G) {
      if (!P->colside) continue;
      const std::vector<int>& m = P->lf().m;
      for (int i = 0; i < P->nb; ++i)
        if (m[i] > 0)
          ct.add(P->partner->Dinv.as<double>() + P->offSq[i], m[i],
                 P->Dinv.as<double>() + P->offSq[i], m[i], m[i], m[i], true);
    }
    ct.run(st);
    st.sync();
  }
  tick("b_inverse");
  // inverse T factors of the children (T-hat^-1 is block diagonal)
  {
    std::vector<DBuf> Tw;
    CopyBatch cb;
    std::vector<SqMat> mats;
    for (Prob* P : G) {
      if (P->lev == P->L()) continue;
      const int nb = P->nb;
      const LevelFactor& ch = P->F->levels[P->lev + 1];
      P->offTinv.assign(2 * nb + 1, 0);
      for (int c = 0; c < 2 * nb; ++c)
        P->offTinv[c + 1] = P->offTinv[c] + (int64_t)ch.k[c] * ch.k[c];
      P->Tinv.alloc(std::max<int64_t>(P->offTinv[2 * nb], 1) * sizeof(double));
      Tw.emplace_back(std::max<int64_t>(P->offTinv[2 * nb], 1) * sizeof(double));
      double* W = Tw.back().as<double>();
      for (int c = 0; c < 2 * nb; ++c) {
        if (ch.k[c] == 0) continue;
        cb.add(ch.Tt.as<double>() + ch.offT[c], ch.k[c], W + P->offTinv[c], ch.k[c], ch.k[c],
               ch.k[c]);
        mats.push_back(SqMat{W + P->offTinv[c], ch.k[c], ch.k[c],
                             P->Tinv.as<double>() + P->offTinv[c], ch.k[c]});
      }
    }
    if (!mats.empty()) {
      cb.run(st);
      batched_triu_inverse(st, mats);
      st.sync();
    }
  }
  // Z'_ik only for the boxes whose M' is formed (not sketched); D^-1 and
  // T-hat^-1 stay until the basis step has settled every box
  std::vector<Box> need;
  for (Prob* P : G)
    for (int i = 0; i < P->nb; ++i)
      if (P->lf().sk_state[i] == 0) need.push_back(Box{P, i});
  fill_z(st, need);
}

// Z'_ik = T-hat_i^-1 D_ik D_kk^-1 for k in Near(i) \ {i} of the given boxes,
// stored at the CSR position of (i, k) (the buffer is allocated on first use)
void Driver::fill_z(Stage& st, const std::vector<Box>& boxes) {
  if (boxes.empty()) return;
  std::vector<DBuf> Ztmp;
  std::map<Prob*, double*> tmp;
  GemmBatch<double> g, g2;
  for (const Box& b : boxes) {
    Prob* P = b.P;
    const int i = b.i;
    const std::vector<int>& m = P->lf().m;
    const auto& np = P->np();
    const auto& ni = P->ni();
    const bool upper = P->lev < P->L();
    const int64_t words = std::max<int64_t>(P->Doff[P->nnear()], 1);
    if (!P->Z.p) P->Z.alloc(words * sizeof(double));
    double* Zp = P->Z.as<double>();
    double* Zt = Zp;
    if (upper) {
      if (!tmp.count(P)) {
        Ztmp.emplace_back(words * sizeof(double));
        tmp[P] = Ztmp.back().as<double>();
      }
      Zt = tmp[P];
    }
    const double* Dp = P->D.as<double>();
    for (int64_t e = np[i]; e < np[i + 1]; ++e) {
      const int k = ni[e];
      if (k == i || m[i] == 0 || m[k] == 0) continue;
      g.one(Zt + P->Doff[e], m[i], m[i], m[k], m[k], Dp + P->Doff[e], m[i], false,
            P->Dinv.as<double>() + P->offSq[k], m[k], false);
      P->fl_fill += 2.0 * m[i] * (double)m[k] * m[k];
      if (!upper) continue;
      const LevelFactor& ch = P->F->levels[P->lev + 1];
      const int k1 = ch.k[2 * i], k2 = ch.k[2 * i + 1];
      const double* Ti = P->Tinv.as<double>();
      if (k1 > 0)
        g2.one(Zp + P->Doff[e], m[i], k1, m[k], k1, Ti + P->offTinv[2 * i], k1, false,
               Zt + P->Doff[e], m[i], false);
      if (k2 > 0)
        g2.one(Zp + P->Doff[e] + k1, m[i], k2, m[k], k2, Ti + P->offTinv[2 * i + 1], k2, false,
               Zt + P->Doff[e] + k1, m[i], false);
    }
  }
  g.run(st, "fill_z");
  g2.run(st, "fill_z");
  if (fill32) {
    // FP32 copy of Z' for the fill-in products (entries of sketched boxes are
    // converted too but never read)
    std::vector<Prob*> done;
    for (const Box& b : boxes)
      if (std::find(done.begin(), done.end(), b.P) == done.end()) {
        done.push_back(b.P);
        b.P->Z32 = to_f32(b.P->Z.as<double>(), b.P->Doff[b.P->nnear()], s);
      }
  }
  st.sync();
}

// ---- (c) preparation of the basis step: fill targets, far-field columns,
// features, and (with a rank model) the predicted ranks and sketch sizes
void Driver::basis_prepare(Stage& st, const std::vector<Prob*>& G) {
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const int nb = P->nb;
    const std::vector<int>& m = lf.m;
    const Lists& ls = P->F->lists;
    P->targets.assign(nb, {});
    P->farcols.assign(nb, {});
    P->ncols.assign(nb, 0);
    lf.k.assign(nb, 0);
    lf.feat.assign((size_t)nb * MLP_NF, 0.0f);
    lf.khat.assign(nb, -1);
    lf.ell.assign(nb, 0);
    lf.sk_state.assign(nb, 0);
    P->Eptr.assign(nb, nullptr);
    P->ldE.assign(nb, 1);
    P->offSq.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i) P->offSq[i + 1] = P->offSq[i] + (int64_t)m[i] * m[i];
    const bool upper = P->lev < P->L();
    const double th = now_s();
    parallel_for(nb, 8, [&](int64_t i) {
      // the ablation without fill-ins in the basis has no fill targets
      if (p.fill_in) P->targets[i] = fill_targets(ls, P->lev, (int)i);
      // own-level far boxes are sampled at their candidates of the other side
      // (the columns of the far blocks for the row basis, the rows for the column
      // basis); shared bases have one candidate set
      const auto& fc = P->partner ? P->partner->lf().cand : lf.cand;
      P->farcols[i] = far_columns(P->F->tree, ls, P->lev, (int)i, fc, p.far_sample);
      int64_t nc = (int64_t)P->farcols[i].size();
      for (int j : P->targets[i]) nc += m[j];
      P->ncols[i] = nc;
      double ratio = 1.0;
      if (upper) {
        const LevelFactor& ch = P->F->levels[P->lev + 1];
        const int den = ch.m[2 * i] + ch.m[2 * i + 1];
        ratio = den > 0 ? (double)(ch.k[2 * i] + ch.k[2 * i + 1]) / den : 0.0;
      }
      box_features(*P->F, P->lev, (int)i, m[i], (int)P->targets[i].size(), nc, ratio,
                   lf.feat.data() + (size_t)i * MLP_NF);
    });
    // far-field columns of every box as indices into the shared point buffer,
    // one device array for the level (staged through pinned memory that lives
    // until the stage synchronises)
    P->far_off.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i)
      P->far_off[i + 1] = P->far_off[i] + (int64_t)P->farcols[i].size();
    const int64_t nfar = P->far_off[nb];
    P->dfar.alloc(std::max<int64_t>(nfar, 1) * sizeof(int64_t));
    if (nfar > 0) {
      size_t got = 0;
      char* hb = pinned_get(nfar * sizeof(int64_t), &got);
      st.host.push_back(std::shared_ptr<void>(hb, [got](void* q) { pinned_put((char*)q, got); }));
      int64_t* hf = reinterpret_cast<int64_t*>(hb);
      const int64_t poff = P->poff;
      parallel_for(nb, 8, [&](int64_t i) {
        int64_t* o = hf + P->far_off[i];
        for (int64_t c : P->farcols[i]) *o++ = c + poff;
      });
      H2ULV_HIP(hipMemcpyAsync(P->dfar.p, hb, nfar * sizeof(int64_t), hipMemcpyHostToDevice, s));
    }
    htime("h_prepare", th);
    // mixed precision: the rotations, low-rank couplings and Schur updates run on
    // FP32 matrix cores with FP32 accumulation.  The fill-in products feed the
    // rank-revealing QR, whose decisions at tol ~1e-6 sit at FP32 rounding level:
    // without a rank cap FP32 fill-ins inflate the upper-level ranks several
    // times, so they are FP32 only when a cap bounds the ranks; inverses, QR/ID,
    // solve and residual are FP64
    if (mixed) P->D32 = to_f32(P->D.as<double>(), P->Doff[P->nnear()], s);
    // per-box pivoted-QR matrices (m x m) kept until W' is built
    P->PQ.alloc(std::max<int64_t>(P->offSq[nb], 1) * sizeof(double));
    P->pivd.alloc(std::max<int64_t>(P->cand_off[nb], 1) * sizeof(int32_t));
    P->kd.alloc(std::max(nb, 1) * sizeof(int32_t));
    H2ULV_HIP(hipMemsetAsync(P->PQ.p, 0, P->PQ.bytes, s));
  }
  if (!p.rank_model) return;
  // predicted ranks: one forward pass over the features of every box
  std::vector<float> feats;
  for (Prob* P : G) {
    const std::vector<float>& f = P->lf().feat;
    feats.insert(feats.end(), f.begin(), f.end());
  }
  const int64_t nf = (int64_t)feats.size() / MLP_NF;
  if (nf == 0) return;
  const float* dfeat = st.up(std::move(feats));
  float* dy = st.scratch<float>(nf);
  launch_mlp_forward(p.rank_model->theta.as<float>(), dfeat, nf, dy, s);
  H2ULV_HIP(hipGetLastError());
  std::vector<float> hy(nf);
  H2ULV_HIP(hipMemcpyAsync(hy.data(), dy, nf * sizeof(float), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  int64_t q = 0;
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    for (int i = 0; i < P->nb; ++i, ++q) {
      double kh = std::floor(std::pow(2.0, (double)hy[q]) - 1.0 + 0.5);
      if (!(kh < 1e8)) kh = 1e8;  // also catches a non-finite output
      lf.khat[i] = std::max(0, (int)kh);
      const int mi = lf.m[i];
      // at most m - probes columns: a box whose predicted rank leaves no room
      // (k-hat >= m - probes included) is still sketched at full width, which
      // the probe check accepts whenever its true rank is below that width; with
      // a rank cap the sketch is sized for min(k-hat, cap).  Levels above
      // sketch_min_level keep the full pivoted QR.
      const int64_t ks = p.rank_cap > 0 ? std::min(lf.khat[i], p.rank_cap) : lf.khat[i];
      const int64_t ell = std::min<int64_t>((5 * ks + 3) / 4 + p.oversample, mi - SKETCH_PROBES);
      if (ell > 0 && ell < P->ncols[i] && P->lev >= p.sketch_min_level) {
        lf.ell[i] = (int)ell;
        lf.sk_state[i] = 1;
      }
    }
  }
}

// ---- (c) sketch of M' without forming it.  Omega's rows are keyed by point:
// far-field column p takes row p of the far stream, the fill-in columns of
// target j take the rows G_j of j's candidates in the fill stream.  Since
// T-hat^-1 F_ij = T-hat^-1 sum_k D_ik D_kk^-1 D_kj over the k next to both i and j,
//   (M' Omega)^T = Omega_far^T K(P_i, far)^T + (sum_{k in Near(i), k != i} Q'_k^T D_ik^T) T-hat^-T,
//   Q'_k = D_kk^-1 Q_k,  Q_k = sum_{j in Near(k), j != k} D_kj G_j,
// and every Q'_k is shared by all boxes next to k (no Z'_ik is formed).  Q is
// as wide as the widest sketch of the pass in its problem; box i takes its
// first l_i + q columns.
void Driver::build_sketch(Stage& st, const std::vector<Box>& boxes, bool rebuild) {
  struct PS {
    Prob* P;
    std::vector<int> bx;
    int C = 0;
    std::vector<int64_t> goff, qoff;  // -1: block not needed
  };
  std::vector<PS> ps;
  auto find_ps = [&](const Prob* P) -> PS* {
    for (PS& x : ps)
      if (x.P == P) return &x;
    return nullptr;
  };
  for (const Box& b : boxes) {
    if (!find_ps(b.P)) ps.push_back(PS{b.P, {}, 0, {}, {}});
    find_ps(b.P)->bx.push_back(b.i);
  }
  int64_t gwords = 0, qwords = 0;
  for (PS& x : ps) {
    Prob* P = x.P;
    const std::vector<int>& m = P->lf().m;
    const auto& np = P->np();
    const auto& ni = P->ni();
    std::vector<char> needK(P->nb, 0), needJ(P->nb, 0);
    for (int i : x.bx) {
      x.C = std::max(x.C, P->lf().ell[i] + SKETCH_PROBES);
      for (int64_t e = np[i]; e < np[i + 1]; ++e)
        if (ni[e] != i && m[ni[e]] > 0) needK[ni[e]] = 1;
    }
    for (int k = 0; k < P->nb; ++k)
      if (needK[k])
        for (int64_t e = np[k]; e < np[k + 1]; ++e)
          if (ni[e] != k && m[ni[e]] > 0) needJ[ni[e]] = 1;
    x.goff.assign(P->nb, -1);
    x.qoff.assign(P->nb, -1);
    for (int j = 0; j < P->nb; ++j) {
      if (needJ[j]) {
        x.goff[j] = gwords;
        gwords += (int64_t)m[j] * x.C;
      }
      if (needK[j]) {
        x.qoff[j] = qwords;
        qwords += (int64_t)m[j] * x.C;
      }
    }
  }
  DBuf Qb(std::max<int64_t>(qwords, 1) * sizeof(double));
  double* Qp = Qb.as<double>();
  {
    DBuf Gb(std::max<int64_t>(gwords, 1) * sizeof(double));
    DBuf Qtb(std::max<int64_t>(qwords, 1) * sizeof(double));
    double* Gp = Gb.as<double>();
    double* Qt = Qtb.as<double>();
    std::vector<GaussItem> gi;
    std::vector<int64_t> tp(1, 0);
    GemmBatch<double> gq;
    for (PS& x : ps) {
      Prob* P = x.P;
      const std::vector<int>& m = P->lf().m;
      const auto& np = P->np();
      const auto& ni = P->ni();
      const uint64_t key = sketch_key(p.sketch_seed, P->lev, STREAM_BASE + STREAM_FILL);
      for (int j = 0; j < P->nb; ++j) {
        if (x.goff[j] < 0) continue;
        gi.push_back(GaussItem{Gp + x.goff[j], m[j], P->candp(j), P->poff, P->F->n, key, m[j],
                               x.C});
        tp.push_back(tp.back() + tiles64(m[j], x.C));
      }
      for (int k = 0; k < P->nb; ++k) {
        if (x.qoff[k] < 0) continue;
        gq.item(Qt + x.qoff[k], m[k], m[k], x.C);
        for (int64_t e = np[k]; e < np[k + 1]; ++e) {
          const int j = ni[e];
          if (j == k || m[j] == 0) continue;
          gq.term(P->D.as<double>() + P->Doff[e], m[k], false, Gp + x.goff[j], m[j], false, m[j]);
          P->fl_fill += 2.0 * m[k] * (double)m[j] * x.C;
        }
      }
    }
    if (!gi.empty()) {
      const int ngi = (int)gi.size();
      const int64_t nt = tp.back();
      GaussItem* dgi = st.up(std::move(gi));
      int64_t* dtp = st.up(std::move(tp));
      ProfScope pg("gauss", 0, 0, s);
      launch_gauss(dgi, dtp, nt, ngi, s);
      H2ULV_HIP(hipGetLastError());
    }
    gq.run(st, "sketch_q");
    // Q'_k = D_kk^-1 Q_k
    GemmBatch<double> gi2;
    for (PS& x : ps) {
      Prob* P = x.P;
      const std::vector<int>& m = P->lf().m;
      for (int k = 0; k < P->nb; ++k) {
        if (x.qoff[k] < 0) continue;
        gi2.one(Qp + x.qoff[k], m[k], m[k], x.C, m[k], P->Dinv.as<double>() + P->offSq[k], m[k],
                false, Qt + x.qoff[k], m[k], false);
        P->fl_fill += 2.0 * m[k] * (double)m[k] * x.C;
      }
    }
    gi2.run(st, "sketch_q");
  }
  // per box: K(P_i, far)^T and Omega_far, then [Y^T; Z^T] (chunked by memory)
  std::vector<Box> order;
  for (PS& x : ps)
    for (int i : x.bx) order.push_back(Box{x.P, i});
  const int64_t budget =
      std::max<int64_t>((int64_t)(free_device_bytes() * 0.4) / (int64_t)sizeof(double), 1 << 20);
  auto box_words = [&](const Box& b) {
    const int64_t nf = (int64_t)b.P->farcols[b.i].size();
    const int64_t mi = b.P->lf().m[b.i], ci = b.P->lf().ell[b.i] + SKETCH_PROBES;
    return nf * (mi + ci) + ci * mi + 4096;
  };
  size_t b0 = 0;
  while (b0 < order.size()) {
    size_t b1 = b0;
    int64_t acc = 0;
    while (b1 < order.size() && (b1 == b0 || acc + box_words(order[b1]) <= budget)) {
      acc += box_words(order[b1]);
      ++b1;
    }
    const size_t nc = b1 - b0;
    const double th = now_s();
    std::vector<int64_t> koff(nc + 1, 0), ooff(nc + 1, 0), roff(nc + 1, 0);
    for (size_t q = 0; q < nc; ++q) {
      const Box& b = order[b0 + q];
      const int64_t nf = (int64_t)b.P->farcols[b.i].size();
      const int64_t ci = b.P->lf().ell[b.i] + SKETCH_PROBES;
      koff[q + 1] = koff[q] + nf * b.P->lf().m[b.i];
      ooff[q + 1] = ooff[q] + nf * ci;
      roff[q + 1] = roff[q] + (b.P->lev < b.P->L() ? ci * b.P->lf().m[b.i] : 0);
    }
    DBuf Kb(std::max<int64_t>(koff.back(), 1) * sizeof(double));
    DBuf Ob(std::max<int64_t>(ooff.back(), 1) * sizeof(double));
    DBuf Rb(std::max<int64_t>(roff.back(), 1) * sizeof(double));
    KgenBatch kb;
    GemmBatch<double> gr, gs;
    std::vector<GaussItem> gi;
    std::vector<int64_t> tp(1, 0);
    for (size_t q = 0; q < nc; ++q) {
      const Box& b = order[b0 + q];
      Prob* P = b.P;
      const PS* x = find_ps(b.P);
      const int i = b.i;
      const std::vector<int>& m = P->lf().m;
      const int mi = m[i];
      const int ci = P->lf().ell[i] + SKETCH_PROBES;
      const int64_t nf = (int64_t)P->farcols[i].size();
      double* Kf = Kb.as<double>() + koff[q];
      double* Of = Ob.as<double>() + ooff[q];
      double* PQi = P->PQ.as<double>() + P->offSq[i];
      const bool upper = P->lev < P->L();
      if (nf > 0) {
        kb.add(P->farp(i), (int)nf, P->candp(i), mi, Kf, nf);
        if (!rebuild) P->kevals += (double)mi * nf;
        gi.push_back(GaussItem{Of, nf, P->farp(i), P->poff, P->F->n,
                               sketch_key(p.sketch_seed, P->lev, STREAM_BASE + STREAM_FAR),
                               (int32_t)nf, ci});
        tp.push_back(tp.back() + tiles64(nf, ci));
        P->fl_basis += 2.0 * (double)nf * mi * ci;
      }
      // fill part sum_k Q'_k^T D_ik^T: straight into the sketch at the leaves,
      // into R_i above them (then times T-hat^-T)
      double* Ri = upper ? Rb.as<double>() + roff[q] : PQi;
      const auto& np = P->np();
      const auto& ni = P->ni();
      if (upper) gr.item(Ri, ci, ci, mi);
      else gs.item(PQi, ci, ci, mi);
      GemmBatch<double>& gf = upper ? gr : gs;
      if (!upper && nf > 0) gs.term(Of, nf, true, Kf, nf, false, (int)nf);
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        const int k = ni[e];
        if (k == i || m[k] == 0) continue;
        gf.term(Qp + x->qoff[k], m[k], true, P->D.as<double>() + P->Doff[e], mi, true, m[k]);
        P->fl_fill += 2.0 * ci * (double)m[k] * mi;
      }
      if (upper) {
        // [Y^T; Z^T](:, child c) = Omega_far^T K_far^T(:, c) + R_i(:, c) T_c^-T
        const LevelFactor& ch = P->F->levels[P->lev + 1];
        const int kc[2] = {ch.k[2 * i], ch.k[2 * i + 1]};
        int c0 = 0;
        for (int h = 0; h < 2; ++h) {
          if (kc[h] == 0) continue;
          gs.item(PQi + (int64_t)c0 * ci, ci, ci, kc[h]);
          if (nf > 0) gs.term(Of, nf, true, Kf + (int64_t)c0 * nf, nf, false, (int)nf);
          gs.term(Ri + (int64_t)c0 * ci, ci, false, P->Tinv.as<double>() + P->offTinv[2 * i + h],
                  kc[h], true, kc[h]);
          c0 += kc[h];
        }
      }
    }
    htime("h_sketch", th);
    kb.run(st, pts, kf, dup);
    if (!gi.empty()) {
      const int ngi = (int)gi.size();
      const int64_t nt = tp.back();
      GaussItem* dgi = st.up(std::move(gi));
      int64_t* dtp = st.up(std::move(tp));
      ProfScope pg("gauss", 0, 0, s);
      launch_gauss(dgi, dtp, nt, ngi, s);
      H2ULV_HIP(hipGetLastError());
    }
    gr.run(st, "sketch");
    gs.run(st, "sketch");
    tick("c_sketch");
    st.sync();
    b0 = b1;
  }
}

// ---- (c) M'^T of each remaining box (chunked over boxes by memory) and its
// tall QR -> m x m triangle
void Driver::build_triangles(Stage& st, const std::vector<Box>& boxes, bool rebuild) {
  // sketched boxes never form M'; the rest get the triangle of their M'^T
  std::vector<Box> sk, full;
  for (const Box& b : boxes) (b.P->lf().sk_state[b.i] == 1 ? sk : full).push_back(b);
  if (!sk.empty()) build_sketch(st, sk, rebuild);
  if (full.empty()) return;
  const size_t freeb = free_device_bytes();
  int64_t budget = (int64_t)(freeb * 0.4) / (int64_t)sizeof(double);
  budget = std::max<int64_t>(budget, 1 << 20);
  auto box_words = [&](const Box& b) {
    const int64_t mi = b.P->lf().m[b.i], nc = b.P->ncols[b.i];
    // M'^T plus the QR workspaces of its chunks (reflector panels, T, GEMM scratch)
    return mi * nc * 3 / 2 + 8 * mi * mi + 4096;
  };
  const size_t nbox = full.size();
  size_t b0 = 0;
  while (b0 < nbox) {
    size_t b1 = b0;
    int64_t acc = 0;
    while (b1 < nbox && (b1 == b0 || acc + box_words(full[b1]) <= budget)) {
      acc += box_words(full[b1]);
      ++b1;
    }
    const size_t nc = b1 - b0;
    // M'^T (ncols x m, column-major): far-field rows then fill-in rows
    std::vector<int64_t> moff(nc + 1, 0);
    for (size_t q = 0; q < nc; ++q) {
      const Box& b = full[b0 + q];
      moff[q + 1] = moff[q] + (int64_t)b.P->lf().m[b.i] * b.P->ncols[b.i];
    }
    DBuf Mb(std::max<int64_t>(moff.back(), 1) * sizeof(double));
    double* Mp = Mb.as<double>();
    KgenBatch kb;
    GemmBatch<double> g;
    GemmBatch<float, double> g32;
    for (size_t q = 0; q < nc; ++q) {
      Prob* P = full[b0 + q].P;
      const int i = full[b0 + q].i;
      const std::vector<int>& m = P->lf().m;
      if (m[i] == 0) continue;
      const auto& np = P->np();
      const auto& ni = P->ni();
      double* Mi = Mp + moff[q];
      const int64_t ld = P->ncols[i];
      const int64_t nf = (int64_t)P->farcols[i].size();
      // M'^T(a, b) = K(cand_b, far_a) (row side; the column side of a
      // nonsymmetric matrix has M'^T(a, b) = K(far_a, cand_b))
      kb.add(P->farp(i), (int)nf, P->candp(i), m[i], Mi, ld, !P->colside);
      // a rebuilt box (a rejected sketch) has had its kernel entries counted
      if (!rebuild) P->kevals += (double)m[i] * nf;
      int64_t row = nf;
      for (int j : P->targets[i]) {
        if (m[j] > 0) {
          // (T^-1 F_ij)^T = sum_k D_kj^T Z'_ik^T
          if (fill32)
            g32.item(Mi + row, ld, m[j], m[i]);
          else
            g.item(Mi + row, ld, m[j], m[i]);
          for (int64_t e = np[i]; e < np[i + 1]; ++e) {
            int k = ni[e];
            if (k == i || k == j || m[k] == 0) continue;
            int64_t ekj = csr_find(np, ni, k, j);
            if (ekj < 0) continue;
            if (fill32)
              g32.term(P->D32.as<float>() + P->Doff[ekj], m[k], true,
                       P->Z32.as<float>() + P->Doff[e], m[i], true, m[k]);
            else
              g.term(P->D.as<double>() + P->Doff[ekj], m[k], true,
                     P->Z.as<double>() + P->Doff[e], m[i], true, m[k]);
            P->fl_fill += 2.0 * m[i] * (double)m[k] * m[j];
          }
        }
        row += m[j];
      }
    }
    kb.run(st, pts, kf, dup);
    g.run(st, "fill_m");
    g32.run(st, "fill_m");
    tick("c_fill_gemm");
    // tall QR of every other M'^T: a tree of blocked Householder QRs (leaf
    // chunks factored in place, then stacked triangles merged in groups)
    struct Rref {
      double* p;
      int64_t ld;
      int r;
    };
    std::vector<std::vector<Rref>> cur(nc);
    std::vector<int> mq(nc);
    std::vector<TallQr> leaf;
    for (size_t q = 0; q < nc; ++q) {
      Prob* P = full[b0 + q].P;
      const int i = full[b0 + q].i;
      const int mi = P->lf().m[i];
      const int64_t nci = P->ncols[i];
      mq[q] = mi;
      if (mi == 0 || nci == 0) continue;
      double* Mi = Mp + moff[q];
      // leaf chunks as tall as the LDS panel kernel takes (4096 rows), at least
      // 4m: the panel's cost per column hardly grows with its height, and fewer
      // chunks mean fewer panels and merge rounds
      const int64_t h = std::max<int64_t>(4 * (int64_t)mi, std::min<int64_t>(16 * (int64_t)mi, 4096));
      for (int64_t r0 = 0; r0 < nci; r0 += h) {
        int hc = (int)std::min<int64_t>(h, nci - r0);
        leaf.push_back(TallQr{Mi + r0, nci, hc, mi});
        cur[q].push_back(Rref{Mi + r0, nci, std::min(hc, mi)});
      }
      double ncd = (double)nci, mm = (double)mi;
      P->fl_basis += (ncd >= mm) ? 2.0 * ncd * mm * mm - 2.0 / 3.0 * mm * mm * mm
                                 : 2.0 * mm * ncd * ncd - 2.0 / 3.0 * ncd * ncd * ncd;
    }
    batched_qr_R(st, leaf);
    std::vector<DBuf> rounds;
    // merge rounds: each stacks as many consecutive triangles as fit in the LDS
    // panel kernel's 4096 rows (at least two) and factors the stack
    auto group_of = [](int mi) { return std::max(2, 4096 / std::max(mi, 1)); };
    for (;;) {
      int64_t words = 0;
      bool more = false;
      for (size_t q = 0; q < nc; ++q) {
        const size_t G = (size_t)group_of(mq[q]);
        for (size_t u = 0; u < cur[q].size(); u += G) {
          const size_t e = std::min(cur[q].size(), u + G);
          if (e - u < 2) continue;
          for (size_t v = u; v < e; ++v) words += (int64_t)cur[q][v].r * mq[q];
          more = true;
        }
      }
      if (!more) break;
      DBuf buf(std::max<int64_t>(words, 1) * sizeof(double));
      double* bp = buf.as<double>();
      int64_t off = 0;
      CopyBatch cb;
      std::vector<CopyItem> zl;
      std::vector<TallQr> qs;
      for (size_t q = 0; q < nc; ++q) {
        auto& v = cur[q];
        const int mi = mq[q];
        const size_t G = (size_t)group_of(mi);
        std::vector<Rref> nxt;
        for (size_t u = 0; u < v.size(); u += G) {
          const size_t e = std::min(v.size(), u + G);
          if (e - u == 1) {
            nxt.push_back(v[u]);
            continue;
          }
          int hs = 0;
          for (size_t t = u; t < e; ++t) hs += v[t].r;
          double* Sb = bp + off;
          off += (int64_t)hs * mi;
          int ro = 0;
          for (size_t t = u; t < e; ++t) {
            cb.add(v[t].p, v[t].ld, Sb + ro, hs, v[t].r, mi);
            zl.push_back(CopyItem{nullptr, Sb + ro, 0, hs, v[t].r, mi, 0, 0});
            ro += v[t].r;
          }
          qs.push_back(TallQr{Sb, hs, hs, mi});
          nxt.push_back(Rref{Sb, hs, std::min(hs, mi)});
        }
        v.swap(nxt);
      }
      cb.run(st);
      int nz = (int)zl.size();
      CopyItem* dz = st.up(std::move(zl));
      launch_zero_lower(dz, nz, s);
      H2ULV_HIP(hipGetLastError());
      batched_qr_R(st, qs);
      rounds.push_back(std::move(buf));
    }
    // final triangles into the m x m pivoted-QR matrices (zero below)
    {
      CopyBatch cb;
      std::vector<CopyItem> zl;
      for (size_t q = 0; q < nc; ++q) {
        if (cur[q].empty()) continue;
        Prob* P = full[b0 + q].P;
        const int i = full[b0 + q].i;
        const int mi = mq[q];
        const Rref& r = cur[q][0];
        double* PQi = P->PQ.as<double>() + P->offSq[i];
        cb.add(r.p, r.ld, PQi, mi, r.r, mi);
        zl.push_back(CopyItem{nullptr, PQi, 0, mi, r.r, mi, 0, 0});
      }
      cb.run(st);
      int nz = (int)zl.size();
      CopyItem* dz = st.up(std::move(zl));
      launch_zero_lower(dz, nz, s);
      H2ULV_HIP(hipGetLastError());
    }
    tick("c_tsqr");
    st.sync();
    b0 = b1;
  }
}

// ---- (c) column-pivoted QR of each box's matrix (the m x m triangle, or the
// l x m sketch of a sketched box): small boxes one workgroup each, large boxes
// over many workgroups, one pivot step per pair of launches.  Ranks come back
// to the host; E = R11^-1 R12 is left in place (small) or solved into a
// buffer (large).
void Driver::pivot_boxes(Stage& st, const std::vector<Box>& boxes, const std::vector<int>* force) {
  const int BIG = 512;
  struct Job {
    Prob* P;
    int i;
    int rows;
    int64_t lda;
    int big;  // index into the large-box states, or -1
  };
  std::vector<Job> jobs;
  int64_t tot_cand = 0;
  for (const Box& b : boxes) tot_cand += b.P->lf().m[b.i];
  const size_t nbox = boxes.size();
  std::vector<PivQrItem> pq;
  std::vector<PivQrState> big;
  double* nrm = st.scratch<double>(std::max<int64_t>(tot_cand, 1));
  double* dg = st.scratch<double>(std::max<int64_t>(tot_cand, 1));
  double* scal = st.scratch<double>(2 * nbox + 2);
  int32_t* flg = st.scratch<int32_t>(2 * nbox + 2);
  int64_t co = 0;
  for (size_t q = 0; q < nbox; ++q) {
    Prob* P = boxes[q].P;
    const int i = boxes[q].i;
    const LevelFactor& lf = P->lf();
    const int mi = lf.m[i];
    if (mi == 0) continue;
    int cap = (int)std::min<int64_t>(mi, P->ncols[i]);
    if (p.rank_cap > 0) cap = std::min(cap, p.rank_cap);
    double tol = p.tol;
    if (force) {
      cap = std::min(cap, (*force)[q]);
      tol = 0.0;
    }
    int rows = mi;
    int64_t lda = mi;
    if (lf.sk_state[i] == 1) {
      rows = lf.ell[i];
      lda = lf.ell[i] + SKETCH_PROBES;
      cap = std::min(cap, rows);
    }
    double* A = P->PQ.as<double>() + P->offSq[i];
    Job jb{P, i, rows, lda, -1};
    if (mi <= BIG) {
      // the one-workgroup kernel holds at most 512 rows and columns
      if (rows > BIG) fail(H2ULV_ERR_HIP, "internal: pivoted-QR matrix exceeds 512 rows");
      PivQrItem it{};
      it.A = A;
      it.lda = lda;
      it.m = rows;
      it.n = mi;
      it.piv = P->pivd.as<int32_t>() + P->cand_off[i];
      it.kout = P->kd.as<int32_t>() + i;
      it.diag = dg + co;
      it.work = nrm + co;
      it.tol = tol;
      it.cap = std::max(cap, 0);
      pq.push_back(it);
    } else {
      PivQrState ps{};
      ps.A = A;
      ps.lda = lda;
      ps.m = rows;
      ps.n = mi;
      ps.cap = cap;
      ps.nrm = nrm + co;
      ps.piv = P->pivd.as<int32_t>() + P->cand_off[i];
      ps.scal = scal + 2 * q;
      ps.flags = flg + 2 * q;
      ps.tol = tol;
      jb.big = (int)big.size();
      big.push_back(ps);
    }
    jobs.push_back(jb);
    co += mi;
  }
  const int npq = (int)pq.size();
  PivQrItem* dpq = st.up(std::move(pq));
  {
    ProfScope ps("pivqr_small", 0, 0, s);
    launch_pivqr(dpq, npq, s);
  }
  H2ULV_HIP(hipGetLastError());
  const int nbig = (int)big.size();
  if (nbig > 0) {
    int maxcap = 0, maxcols = 0;
    std::vector<int64_t> sp(1, 0);
    for (auto& b : big) {
      sp.push_back(sp.back() + (b.n + 3) / 4);
      maxcap = std::max(maxcap, b.cap);
      maxcols = std::max(maxcols, b.n);
    }
    const int64_t ns = sp.back();
    PivQrState* dst_ = st.up(std::move(big));
    int64_t* dsp = st.up(std::move(sp));
    ProfScope ps("pivqr_large", 0, 0, s);
    launch_pivqr_init(dst_, dsp, ns, nbig, s);
    // every 64 steps the stop flags come back to the host, and the loop ends
    // once every box has stopped (ranks are usually well below the step cap)
    std::vector<int32_t> fl(2 * nbox + 2);
    for (int t = 0; t < maxcap; ++t) {
      launch_pivqr_pick(dst_, nbig, t, s);
      launch_pivqr_apply(dst_, nbig, maxcols, t, s);
      if ((t + 1) % 64 == 0 && t + 1 < maxcap) {
        H2ULV_HIP(hipGetLastError());
        H2ULV_HIP(hipMemcpyAsync(fl.data(), flg, fl.size() * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, s));
        H2ULV_HIP(hipStreamSynchronize(s));
        bool any = false;  // a large box (flags at 2 q) still running
        for (size_t q = 0; q < nbox; ++q)
          if (boxes[q].P->lf().m[boxes[q].i] > BIG && fl[2 * q] == 0) any = true;
        if (!any) break;
      }
    }
    H2ULV_HIP(hipGetLastError());
  }
  // ranks to the host: small boxes from their rank slot, large from their flags
  std::vector<int32_t> hf(2 * nbox + 2);
  std::vector<std::vector<int32_t>> hk;
  std::vector<Prob*> probs;
  for (const Job& jb : jobs)
    if (std::find(probs.begin(), probs.end(), jb.P) == probs.end()) probs.push_back(jb.P);
  hk.resize(probs.size());
  for (size_t g = 0; g < probs.size(); ++g) {
    hk[g].resize(probs[g]->nb);
    H2ULV_HIP(hipMemcpyAsync(hk[g].data(), probs[g]->kd.p, probs[g]->nb * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
  }
  if (nbig > 0)
    H2ULV_HIP(hipMemcpyAsync(hf.data(), flg, hf.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  // algorithmic work of the pivoted QRs from the ranks reached: k Householder
  // steps on a rows x m matrix, 4 sum_t (rows - t)(m - t) flops, then
  // E = R11^-1 R12 (k^2 (m - k)); bytes: the matrix read and written once
  double fl_small = 0, by_small = 0, fl_large = 0, by_large = 0;
  std::map<Prob*, int64_t> ewords;
  for (size_t q = 0, j = 0; q < nbox && j < jobs.size(); ++q) {
    if (boxes[q].P != jobs[j].P || boxes[q].i != jobs[j].i) continue;
    Job& jb = jobs[j++];
    LevelFactor& lf = jb.P->lf();
    const size_t g = std::find(probs.begin(), probs.end(), jb.P) - probs.begin();
    const int k = jb.big >= 0 ? hf[2 * q + 1] : hk[g][jb.i];
    lf.k[jb.i] = k;
    {
      const double rw = jb.rows, mm = lf.m[jb.i];
      double fl = (double)k * k * (mm - k);
      for (int t = 0; t < k; ++t) fl += 4.0 * (rw - t) * (mm - t);
      (jb.big >= 0 ? fl_large : fl_small) += fl;
      (jb.big >= 0 ? by_large : by_small) += 16.0 * rw * mm;
    }
    if (jb.big >= 0) {
      ewords[jb.P] += (int64_t)k * (lf.m[jb.i] - k);
    } else {
      jb.P->Eptr[jb.i] = jb.P->PQ.as<double>() + jb.P->offSq[jb.i] + (int64_t)k * jb.lda;
      jb.P->ldE[jb.i] = jb.lda;
    }
  }
  profiler().amend_last("pivqr_small", fl_small, by_small);
  if (nbig > 0) profiler().amend_last("pivqr_large", fl_large, by_large);
  // E = R11^-1 R12 of the large boxes by triangular blocks
  std::map<Prob*, double*> ebase;
  for (auto& kv : ewords) {
    kv.first->Ebufs.emplace_back(std::max<int64_t>(kv.second, 1) * sizeof(double));
    ebase[kv.first] = kv.first->Ebufs.back().as<double>();
  }
  std::vector<TriRhs> sys;
  for (const Job& jb : jobs) {
    if (jb.big < 0) continue;
    LevelFactor& lf = jb.P->lf();
    const int k = lf.k[jb.i], mi = lf.m[jb.i];
    double*& eb = ebase[jb.P];
    jb.P->Eptr[jb.i] = eb;
    jb.P->ldE[jb.i] = std::max(k, 1);
    if (k > 0 && k < mi) {
      double* A = jb.P->PQ.as<double>() + jb.P->offSq[jb.i];
      sys.push_back(TriRhs{A, jb.lda, k, A + (int64_t)k * jb.lda, jb.lda, eb, k, mi - k});
    }
    eb += (int64_t)k * (mi - k);
  }
  trsm_upper(st, sys);
  tick("c_pivqr");
  st.sync();
}

// ---- (c) randomized check of the sketched row IDs: with Z^T the probe rows
// below the sketch, res = Z^T[:, piv[k:]] - Z^T[:, piv[:k]] E; accepted iff the
// sketch was not exhausted and |res|_F <= slack sqrt(m - k) tol max_j |Z^T[:, j]|,
// or the rank cap ended the pivot loop with q columns of oversampling left.
// Returns the rejected boxes.
std::vector<Box> Driver::check_sketches(Stage& st, const std::vector<Box>& boxes) {
  const int q = SKETCH_PROBES;
  std::vector<Box> fails, probed;
  std::vector<GatherItem> gi;
  std::vector<int64_t> tp(1, 0);
  std::vector<NormItem> ni;
  GemmBatch<double> g;
  int64_t zw = 0;
  for (const Box& b : boxes) {
    const LevelFactor& lf = b.P->lf();
    if (lf.k[b.i] >= lf.ell[b.i]) {
      fails.push_back(b);  // exhausted: the rank may exceed the sketch
      continue;
    }
    probed.push_back(b);
    zw += (int64_t)q * lf.m[b.i];
  }
  if (!probed.empty()) {
    double* Zp = st.scratch<double>(std::max<int64_t>(zw, 1));
    double* out = st.scratch<double>(4 * probed.size());
    int64_t off = 0;
    for (size_t u = 0; u < probed.size(); ++u) {
      Prob* P = probed[u].P;
      const int i = probed[u].i;
      const LevelFactor& lf = P->lf();
      const int mi = lf.m[i], k = lf.k[i], ell = lf.ell[i];
      const int64_t ldy = ell + q;
      const double* Zt = P->PQ.as<double>() + P->offSq[i] + ell;
      double* Zi = Zp + off;
      off += (int64_t)q * mi;
      gi.push_back(GatherItem{Zt, ldy, Zi, q, P->pivd.as<int32_t>() + P->cand_off[i], q, mi});
      tp.push_back(tp.back() + tiles64(q, mi));
      if (k > 0)
        g.one(Zi + (int64_t)k * q, q, q, mi - k, k, Zi, q, false, P->Eptr[i], P->ldE[i], false,
              -1.0, 1.0);
      ni.push_back(NormItem{Zi + (int64_t)k * q, q, out + 4 * u, q, mi - k});
      ni.push_back(NormItem{Zt, ldy, out + 4 * u + 2, q, mi});
    }
    const int ngi = (int)gi.size();
    const int64_t nt = tp.back();
    GatherItem* dgi = st.up(std::move(gi));
    int64_t* dtp = st.up(std::move(tp));
    launch_gather_cols(dgi, dtp, nt, ngi, s);
    H2ULV_HIP(hipGetLastError());
    g.run(st, "probe");
    const int nni = (int)ni.size();
    NormItem* dni = st.up(std::move(ni));
    launch_norms(dni, nni, s);
    H2ULV_HIP(hipGetLastError());
    std::vector<double> h(4 * probed.size());
    H2ULV_HIP(hipMemcpyAsync(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    H2ULV_HIP(hipStreamSynchronize(s));
    for (size_t u = 0; u < probed.size(); ++u) {
      const LevelFactor& lf = probed[u].P->lf();
      const int mi = lf.m[probed[u].i], k = lf.k[probed[u].i];
      const double res = std::sqrt(h[4 * u]), zmax = std::sqrt(h[4 * u + 3]);
      // the cap ended the pivot loop: the full pivoted QR misses tol as well, so
      // the sketch stands if it keeps q columns of oversampling beyond k
      const bool capped =
          p.rank_cap > 0 && k == p.rank_cap && lf.ell[probed[u].i] - k >= SKETCH_PROBES;
      if (!capped && !(res <= SKETCH_SLACK * std::sqrt((double)(mi - k)) * p.tol * zmax))
        fails.push_back(probed[u]);
    }
  }
  st.sync();
  return fails;
}

// ---- (c) the basis step up to the pivots: sketches and triangles, pivoted QR,
// checks and fallback; then skeletons on the host
// Separate bases: the row and column IDs of a box keep the same number of
// pivots, k = min(max(k_row, k_col), steps_row, steps_col) with steps =
// min(m, columns of M'), so that S^RR stays square.  A side whose tolerance
// rank differs pivots again from its saved triangle, keeping exactly k.
void Driver::couple_ranks(Stage& st, const std::vector<Prob*>& G) {
  for (int round = 0; round < 2; ++round) {
    std::vector<Box> redo;
    std::vector<int> want;
    for (Prob* P : G) {
      if (P->colside) continue;
      Prob* C = P->partner;
      LevelFactor& a = P->lf();
      LevelFactor& b = C->lf();
      for (int i = 0; i < P->nb; ++i) {
        const int mi = a.m[i];
        if (mi == 0) continue;
        const int sa = (int)std::min<int64_t>(mi, P->ncols[i]);
        const int sb = (int)std::min<int64_t>(mi, C->ncols[i]);
        const int k = round == 0 ? std::min({std::max(a.k[i], b.k[i]), sa, sb})
                                 : std::min(a.k[i], b.k[i]);
        if (a.k[i] != k) {
          redo.push_back(Box{P, i});
          want.push_back(k);
        }
        if (b.k[i] != k) {
          redo.push_back(Box{C, i});
          want.push_back(k);
        }
      }
    }
    if (redo.empty()) return;
    for (const Box& bx : redo) {
      const int mi = bx.P->lf().m[bx.i];
      const int64_t o = bx.P->offSq[bx.i];
      H2ULV_HIP(hipMemcpyAsync(bx.P->PQ.as<double>() + o, bx.P->PQ0 + o,
                               (size_t)mi * mi * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    pivot_boxes(st, redo, &want);
  }
  for (Prob* P : G)
    if (!P->colside)
      for (int i = 0; i < P->nb; ++i)
        if (P->lf().k[i] != P->partner->lf().k[i])
          fail(H2ULV_ERR_HIP, "internal: row and column ranks of a box differ");
}

void Driver::row_ids(Stage& st, const std::vector<Prob*>& G) {
  std::vector<Box> all, sk;
  for (Prob* P : G)
    for (int i = 0; i < P->nb; ++i) {
      all.push_back(Box{P, i});
      if (P->lf().sk_state[i] == 1) sk.push_back(Box{P, i});
    }
  build_triangles(st, all);
  const bool two = G.size() > 0 && G[0]->partner != nullptr;
  std::vector<DBuf> keep;  // separate bases: the triangles before pivoting
  if (two)
    for (Prob* P : G) {
      keep.emplace_back(P->PQ.bytes);
      H2ULV_HIP(hipMemcpyAsync(keep.back().p, P->PQ.p, P->PQ.bytes, hipMemcpyDeviceToDevice, s));
      P->PQ0 = keep.back().as<double>();
    }
  pivot_boxes(st, all);
  if (two) couple_ranks(st, G);
  if (!sk.empty()) {
    auto clear = [&](const Box& b) {
      const int mi = b.P->lf().m[b.i];
      H2ULV_HIP(hipMemsetAsync(b.P->PQ.as<double>() + b.P->offSq[b.i], 0,
                               (size_t)mi * mi * sizeof(double), s));
    };
    std::vector<Box> fails = check_sketches(st, sk), retry, full;
    // a rejected sketch is retried once at full width (m - probes columns)
    for (const Box& b : fails) {
      LevelFactor& lf = b.P->lf();
      const int w = lf.m[b.i] - SKETCH_PROBES;
      if (lf.ell[b.i] < w && w < b.P->ncols[b.i]) {
        lf.ell[b.i] = w;
        retry.push_back(b);
      } else {
        full.push_back(b);
      }
    }
    if (!retry.empty()) {
      for (const Box& b : retry) clear(b);
      build_triangles(st, retry, true);
      pivot_boxes(st, retry);
      std::vector<Box> again = check_sketches(st, retry);
      for (const Box& b : retry) b.P->lf().sk_state[b.i] = 3;
      full.insert(full.end(), again.begin(), again.end());
    }
    if (!full.empty() && !p.sketch_fallback)
      fail(H2ULV_ERR_RANK_CHECK, "a sketched row ID failed its randomized check (no fallback)");
    if (!full.empty()) {
      // the full pivoted QR of their M' (rebuilt)
      for (const Box& b : full) {
        b.P->lf().sk_state[b.i] = 2;
        clear(b);
      }
      fill_z(st, full);
      build_triangles(st, full, true);
      pivot_boxes(st, full);
    }
  }
  for (Prob* P : G) {
    P->Z.reset();
    P->Dinv.reset();
    P->Tinv.reset();
  }
  check_dup();
  // pivots to the host: skeletons
  std::vector<std::vector<int32_t>> hp(G.size());
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    hp[g].resize(P->cand_off[P->nb]);
    if (!hp[g].empty())
      H2ULV_HIP(hipMemcpyAsync(hp[g].data(), P->pivd.p, hp[g].size() * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
  }
  H2ULV_HIP(hipStreamSynchronize(s));
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    LevelFactor& lf = P->lf();
    lf.sk.assign(P->nb, {});
    for (int i = 0; i < P->nb; ++i) {
      if (lf.m[i] == 0) lf.k[i] = 0;
      lf.sk[i].resize(lf.k[i]);
      const int32_t* piv = hp[g].data() + P->cand_off[i];
      for (int t = 0; t < lf.k[i]; ++t) lf.sk[i][t] = lf.cand[i][piv[t]];
    }
  }
}

// ---- (c) W', W = T-hat W', its QR -> U, T ------------------------------------
void Driver::bases(Stage& st, const std::vector<Prob*>& G) {
  std::vector<DBuf> Wps, Ws;
  std::vector<WpItem> wi;
  GemmBatch<double> g;
  std::vector<QrW> qs;
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const int nb = P->nb;
    const std::vector<int>& m = lf.m;
    const std::vector<int>& k = lf.k;
    const bool upper = P->lev < P->L();
    lf.offU.assign(nb + 1, 0);
    lf.offT.assign(nb + 1, 0);
    P->offW.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      lf.offU[i + 1] = lf.offU[i] + (int64_t)m[i] * m[i];
      lf.offT[i + 1] = lf.offT[i] + (int64_t)k[i] * k[i];
      P->offW[i + 1] = P->offW[i] + (int64_t)m[i] * k[i];
    }
    lf.U.alloc(std::max<int64_t>(lf.offU[nb], 1) * sizeof(double));
    lf.Tt.alloc(std::max<int64_t>(lf.offT[nb], 1) * sizeof(double));
    const int64_t ww = std::max<int64_t>(P->offW[nb], 1) * sizeof(double);
    Ws.emplace_back(ww);
    double* W = Ws.back().as<double>();
    double* Wp = W;
    if (upper) {
      Wps.emplace_back(ww);
      Wp = Wps.back().as<double>();
    }
    for (int i = 0; i < nb; ++i) {
      if (k[i] == 0) continue;
      wi.push_back(WpItem{P->pivd.as<int32_t>() + P->cand_off[i], P->Eptr[i], Wp + P->offW[i],
                          P->ldE[i], m[i], m[i], k[i]});
    }
    if (upper) {
      const LevelFactor& ch = P->F->levels[P->lev + 1];
      for (int i = 0; i < nb; ++i) {
        if (k[i] == 0) continue;
        int k1 = ch.k[2 * i], k2 = ch.k[2 * i + 1];
        double* Wi = W + P->offW[i];
        const double* Wpi = Wp + P->offW[i];
        if (k1 > 0)
          g.one(Wi, m[i], k1, k[i], k1, ch.Tt.as<double>() + ch.offT[2 * i], k1, false, Wpi, m[i],
                false);
        if (k2 > 0)
          g.one(Wi + k1, m[i], k2, k[i], k2, ch.Tt.as<double>() + ch.offT[2 * i + 1], k2, false,
                Wpi + k1, m[i], false);
      }
    }
    for (int i = 0; i < nb; ++i) {
      if (m[i] == 0) continue;
      qs.push_back(QrW{W + P->offW[i], m[i], k[i], lf.U.as<double>() + lf.offU[i],
                       lf.Tt.as<double>() + lf.offT[i]});
      P->fl_basis += 4.0 * m[i] * (double)k[i] * k[i] + 4.0 * (double)m[i] * m[i] * k[i];
    }
  }
  int nw = (int)wi.size();
  WpItem* dwi = st.up(std::move(wi));
  launch_wprime(dwi, nw, s);
  H2ULV_HIP(hipGetLastError());
  g.run(st, "basis");
  batched_qr_basis(st, qs);
  st.sync();
  for (Prob* P : G) {
    P->PQ.reset();
    P->pivd.reset();
    P->Ebufs.clear();
    P->kd.reset();
  }
}

// ---- (d) low-rank couplings -------------------------------------------------
void Driver::couplings(Stage& st, const std::vector<Prob*>& G) {
  // new skeleton blocks of this level: near pairs then far pairs
  for (Prob* P : G) {
    const int nb = P->nb;
    const std::vector<int>& k = P->lf().k;
    const auto& np = P->np();
    const auto& ni = P->ni();
    const auto& fp = P->fp();
    const auto& fi = P->fi();
    P->shat_near_off.assign(P->nnear() + 1, 0);
    P->shat_far_off.assign(P->nfar() + 1, 0);
    int64_t tot = 0;
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        P->shat_near_off[e] = tot;
        tot += (int64_t)k[i] * k[ni[e]];
      }
    for (int i = 0; i < nb; ++i)
      for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
        P->shat_far_off[e] = tot;
        tot += (int64_t)k[i] * k[fi[e]];
      }
    P->Shat.alloc(std::max<int64_t>(tot, 1) * sizeof(double));
  }
  // row skeletons of box i and column skeletons of box j (the same for shared
  // bases): S^SS_ij = T_i K(sk_i, sk'_j) T'_j^T
  std::vector<int64_t> skall;
  std::vector<std::vector<int64_t>> skoff(G.size()), skoffc(G.size()), kcoff(G.size());
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    const LevelFactor& lf = P->lf();
    skoff[g].assign(P->nb + 1, 0);
    for (int i = 0; i < P->nb; ++i) {
      skoff[g][i] = (int64_t)skall.size();
      for (int64_t a : lf.sk[i]) skall.push_back(a + P->poff);
    }
    skoffc[g] = skoff[g];
    if (P->partner) {
      const LevelFactor& rl = P->rlf();
      for (int i = 0; i < P->nb; ++i) {
        skoffc[g][i] = (int64_t)skall.size();
        for (int64_t a : rl.sk[i]) skall.push_back(a + P->poff);
      }
    }
    const auto& fp = P->fp();
    const auto& fi = P->fi();
    kcoff[g].assign(P->nfar() + 1, 0);
    for (int i = 0; i < P->nb; ++i)
      for (int64_t e = fp[i]; e < fp[i + 1]; ++e)
        kcoff[g][e + 1] = kcoff[g][e] + (int64_t)lf.k[i] * lf.k[fi[e]];
  }
  const int64_t* dsk = st.up(std::move(skall));
  std::vector<double*> Kc(G.size()), Tmp(G.size());
  KgenBatch kb;
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    const std::vector<int>& k = P->lf().k;
    const auto& fp = P->fp();
    const auto& fi = P->fi();
    const int64_t words = std::max<int64_t>(kcoff[g].back(), 1);
    Kc[g] = st.scratch<double>(words);
    Tmp[g] = st.scratch<double>(words);
    for (int i = 0; i < P->nb; ++i)
      for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
        int j = fi[e];
        if (k[i] == 0 || k[j] == 0) continue;
        kb.add(dsk + skoff[g][i], k[i], dsk + skoffc[g][j], k[j], Kc[g] + kcoff[g][e], k[i]);
        P->kevals += (double)k[i] * k[j];
        P->fl_couple += 2.0 * k[i] * (double)k[j] * k[j] + 2.0 * k[i] * (double)k[i] * k[j];
      }
  }
  kb.run(st, pts, kf, dup);
  // tmp = Kc T_j^T ; S = T_i tmp
  if (!mixed) {
    GemmBatch<double> g1, g2;
    for (size_t g = 0; g < G.size(); ++g) {
      Prob* P = G[g];
      const LevelFactor& lf = P->lf();
      const LevelFactor& rl = P->rlf();
      const std::vector<int>& k = lf.k;
      const auto& fp = P->fp();
      const auto& fi = P->fi();
      double* Sh = P->Shat.as<double>();
      for (int i = 0; i < P->nb; ++i)
        for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
          int j = fi[e];
          if (k[i] == 0 || k[j] == 0) continue;
          const int64_t o = kcoff[g][e];
          g1.one(Tmp[g] + o, k[i], k[i], k[j], k[j], Kc[g] + o, k[i], false,
                 rl.Tt.as<double>() + rl.offT[j], k[j], true);
          g2.one(Sh + P->shat_far_off[e], k[i], k[i], k[j], k[i], lf.Tt.as<double>() + lf.offT[i],
                 k[i], false, Tmp[g] + o, k[i], false);
        }
    }
    g1.run(st, "couple");
    g2.run(st, "couple");
    st.sync();
  } else {
    std::vector<DBuf> Kc32, T32, Tmp32;
    GemmBatch<float> g1;
    GemmBatch<float, double> g2;
    for (size_t g = 0; g < G.size(); ++g) {
      Prob* P = G[g];
      const LevelFactor& lf = P->lf();
      const std::vector<int>& k = lf.k;
      const auto& fp = P->fp();
      const auto& fi = P->fi();
      double* Sh = P->Shat.as<double>();
      Kc32.push_back(to_f32(Kc[g], kcoff[g].back(), s));
      T32.push_back(to_f32(lf.Tt.as<double>(), lf.offT[P->nb], s));
      Tmp32.emplace_back(std::max<int64_t>(kcoff[g].back(), 1) * sizeof(float));
      const float* Tf = T32.back().as<float>();
      const float* Kf = Kc32.back().as<float>();
      float* Tm = Tmp32.back().as<float>();
      for (int i = 0; i < P->nb; ++i)
        for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
          int j = fi[e];
          if (k[i] == 0 || k[j] == 0) continue;
          const int64_t o = kcoff[g][e];
          g1.one(Tm + o, k[i], k[i], k[j], k[j], Kf + o, k[i], false, Tf + lf.offT[j], k[j], true);
          g2.one(Sh + P->shat_far_off[e], k[i], k[i], k[j], k[i], Tf + lf.offT[i], k[i], false,
                 Tm + o, k[i], false);
        }
    }
    g1.run(st, "couple");
    g2.run(st, "couple");
    st.sync();
  }
}

// ---- (e) rotation -------------------------------------------------------------
void Driver::rotations(Stage& st, const std::vector<Prob*>& G) {
  std::vector<DBuf> U32(G.size());
  // off-diagonal near blocks: S_ij = U^S_i^T D_ij U^S_j
  {
    GemmBatch<double> g1, g2;
    GemmBatch<float> h1;
    GemmBatch<float, double> h2;
    for (size_t g = 0; g < G.size(); ++g) {
      Prob* P = G[g];
      const LevelFactor& lf = P->lf();
      const std::vector<int>& m = lf.m;
      const std::vector<int>& k = lf.k;
      const auto& np = P->np();
      const auto& ni = P->ni();
      std::vector<int64_t> toff(P->nnear() + 1, 0);
      for (int i = 0; i < P->nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e)
          toff[e + 1] = toff[e] + (int64_t)m[i] * k[ni[e]];
      for (int i = 0; i < P->nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e) {
          int j = ni[e];
          if (j == i || k[i] == 0 || k[j] == 0) continue;
          P->fl_rotate += 2.0 * m[i] * (double)m[j] * k[j] + 2.0 * k[i] * (double)m[i] * k[j];
        }
      double* Sh = P->Shat.as<double>();
      if (!mixed) {
        double* Tmp = st.scratch<double>(std::max<int64_t>(toff.back(), 1));
        const double* U = lf.U.as<double>();
        const LevelFactor& rl = P->rlf();  // V (= U for shared bases)
        const double* Dp = P->D.as<double>();
        for (int i = 0; i < P->nb; ++i)
          for (int64_t e = np[i]; e < np[i + 1]; ++e) {
            int j = ni[e];
            if (j == i || k[i] == 0 || k[j] == 0) continue;
            g1.one(Tmp + toff[e], m[i], m[i], k[j], m[j], Dp + P->Doff[e], m[i], false,
                   rl.U.as<double>() + rl.offU[j], m[j], false);
            g2.one(Sh + P->shat_near_off[e], k[i], k[i], k[j], m[i], U + lf.offU[i], m[i], true,
                   Tmp + toff[e], m[i], false);
          }
      } else {
        U32[g] = to_f32(lf.U.as<double>(), lf.offU[P->nb], s);
        float* Tmp = st.scratch<float>(std::max<int64_t>(toff.back(), 1));
        const float* U = U32[g].as<float>();
        const float* D32p = P->D32.as<float>();
        for (int i = 0; i < P->nb; ++i)
          for (int64_t e = np[i]; e < np[i + 1]; ++e) {
            int j = ni[e];
            if (j == i || k[i] == 0 || k[j] == 0) continue;
            h1.one(Tmp + toff[e], m[i], m[i], k[j], m[j], D32p + P->Doff[e], m[i], false,
                   U + lf.offU[j], m[j], false);
            h2.one(Sh + P->shat_near_off[e], k[i], k[i], k[j], m[i], U + lf.offU[i], m[i], true,
                   Tmp + toff[e], m[i], false);
          }
      }
    }
    g1.run(st, "rotate");
    g2.run(st, "rotate");
    h1.run(st, "rotate");
    h2.run(st, "rotate");
    st.sync();
  }
  // diagonal: S_ii = U_i^T D_ii U_i
  {
    std::vector<DBuf> Tmps;
    GemmBatch<double> g1, g2;
    GemmBatch<float> h1;
    GemmBatch<float, double> h2;
    for (size_t g = 0; g < G.size(); ++g) {
      Prob* P = G[g];
      const LevelFactor& lf = P->lf();
      const std::vector<int>& m = lf.m;
      const int nb = P->nb;
      P->S.alloc(std::max<int64_t>(P->offSq[nb], 1) * sizeof(double));
      double* Sp = P->S.as<double>();
      for (int i = 0; i < nb; ++i)
        if (m[i] > 0) P->fl_rotate += 4.0 * std::pow((double)m[i], 3);
      if (!mixed) {
        Tmps.emplace_back(std::max<int64_t>(P->offSq[nb], 1) * sizeof(double));
        double* Tmp = Tmps.back().as<double>();
        const double* U = lf.U.as<double>();
        const LevelFactor& rl = P->rlf();
        for (int i = 0; i < nb; ++i) {
          if (m[i] == 0) continue;
          g1.one(Tmp + P->offSq[i], m[i], m[i], m[i], m[i], P->Dblk(i, i), m[i], false,
                 rl.U.as<double>() + rl.offU[i], m[i], false);
          g2.one(Sp + P->offSq[i], m[i], m[i], m[i], m[i], U + lf.offU[i], m[i], true,
                 Tmp + P->offSq[i], m[i], false);
        }
      } else {
        Tmps.emplace_back(std::max<int64_t>(P->offSq[nb], 1) * sizeof(float));
        float* Tmp = Tmps.back().as<float>();
        const float* U = U32[g].as<float>();
        const float* D32p = P->D32.as<float>();
        for (int i = 0; i < nb; ++i) {
          if (m[i] == 0) continue;
          int64_t e = csr_find(P->np(), P->ni(), i, i);
          h1.one(Tmp + P->offSq[i], m[i], m[i], m[i], m[i], D32p + P->Doff[e], m[i], false,
                 U + lf.offU[i], m[i], false);
          h2.one(Sp + P->offSq[i], m[i], m[i], m[i], m[i], U + lf.offU[i], m[i], true,
                 Tmp + P->offSq[i], m[i], false);
        }
      }
    }
    g1.run(st, "rotate");
    g2.run(st, "rotate");
    h1.run(st, "rotate");
    h2.run(st, "rotate");
    st.sync();
  }
  for (Prob* P : G) {
    P->D.reset();
    P->D32.reset();
  }
}

// ---- (f) elimination: S^RR inverse, X = S^RR^-1 S^RS, S^SR copy and the Schur
// update into the new diagonal skeleton block
void Driver::elimination(Stage& st, const std::vector<Prob*>& G) {
  std::vector<DBuf> RRw;
  CopyBatch cb, cs, css;
  std::vector<SqMat> mats;
  std::vector<Prob*> owner;
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const int nb = P->nb;
    const std::vector<int>& m = lf.m;
    const std::vector<int>& k = lf.k;
    lf.offR.assign(nb + 1, 0);
    lf.offX.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      int r = m[i] - k[i];
      lf.offR[i + 1] = lf.offR[i] + (int64_t)r * r;
      lf.offX[i + 1] = lf.offX[i] + (int64_t)r * k[i];
    }
    lf.Sinv.alloc(std::max<int64_t>(lf.offR[nb], 1) * sizeof(double));
    lf.Xs.alloc(std::max<int64_t>(lf.offX[nb], 1) * sizeof(double));
    lf.SSR.alloc(std::max<int64_t>(lf.offX[nb], 1) * sizeof(double));
    RRw.emplace_back(std::max<int64_t>(lf.offR[nb], 1) * sizeof(double));
    double* RR = RRw.back().as<double>();
    double* Sh = P->Shat.as<double>();
    for (int i = 0; i < nb; ++i) {
      int r = m[i] - k[i], ki = k[i];
      const double* Si = P->S.as<double>() + P->offSq[i];
      if (r > 0) {
        cb.add(Si + ki + (int64_t)ki * m[i], m[i], RR + lf.offR[i], r, r, r);
        mats.push_back(SqMat{RR + lf.offR[i], r, r, lf.Sinv.as<double>() + lf.offR[i], r});
        owner.push_back(P);
        if (ki > 0) cs.add(Si + (int64_t)ki * m[i], m[i], lf.SSR.as<double>() + lf.offX[i], ki, ki, r);
        P->fl_elim += 2.0 / 3.0 * r * (double)r * r + 2.0 * ki * (double)r * r +
                      2.0 * ki * (double)ki * r;
      }
      if (ki > 0) {
        int64_t e = csr_find(P->np(), P->ni(), i, i);
        css.add(Si, m[i], Sh + P->shat_near_off[e], ki, ki, ki);
      }
    }
  }
  cb.run(st);
  cs.run(st);
  css.run(st);
  int32_t* info = nullptr;
  int32_t* ipiv = nullptr;
  std::vector<int64_t> ipo;
  batched_inverse(st, mats, &info, &ipiv, &ipo);
  // log|det S^RR| from the LU diagonals
  if (!mats.empty()) {
    std::vector<MatDesc> ds;
    for (auto& mt : mats) {
      MatDesc d{};
      d.A = mt.A;
      d.lda = mt.lda;
      d.m = mt.m;
      ds.push_back(d);
    }
    int nd = (int)ds.size();
    double* ld = st.scratch<double>(nd);
    MatDesc* dd = st.up(std::move(ds));
    launch_logdet(dd, nd, ld, s);
    std::vector<double> hl(nd);
    H2ULV_HIP(hipMemcpyAsync(hl.data(), ld, nd * sizeof(double), hipMemcpyDeviceToHost, s));
    check_info(info, mats.size(), s, "S^RR (elimination step)");
    for (int q = 0; q < nd; ++q) owner[q]->F->stats.logabsdet += hl[q];
  }
  GemmBatch<double> g1, g2;
  GemmBatch<float, double> g3;
  std::vector<DBuf> SSR32, X32;
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const std::vector<int>& m = lf.m;
    const std::vector<int>& k = lf.k;
    for (int i = 0; i < P->nb; ++i) {
      int r = m[i] - k[i], ki = k[i];
      if (r == 0 || ki == 0) continue;
      const double* Si = P->S.as<double>() + P->offSq[i];
      g1.one(lf.Xs.as<double>() + lf.offX[i], r, r, ki, r, lf.Sinv.as<double>() + lf.offR[i], r,
             false, Si + ki, m[i], false);
    }
  }
  g1.run(st, "elim");
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const std::vector<int>& m = lf.m;
    const std::vector<int>& k = lf.k;
    double* Sh = P->Shat.as<double>();
    const float* S32 = nullptr;
    const float* X32p = nullptr;
    if (mixed) {
      SSR32.push_back(to_f32(lf.SSR.as<double>(), lf.offX[P->nb], s));
      X32.push_back(to_f32(lf.Xs.as<double>(), lf.offX[P->nb], s));
      S32 = SSR32.back().as<float>();
      X32p = X32.back().as<float>();
    }
    for (int i = 0; i < P->nb; ++i) {
      int r = m[i] - k[i], ki = k[i];
      if (r == 0 || ki == 0) continue;
      int64_t e = csr_find(P->np(), P->ni(), i, i);
      if (!mixed)
        g2.one(Sh + P->shat_near_off[e], ki, ki, ki, r, lf.SSR.as<double>() + lf.offX[i], ki,
               false, lf.Xs.as<double>() + lf.offX[i], r, false, -1.0, 1.0);
      else
        g3.one(Sh + P->shat_near_off[e], ki, ki, ki, r, S32 + lf.offX[i], ki, false,
               X32p + lf.offX[i], r, false, -1.0, 1.0);
    }
  }
  g2.run(st, "elim");
  g3.run(st, "elim");
  st.sync();
}

void Driver::level(const std::vector<Prob*>& G) {
  Stage st(s);
  for (Prob* P : G) {
    LevelFactor& lf = P->lf();
    const int nb = 1 << P->lev;
    P->nb = nb;
    lf.lev = P->lev;
    lf.nb = nb;
    lf.m.resize(nb);
    P->cand_off.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      lf.m[i] = (int)lf.cand[i].size();
      P->cand_off[i + 1] = P->cand_off[i] + lf.m[i];
    }
    // candidate rows on the device as indices into the shared point buffer;
    // the host vector stays alive until the level ends
    P->cand_all.clear();
    P->cand_all.reserve(P->cand_off[nb]);
    for (int i = 0; i < nb; ++i)
      for (int64_t a : lf.cand[i]) P->cand_all.push_back(a + P->poff);
    P->dcand.alloc(std::max<int64_t>(P->cand_off[nb], 1) * sizeof(int64_t));
    if (P->cand_off[nb] > 0)
      H2ULV_HIP(hipMemcpyAsync(P->dcand.p, P->cand_all.data(), P->cand_off[nb] * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
  }
  tick(nullptr);
  dense_blocks(st, G);
  tick("a_dense");
  basis_prepare(st, G);
  fill_products(st, G);
  tick("b_zprod");
  row_ids(st, G);
  bases(st, G);
  tick("c_basis_qr");
  // the column sides (separate bases) stop after their bases: the row side
  // rotates with both and eliminates
  std::vector<Prob*> rows;
  for (Prob* P : G)
    if (!P->colside) rows.push_back(P);
  couplings(st, rows);
  tick("d_couple");
  rotations(st, rows);
  tick("e_rotate");
  elimination(st, rows);
  tick("f_elim");
  st.sync();
  for (Prob* P : G) {
    // next level's candidate rows: the children's skeletons (the flat
    // structure has no next level: its root takes every leaf skeleton)
    if (P->lev > 1 && p.structure == 0) {
      LevelFactor& lf = P->lf();
      LevelFactor& pa = P->F->levels[P->lev - 1];
      pa.cand.assign(P->nb / 2, {});
      for (int q = 0; q < P->nb / 2; ++q) {
        pa.cand[q] = lf.sk[2 * q];
        pa.cand[q].insert(pa.cand[q].end(), lf.sk[2 * q + 1].begin(), lf.sk[2 * q + 1].end());
      }
    }
    P->end_level();
  }
}

void Driver::roots(const std::vector<Prob*>& G) {
  Stage st(s);
  std::vector<DBuf> D0(G.size());
  KgenBatch kb;
  CopyBatch cb;
  std::vector<int64_t> perms;
  std::vector<int64_t> permoff(G.size(), 0);
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    if (P->L() != 0) continue;
    permoff[g] = (int64_t)perms.size();
    for (int64_t a : P->F->tree.perm) perms.push_back(a + P->poff);
  }
  const int64_t* dperm = st.up(std::move(perms));
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    h2ulv_factor& F = *P->F;
    int m0;
    if (P->L() == 0) {
      m0 = (int)F.n;
      D0[g].alloc((size_t)m0 * m0 * sizeof(double));
      kb.add(dperm + permoff[g], m0, dperm + permoff[g], m0, D0[g].as<double>(), m0);
      P->kevals += (double)m0 * m0;
    } else {
      // the skeleton blocks of the top factored level: the two children of the
      // root, or (flat) every leaf, in box order (Eq. BLR2final)
      const int top = p.structure == 1 ? P->L() : 1;
      const std::vector<int>& k = F.levels[top].k;
      const int nt = 1 << top;
      m0 = 0;
      for (int a = 0; a < nt; ++a) m0 += k[a];
      D0[g].alloc(std::max<size_t>((size_t)m0 * m0, 1) * sizeof(double));
      int ro = 0;
      for (int a = 0; a < nt; ++a) {
        int co = 0;
        for (int b = 0; b < nt; ++b) {
          if (k[a] > 0 && k[b] > 0) {
            int64_t ld;
            const double* src = P->shat_block(top, a, b, &ld);
            cb.add(src, std::max<int64_t>(ld, 1), D0[g].as<double>() + ro + (int64_t)co * m0,
                   m0, k[a], k[b]);
          }
          co += k[b];
        }
        ro += k[a];
      }
    }
    F.m_root = m0;
    F.root_inv.alloc(std::max<size_t>((size_t)m0 * m0, 1) * sizeof(double));
  }
  kb.run(st, pts, kf, dup);
  cb.run(st);
  st.sync();
  check_dup();
  for (Prob* P : G) P->Shat.reset();
  std::vector<SqMat> mats;
  std::vector<Prob*> owner;
  std::vector<MatDesc> ds;
  for (size_t g = 0; g < G.size(); ++g) {
    Prob* P = G[g];
    const int m0 = P->F->m_root;
    if (m0 == 0) continue;
    mats.push_back(SqMat{D0[g].as<double>(), m0, m0, P->F->root_inv.as<double>(), m0});
    owner.push_back(P);
    MatDesc d{};
    d.A = D0[g].as<double>();
    d.lda = m0;
    d.m = m0;
    ds.push_back(d);
    P->fl_root += 2.0 / 3.0 * std::pow((double)m0, 3);
  }
  if (!mats.empty()) {
    int32_t* info = nullptr;
    batched_inverse(st, mats, &info, nullptr, nullptr);
    int nd = (int)ds.size();
    double* ld = st.scratch<double>(nd);
    MatDesc* dd = st.up(std::move(ds));
    launch_logdet(dd, nd, ld, s);
    std::vector<double> hl(nd);
    H2ULV_HIP(hipMemcpyAsync(hl.data(), ld, nd * sizeof(double), hipMemcpyDeviceToHost, s));
    check_info(info, mats.size(), s, "the root block");
    for (int q = 0; q < nd; ++q) owner[q]->F->stats.logabsdet += hl[q];
  }
  st.sync();
}

}  // namespace

std::vector<h2ulv_factor*> factorize_many(const std::vector<const double*>& pts,
                                          const std::vector<int64_t>& n,
                                          const h2ulv_params& params, hipStream_t s) {
  validate_params(&params);
  const size_t np = pts.size();
  double t0 = now_s();
  std::vector<std::unique_ptr<h2ulv_factor>> F(np);
  int64_t ntot = 0;
  for (size_t q = 0; q < np; ++q) {
    if (!pts[q]) fail(H2ULV_ERR_INVALID_ARG, "pts is NULL");
    if (n[q] < 1) fail(H2ULV_ERR_INVALID_ARG, "n must be >= 1");
    if (n[q] > ((int64_t)1 << 31) - 1) fail(H2ULV_ERR_INVALID_ARG, "n too large");
    ntot += n[q];
  }
  for (size_t q = 0; q < np; ++q) {
    std::vector<double> hp(n[q] * 3);
    H2ULV_HIP(hipMemcpyAsync(hp.data(), pts[q], n[q] * 3 * sizeof(double), hipMemcpyDeviceToHost,
                             s));
    H2ULV_HIP(hipStreamSynchronize(s));
    for (double v : hp)
      if (!std::isfinite(v)) fail(H2ULV_ERR_INVALID_ARG, "non-finite point coordinate");
    F[q] = std::make_unique<h2ulv_factor>();
    F[q]->p = params;
    F[q]->p.rank_model = nullptr;  // the factor does not keep the model
    F[q]->n = n[q];
    F[q]->tree = build_tree(hp.data(), n[q], params.leaf_size, params.partition);
    F[q]->lists = build_structure_lists(F[q]->tree, params);
    F[q]->hpts = std::move(hp);
  }
  // separate bases: each problem gets its column side, a factor of the
  // transposed matrix on the same tree (bases only)
  const bool two = separate_bases(params);
  std::vector<std::unique_ptr<h2ulv_factor>> FV(two ? np : 0);
  for (size_t q = 0; q < FV.size(); ++q) {
    FV[q] = std::make_unique<h2ulv_factor>();
    FV[q]->p = F[q]->p;
    FV[q]->n = F[q]->n;
    FV[q]->tree = F[q]->tree;
    FV[q]->lists = F[q]->lists;
    FV[q]->hpts = F[q]->hpts;
  }
  double t1 = now_s();
  if (params.verbose) std::fprintf(stderr, "[h2ulv] host setup (tree, lists) %.3f s\n", t1 - t0);
  for (size_t q = 0; q < np; ++q) {
    h2ulv_factor& f = *F[q];
    f.pts.alloc(f.n * 3 * sizeof(double));
    H2ULV_HIP(hipMemcpyAsync(f.pts.p, pts[q], f.n * 3 * sizeof(double), hipMemcpyDeviceToDevice,
                             s));
    f.perm.alloc(f.n * sizeof(int64_t));
    H2ULV_HIP(hipMemcpyAsync(f.perm.p, f.tree.perm.data(), f.n * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    H2ULV_HIP(hipStreamSynchronize(s));
  }
  // one point buffer for every kernel evaluation of the batch
  DBuf shared;
  std::vector<Prob> probs(two ? 2 * np : np);
  const double* allpts = F[0]->pts.as<double>();
  if (np > 1) {
    shared.alloc(ntot * 3 * sizeof(double));
    int64_t off = 0;
    for (size_t q = 0; q < np; ++q) {
      H2ULV_HIP(hipMemcpyAsync(shared.as<double>() + off * 3, F[q]->pts.p,
                               F[q]->n * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
      probs[q].poff = off;
      off += F[q]->n;
    }
    allpts = shared.as<double>();
  }
  mem_stats().peak = mem_stats().live;
  Driver drv(s, params);
  drv.pts = allpts;
  for (size_t q = 0; q < FV.size(); ++q) {
    Prob& C = probs[np + q];
    C.F = FV[q].get();
    C.poff = probs[q].poff;
    C.colside = true;
    C.partner = &probs[q];
    probs[q].partner = &C;
  }
  int H = 0;
  for (size_t q = 0; q < probs.size(); ++q) {
    Prob& P = probs[q];
    h2ulv_factor& f = q < np ? *F[q] : *FV[q - np];
    P.F = &f;
    const int L = f.tree.L;
    H = std::max(H, L);
    f.levels.resize(L + 1);
    if (L == 0) continue;
    LevelFactor& lf = f.levels[L];
    lf.cand.resize((size_t)1 << L);
    for (int i = 0; i < (1 << L); ++i)
      lf.cand[i].assign(f.tree.perm.begin() + f.tree.start[L][i],
                        f.tree.perm.begin() + f.tree.end[L][i]);
  }
  // levels aligned by height above the leaves; the active problems of a height
  // are split into groups whose level buffers fit the free device memory.  The
  // flat structure has the leaf level only.
  const bool flat = params.structure == 1;
  for (int h = 0; h < (flat ? std::min(H, 1) : H); ++h) {
    // a problem and its column side stay in one group
    std::vector<Prob*> act;
    for (size_t q = 0; q < np; ++q) {
      Prob& P = probs[q];
      if (P.F->tree.L - h < 1) continue;
      for (Prob* Q : {&P, P.partner}) {
        if (!Q) continue;
        Q->lev = Q->F->tree.L - h;
        Q->nb = 1 << Q->lev;
        act.push_back(Q);
      }
    }
    const size_t freeb = free_device_bytes();
    const double cap = 0.45 * (double)freeb;
    const bool mixed = params.precision == H2ULV_MIXED;
    size_t a0 = 0;
    while (a0 < act.size()) {
      double t_lev = now_s();
      std::vector<Prob*> grp;
      double acc = 0;
      while (a0 < act.size()) {
        const size_t w = act[a0]->partner ? 2 : 1;
        double b = 0;
        for (size_t u = 0; u < w; ++u) b += act[a0 + u]->level_bytes(mixed);
        if (!grp.empty() && acc + b > cap) break;
        acc += b;
        for (size_t u = 0; u < w; ++u) grp.push_back(act[a0++]);
      }
      drv.level(grp);
      if (params.verbose) {
        int mm = 0, mk = 0, nbx = 0;
        for (Prob* P : grp) {
          const LevelFactor& lf = P->F->levels[P->lev];
          nbx += lf.nb;
          for (int x : lf.m) mm = std::max(mm, x);
          for (int x : lf.k) mk = std::max(mk, x);
        }
        std::fprintf(stderr, "[h2ulv] height %d: %zu problem(s), %d boxes, max m %d, max k %d, "
                     "%.3f s, live %.1f GB, cached %.1f GB, cache releases %lld |", h, grp.size(),
                     nbx, mm, mk, now_s() - t_lev, mem_stats().live / 1e9, cache_bytes() / 1e9,
                     (long long)cache_oom_releases());
        for (auto& kv : drv.step_time) std::fprintf(stderr, " %s %.3f", kv.first.c_str(), kv.second);
        std::fprintf(stderr, "\n");
        drv.step_time.clear();
      }
    }
  }
  {
    std::vector<Prob*> all;
    for (size_t q = 0; q < np; ++q) all.push_back(&probs[q]);
    drv.roots(all);
  }
  H2ULV_HIP(hipStreamSynchronize(s));
  double t2 = now_s();
  std::vector<h2ulv_factor*> out(np);
  for (size_t q = 0; q < np; ++q) {
    Prob& P = probs[q];
    h2ulv_factor& f = *F[q];
    h2ulv_stats& st = f.stats;
    st.levels = f.tree.L;
    st.n = f.n;
    st.root_size = f.m_root;
    int mx = 0;
    for (auto& lf : f.levels)
      for (int x : lf.k) mx = std::max(mx, x);
    st.max_rank = mx;
    // the column side's work (separate bases) is part of the factorization
    const Prob* C = P.partner;
    st.flops_fill = P.fl_fill + (C ? C->fl_fill : 0.0);
    st.flops_basis = P.fl_basis + (C ? C->fl_basis : 0.0);
    st.flops_couple = P.fl_couple;
    st.flops_rotate = P.fl_rotate;
    st.flops_elim = P.fl_elim;
    st.flops_root = P.fl_root;
    st.kernel_evals = P.kevals + (C ? C->kevals : 0.0);
    st.time_setup_s = t1 - t0;
    st.time_factor_s = t2 - t0;
    st.device_bytes = (double)mem_stats().peak;
  }
  for (size_t q = 0; q < FV.size(); ++q) F[q]->colview = std::move(FV[q]);
  for (size_t q = 0; q < np; ++q) out[q] = F[q].release();
  return out;
}

}  // namespace h2ulv
