// H^2-ULV factorization without trailing sub-matrix dependencies: level driver
// and C-ABI.  Each level of the tree is one batched pass over all of its boxes
// (Sec. III of Ma, Deshmukh, Yokota, arXiv 2208.10907):
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
// then the root block is inverted (Eq. BLR2final).  Ranks are read back once
// per level to size the next level.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>

#include "h2ulv_dense.h"

namespace h2ulv {

static thread_local std::string g_last_error;

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ---------------------------------------------------------------------------
// factor storage
// ---------------------------------------------------------------------------
struct LevelFactor {
  int lev = 0;
  int nb = 0;
  std::vector<int> m, k;
  std::vector<std::vector<int64_t>> cand;  // candidate point indices per box
  std::vector<std::vector<int64_t>> sk;    // skeleton point indices per box
  // device storage (one arena each): U (m x m), Sinv (r x r), X = Sinv S^RS (r x k),
  // SSR = S^SR (k x r), T (k x k)
  DBuf U, Sinv, Xs, SSR, Tt;
  std::vector<int64_t> offU, offR, offX, offT;
};

}  // namespace h2ulv

struct h2ulv_factor {
  h2ulv_params p{};
  int64_t n = 0;
  h2ulv::Tree tree;
  h2ulv::Lists lists;
  h2ulv::DBuf pts;   // device copy of the points (n x 3)
  h2ulv::DBuf perm;  // device tree permutation
  std::vector<h2ulv::LevelFactor> levels;  // index = level (0 unused)
  h2ulv::DBuf root_inv;
  int m_root = 0;
  h2ulv_stats stats{};
};

struct h2ulv_structure {
  h2ulv::Tree tree;
  h2ulv::Lists lists;
};

namespace h2ulv {

static KernelFn kfn(const h2ulv_params& p) { return KernelFn{p.kernel, p.alpha, p.diag}; }

// float copy of a device array (mixed precision: operands of the FP32 products)
static DBuf to_f32(const double* src, int64_t count, hipStream_t s) {
  DBuf b(std::max<int64_t>(count, 1) * sizeof(float));
  launch_convert_d2f(src, b.as<float>(), count, s);
  H2ULV_HIP(hipGetLastError());
  return b;
}

// far-field column indices of box i at level lev (see the oracle's docstring for
// the two modes): exact = every point outside the near boxes; sampled = all
// candidate rows of the own-level far boxes + strided samples of ancestors' far
// boxes (all points of a box holding at most s points).
static std::vector<int64_t> far_columns(const Tree& t, const Lists& ls, int lev, int i,
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

static std::vector<int> fill_targets(const Lists& ls, int lev, int i) {
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

static int64_t csr_find(const std::vector<int64_t>& ptr, const std::vector<int32_t>& idx, int i,
                        int j) {
  auto b = idx.begin() + ptr[i], e = idx.begin() + ptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it != e && *it == j) return it - idx.begin();
  return -1;
}

static void check_info(const int32_t* dinfo, size_t n, hipStream_t s, const char* what) {
  if (!dinfo || n == 0) return;
  std::vector<int32_t> h(n);
  H2ULV_HIP(hipMemcpyAsync(h.data(), dinfo, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i)
    if (h[i] != 0)
      fail(H2ULV_ERR_SINGULAR, std::string("zero or non-finite pivot in ") + what);
}

// ---------------------------------------------------------------------------
// The factorization
// ---------------------------------------------------------------------------
struct Factorizer {
  h2ulv_factor& F;
  hipStream_t s;
  KernelFn kf;
  int* dup = nullptr;  // device flag
  DBuf dupbuf;
  double flops_fill = 0, flops_basis = 0, flops_couple = 0, flops_rotate = 0, flops_elim = 0,
         flops_root = 0, kevals = 0;

  // skeleton blocks of the level just finished, keyed by CSR position
  DBuf Shat;
  std::vector<int64_t> shat_near_off, shat_far_off;
  int shat_lev = -1;

  // per-step wall times (verbose mode synchronises at each step)
  std::map<std::string, double> step_time;
  double t_last = 0;
  void tick(const char* name) {
    if (!F.p.verbose) return;
    H2ULV_HIP(hipStreamSynchronize(s));
    double t = now_s();
    if (name) step_time[name] += t - t_last;
    t_last = t;
  }

  Factorizer(h2ulv_factor& f, hipStream_t st) : F(f), s(st), kf(kfn(f.p)) {
    dupbuf.alloc(sizeof(int));
    dup = dupbuf.as<int>();
    H2ULV_HIP(hipMemsetAsync(dup, 0, sizeof(int), s));
  }

  const double* shat_block(int lev, int c, int d, int64_t* ld) {
    const Lists& ls = F.lists;
    *ld = F.levels[lev].k[c];
    int64_t e = csr_find(ls.near_ptr[lev], ls.near_idx[lev], c, d);
    if (e >= 0) return Shat.as<double>() + shat_near_off[e];
    e = csr_find(ls.far_ptr[lev], ls.far_idx[lev], c, d);
    if (e < 0) fail(H2ULV_ERR_HIP, "internal: child pair is neither near nor far");
    return Shat.as<double>() + shat_far_off[e];
  }

  void check_dup() {
    int h = 0;
    H2ULV_HIP(hipMemcpyAsync(&h, dup, sizeof(int), hipMemcpyDeviceToHost, s));
    H2ULV_HIP(hipStreamSynchronize(s));
    if (h) fail(H2ULV_ERR_DUPLICATE_POINTS, "two distinct points coincide");
  }

  void run();
  void level(int lev);
  void root();
};

void Factorizer::run() {
  const int L = F.tree.L;
  F.levels.resize(L + 1);
  if (L == 0) {
    root();
    return;
  }
  // leaf candidate rows
  LevelFactor& lf = F.levels[L];
  lf.lev = L;
  lf.nb = 1 << L;
  lf.cand.resize(lf.nb);
  for (int i = 0; i < lf.nb; ++i)
    lf.cand[i].assign(F.tree.perm.begin() + F.tree.start[L][i],
                      F.tree.perm.begin() + F.tree.end[L][i]);
  for (int lev = L; lev >= 1; --lev) {
    double t0 = now_s();
    level(lev);
    if (F.p.verbose) {
      int mx = 0;
      for (int x : F.levels[lev].k) mx = std::max(mx, x);
      std::fprintf(stderr, "[h2ulv] level %d: %d boxes, max m %d, max k %d, %.3f s |", lev,
                   1 << lev, *std::max_element(F.levels[lev].m.begin(), F.levels[lev].m.end()),
                   mx, now_s() - t0);
      for (auto& kv : step_time) std::fprintf(stderr, " %s %.3f", kv.first.c_str(), kv.second);
      std::fprintf(stderr, "\n");
      step_time.clear();
    }
  }
  root();
}

void Factorizer::level(int lev) {
  const Tree& T = F.tree;
  const Lists& ls = F.lists;
  const int L = T.L;
  const int nb = 1 << lev;
  LevelFactor& lf = F.levels[lev];
  lf.lev = lev;
  lf.nb = nb;
  std::vector<int>& m = lf.m;
  m.resize(nb);
  for (int i = 0; i < nb; ++i) m[i] = (int)lf.cand[i].size();
  const auto& np = ls.near_ptr[lev];
  const auto& ni = ls.near_idx[lev];
  const auto& fp = ls.far_ptr[lev];
  const auto& fi = ls.far_idx[lev];
  const int64_t nnear = np[nb], nfar = fp[nb];
  Stage st(s);

  // candidate rows on the device
  std::vector<int64_t> cand_off(nb + 1, 0);
  for (int i = 0; i < nb; ++i) cand_off[i + 1] = cand_off[i] + m[i];
  std::vector<int64_t> cand_all;
  cand_all.reserve(cand_off[nb]);
  for (int i = 0; i < nb; ++i) cand_all.insert(cand_all.end(), lf.cand[i].begin(), lf.cand[i].end());
  // level-scope device copy (the stage frees its uploads at every sync)
  DBuf dcand_buf(std::max<int64_t>(cand_off[nb], 1) * sizeof(int64_t));
  if (cand_off[nb] > 0)
    H2ULV_HIP(hipMemcpyAsync(dcand_buf.p, cand_all.data(), cand_off[nb] * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
  const int64_t* dcand = dcand_buf.as<int64_t>();
  auto candp = [&](int i) { return dcand + cand_off[i]; };

  tick(nullptr);
  // ---- (a) dense blocks -------------------------------------------------
  std::vector<int64_t> Doff(nnear + 1, 0);
  for (int i = 0; i < nb; ++i)
    for (int64_t e = np[i]; e < np[i + 1]; ++e)
      Doff[e + 1] = Doff[e] + (int64_t)m[i] * m[ni[e]];
  DBuf D(std::max<int64_t>(Doff[nnear], 1) * sizeof(double));
  double* Dp = D.as<double>();
  auto Dblk = [&](int i, int j) -> double* {
    int64_t e = csr_find(np, ni, i, j);
    return Dp + Doff[e];
  };
  if (lev == L) {
    KgenBatch kb;
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        int j = ni[e];
        kb.add(candp(i), m[i], candp(j), m[j], Dp + Doff[e], m[i]);
        kevals += (double)m[i] * m[j];
      }
    kb.run(st, F.pts.as<double>(), kf, dup);
  } else {
    CopyBatch cb;
    const std::vector<int>& kc = F.levels[lev + 1].k;
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        int j = ni[e];
        double* out = Dp + Doff[e];
        int rows[2] = {2 * i, 2 * i + 1}, cols[2] = {2 * j, 2 * j + 1};
        int ro = 0;
        for (int a = 0; a < 2; ++a) {
          int co = 0;
          for (int b = 0; b < 2; ++b) {
            int64_t ld;
            const double* src = shat_block(lev + 1, rows[a], cols[b], &ld);
            cb.add(src, std::max<int64_t>(ld, 1), out + ro + (int64_t)co * m[i], m[i],
                   kc[rows[a]], kc[cols[b]]);
            co += kc[cols[b]];
          }
          ro += kc[rows[a]];
        }
      }
    cb.run(st);
  }
  st.sync();
  Shat.reset();  // children's skeleton blocks are merged now
  tick("a_dense");

  // ---- (b) fill-ins: inverses of the diagonal blocks and Z'_ik = T^-1 D_ik D_kk^-1
  std::vector<int64_t> offSq(nb + 1, 0);
  for (int i = 0; i < nb; ++i) offSq[i + 1] = offSq[i] + (int64_t)m[i] * m[i];
  DBuf Dinv(std::max<int64_t>(offSq[nb], 1) * sizeof(double));
  {
    DBuf LUw(std::max<int64_t>(offSq[nb], 1) * sizeof(double));
    CopyBatch cb;
    std::vector<SqMat> mats;
    for (int i = 0; i < nb; ++i) {
      if (m[i] == 0) continue;
      cb.add(Dblk(i, i), m[i], LUw.as<double>() + offSq[i], m[i], m[i], m[i]);
      mats.push_back(SqMat{LUw.as<double>() + offSq[i], m[i], m[i],
                           Dinv.as<double>() + offSq[i], m[i]});
      flops_fill += 2.0 / 3.0 * std::pow((double)m[i], 3);
    }
    cb.run(st);
    int32_t* info = nullptr;
    batched_inverse(st, mats, &info, nullptr, nullptr);
    check_info(info, mats.size(), s, "a diagonal block (fill-in step)");
    st.sync();
  }
  tick("b_inverse");
  // inverse T factors of the children (T-hat^-1 is block diagonal)
  const bool upper = lev < L;
  // mixed precision: the rotations, low-rank couplings and Schur updates run on
  // FP32 matrix cores with FP32 accumulation; the fill-in products stay FP64
  // because they feed the rank-revealing QR, whose decisions at tol ~1e-6 sit at
  // FP32 rounding level (FP32 fill-ins inflate the upper-level ranks several
  // times); inverses, QR/ID, solve and residual are FP64 as well
  const bool mixed = F.p.precision == H2ULV_MIXED;
  std::vector<int64_t> offTinv;
  DBuf Tinv;
  if (upper) {
    const LevelFactor& ch = F.levels[lev + 1];
    offTinv.assign(2 * nb + 1, 0);
    for (int c = 0; c < 2 * nb; ++c) offTinv[c + 1] = offTinv[c] + (int64_t)ch.k[c] * ch.k[c];
    Tinv.alloc(std::max<int64_t>(offTinv[2 * nb], 1) * sizeof(double));
    DBuf Tw(std::max<int64_t>(offTinv[2 * nb], 1) * sizeof(double));
    CopyBatch cb;
    std::vector<SqMat> mats;
    for (int c = 0; c < 2 * nb; ++c) {
      if (ch.k[c] == 0) continue;
      cb.add(ch.Tt.as<double>() + ch.offT[c], ch.k[c], Tw.as<double>() + offTinv[c], ch.k[c],
             ch.k[c], ch.k[c]);
      mats.push_back(SqMat{Tw.as<double>() + offTinv[c], ch.k[c], ch.k[c],
                           Tinv.as<double>() + offTinv[c], ch.k[c]});
    }
    cb.run(st);
    batched_triu_inverse(st, mats);
    st.sync();
  }
  // Z'_ik for k in Near(i) \ {i}, stored at the CSR position of (i, k)
  DBuf Z(std::max<int64_t>(Doff[nnear], 1) * sizeof(double));
  double* Zp = Z.as<double>();
  {
    DBuf Ztmp;
    double* Zt = Zp;
    if (upper) {
      Ztmp.alloc(std::max<int64_t>(Doff[nnear], 1) * sizeof(double));
      Zt = Ztmp.as<double>();
    }
    GemmBatch<double> g;
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        int k = ni[e];
        if (k == i || m[i] == 0 || m[k] == 0) continue;
        g.one(Zt + Doff[e], m[i], m[i], m[k], m[k], Dp + Doff[e], m[i], false,
              Dinv.as<double>() + offSq[k], m[k], false);
        flops_fill += 2.0 * m[i] * (double)m[k] * m[k];
      }
    g.run(st);
    if (upper) {
      const LevelFactor& ch = F.levels[lev + 1];
      GemmBatch<double> g2;
      for (int i = 0; i < nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e) {
          int k = ni[e];
          if (k == i || m[i] == 0 || m[k] == 0) continue;
          int k1 = ch.k[2 * i], k2 = ch.k[2 * i + 1];
          if (k1 > 0)
            g2.one(Zp + Doff[e], m[i], k1, m[k], k1, Tinv.as<double>() + offTinv[2 * i], k1,
                   false, Zt + Doff[e], m[i], false);
          if (k2 > 0)
            g2.one(Zp + Doff[e] + k1, m[i], k2, m[k], k2,
                   Tinv.as<double>() + offTinv[2 * i + 1], k2, false, Zt + Doff[e] + k1, m[i],
                   false);
        }
      g2.run(st);
    }
    st.sync();
  }
  Dinv.reset();
  tick("b_zprod");

  // ---- (c) shared bases, chunked over boxes by memory -----------------------
  lf.k.assign(nb, 0);
  lf.sk.assign(nb, {});
  std::vector<std::vector<int32_t>> piv(nb);
  std::vector<std::vector<int>> targets(nb);
  std::vector<std::vector<int64_t>> farcols(nb);
  std::vector<int64_t> ncols(nb, 0);
  for (int i = 0; i < nb; ++i) {
    targets[i] = fill_targets(ls, lev, i);
    farcols[i] = far_columns(T, ls, lev, i, lf.cand, F.p.far_sample);
    int64_t nc = (int64_t)farcols[i].size();
    for (int j : targets[i]) nc += m[j];
    ncols[i] = nc;
  }
  DBuf D32;
  if (mixed) D32 = to_f32(Dp, Doff[nnear], s);
  // per-box pivoted-QR matrices (m x m) kept until W' is built
  DBuf PQ(std::max<int64_t>(offSq[nb], 1) * sizeof(double));
  DBuf pivd(std::max<int64_t>(cand_off[nb], 1) * sizeof(int32_t));
  DBuf kd(std::max(nb, 1) * sizeof(int32_t));
  H2ULV_HIP(hipMemsetAsync(PQ.p, 0, PQ.bytes, s));
  {
    size_t freeb = 0, totb = 0;
    H2ULV_HIP(hipMemGetInfo(&freeb, &totb));
    int64_t budget = (int64_t)(freeb * 0.4) / (int64_t)sizeof(double);
    budget = std::max<int64_t>(budget, 1 << 20);
    auto box_words = [&](int i) {
      // M'^T plus the QR workspaces of its chunks (reflector panels, T, GEMM scratch)
      return (int64_t)m[i] * ncols[i] * 3 / 2 + 8 * (int64_t)m[i] * m[i] + 4096;
    };
    int i0 = 0;
    while (i0 < nb) {
      int i1 = i0;
      int64_t acc = 0;
      while (i1 < nb && (i1 == i0 || acc + box_words(i1) <= budget)) {
        acc += box_words(i1);
        ++i1;
      }
      // M'^T (ncols x m, column-major): far-field rows then fill-in rows
      std::vector<int64_t> moff(i1 - i0 + 1, 0);
      for (int i = i0; i < i1; ++i) moff[i - i0 + 1] = moff[i - i0] + (int64_t)m[i] * ncols[i];
      DBuf Mb(std::max<int64_t>(moff.back(), 1) * sizeof(double));
      double* Mp = Mb.as<double>();
      KgenBatch kb;
      GemmBatch<double> g;
      std::vector<int64_t> fc_all;
      std::vector<int64_t> fc_off;
      for (int i = i0; i < i1; ++i) {
        fc_off.push_back((int64_t)fc_all.size());
        fc_all.insert(fc_all.end(), farcols[i].begin(), farcols[i].end());
      }
      const int64_t* dfc = st.up(std::move(fc_all));
      for (int i = i0; i < i1; ++i) {
        if (m[i] == 0) continue;
        double* Mi = Mp + moff[i - i0];
        const int64_t ld = ncols[i];
        int64_t nf = (int64_t)farcols[i].size();
        kb.add(dfc + fc_off[i - i0], (int)nf, candp(i), m[i], Mi, ld);
        kevals += (double)m[i] * nf;
        int64_t row = nf;
        for (int j : targets[i]) {
          if (m[j] > 0) {
            // (T^-1 F_ij)^T = sum_k D_kj^T Z'_ik^T
            g.item(Mi + row, ld, m[j], m[i]);
            for (int64_t e = np[i]; e < np[i + 1]; ++e) {
              int k = ni[e];
              if (k == i || k == j || m[k] == 0) continue;
              int64_t ekj = csr_find(np, ni, k, j);
              if (ekj < 0) continue;
              g.term(Dp + Doff[ekj], m[k], true, Zp + Doff[e], m[i], true, m[k]);
              flops_fill += 2.0 * m[i] * (double)m[k] * m[j];
            }
          }
          row += m[j];
        }
      }
      kb.run(st, F.pts.as<double>(), kf, dup);
      g.run(st);
      tick("c_fill_gemm");
      // tall QR of every M'^T: a tree of blocked Householder QRs (leaf chunks of
      // 4m rows factored in place, then stacked triangles merged pairwise)
      struct Rref {
        double* p;
        int64_t ld;
        int r;
      };
      std::vector<std::vector<Rref>> cur(i1 - i0);
      std::vector<TallQr> leaf;
      for (int i = i0; i < i1; ++i) {
        if (m[i] == 0 || ncols[i] == 0) continue;
        double* Mi = Mp + moff[i - i0];
        const int64_t h = std::max<int64_t>(4 * (int64_t)m[i], 256);
        for (int64_t r0 = 0; r0 < ncols[i]; r0 += h) {
          int hc = (int)std::min<int64_t>(h, ncols[i] - r0);
          leaf.push_back(TallQr{Mi + r0, ncols[i], hc, m[i]});
          cur[i - i0].push_back(Rref{Mi + r0, ncols[i], std::min(hc, m[i])});
        }
        double nc = (double)ncols[i], mm = (double)m[i];
        flops_basis += (nc >= mm) ? 2.0 * nc * mm * mm - 2.0 / 3.0 * mm * mm * mm
                                  : 2.0 * mm * nc * nc - 2.0 / 3.0 * nc * nc * nc;
      }
      batched_qr_R(st, leaf);
      std::vector<DBuf> rounds;
      for (;;) {
        int64_t words = 0;
        bool more = false;
        for (auto& v : cur)
          for (size_t q = 0; q + 1 < v.size(); q += 2) {
            words += (int64_t)(v[q].r + v[q + 1].r) * m[i0 + (&v - &cur[0])];
            more = true;
          }
        if (!more) break;
        DBuf buf(std::max<int64_t>(words, 1) * sizeof(double));
        double* bp = buf.as<double>();
        int64_t off = 0;
        CopyBatch cb;
        std::vector<CopyItem> zl;
        std::vector<TallQr> qs;
        for (size_t bi = 0; bi < cur.size(); ++bi) {
          auto& v = cur[bi];
          const int mi = m[i0 + (int)bi];
          std::vector<Rref> nxt;
          for (size_t q = 0; q < v.size(); q += 2) {
            if (q + 1 == v.size()) {
              nxt.push_back(v[q]);
              continue;
            }
            const Rref& ra = v[q];
            const Rref& rb = v[q + 1];
            const int hs = ra.r + rb.r;
            double* S = bp + off;
            off += (int64_t)hs * mi;
            cb.add(ra.p, ra.ld, S, hs, ra.r, mi);
            cb.add(rb.p, rb.ld, S + ra.r, hs, rb.r, mi);
            zl.push_back(CopyItem{nullptr, S, 0, hs, ra.r, mi, 0, 0});
            zl.push_back(CopyItem{nullptr, S + ra.r, 0, hs, rb.r, mi, 0, 0});
            qs.push_back(TallQr{S, hs, hs, mi});
            nxt.push_back(Rref{S, hs, std::min(hs, mi)});
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
        for (size_t bi = 0; bi < cur.size(); ++bi) {
          if (cur[bi].empty()) continue;
          const int i = i0 + (int)bi;
          const Rref& r = cur[bi][0];
          double* PQi = PQ.as<double>() + offSq[i];
          cb.add(r.p, r.ld, PQi, m[i], r.r, m[i]);
          zl.push_back(CopyItem{nullptr, PQi, 0, m[i], r.r, m[i], 0, 0});
        }
        cb.run(st);
        int nz = (int)zl.size();
        CopyItem* dz = st.up(std::move(zl));
        launch_zero_lower(dz, nz, s);
        H2ULV_HIP(hipGetLastError());
      }
      tick("c_tsqr");
      st.sync();
      i0 = i1;
    }
  }
  // column-pivoted QR of each m x m triangle: small boxes one workgroup each,
  // large boxes over many workgroups, one step per pair of launches
  std::vector<int> capeff(nb, 0);
  for (int i = 0; i < nb; ++i) {
    capeff[i] = (int)std::min<int64_t>(m[i], ncols[i]);
    if (F.p.rank_cap > 0) capeff[i] = std::min(capeff[i], F.p.rank_cap);
  }
  const int BIG = 512;
  DBuf Ebuf;
  std::vector<int64_t> offE(nb + 1, 0);
  {
    std::vector<PivQrItem> pq;
    std::vector<PivQrState> big;
    std::vector<int> bigid;
    double* nrm = st.scratch<double>(std::max<int64_t>(cand_off[nb], 1));
    double* dg = st.scratch<double>(std::max<int64_t>(cand_off[nb], 1));
    double* scal = st.scratch<double>(2 * (size_t)nb + 2);
    int32_t* flg = st.scratch<int32_t>(2 * (size_t)nb + 2);
    for (int i = 0; i < nb; ++i) {
      if (m[i] == 0) continue;
      double* PQi = PQ.as<double>() + offSq[i];
      if (m[i] <= BIG) {
        PivQrItem it{};
        it.A = PQi;
        it.lda = m[i];
        it.m = m[i];
        it.n = m[i];
        it.piv = pivd.as<int32_t>() + cand_off[i];
        it.kout = kd.as<int32_t>() + i;
        it.diag = dg + cand_off[i];
        it.work = nrm + cand_off[i];
        it.tol = F.p.tol;
        it.cap = std::max(capeff[i], 0);
        pq.push_back(it);
      } else {
        PivQrState ps{};
        ps.A = PQi;
        ps.lda = m[i];
        ps.m = m[i];
        ps.cap = capeff[i];
        ps.nrm = nrm + cand_off[i];
        ps.piv = pivd.as<int32_t>() + cand_off[i];
        ps.scal = scal + 2 * i;
        ps.flags = flg + 2 * i;
        ps.tol = F.p.tol;
        big.push_back(ps);
        bigid.push_back(i);
      }
    }
    int npq = (int)pq.size();
    PivQrItem* dpq = st.up(std::move(pq));
    {
      ProfScope ps("pivqr_small", 0, 0, s);
      launch_pivqr(dpq, npq, s);
    }
    H2ULV_HIP(hipGetLastError());
    if (!big.empty()) {
      int nbig = (int)big.size();
      int maxcap = 0;
      std::vector<int64_t> sp(1, 0);
      for (auto& b : big) {
        sp.push_back(sp.back() + (b.m + 3) / 4);
        maxcap = std::max(maxcap, b.cap);
      }
      int64_t ns = sp.back();
      PivQrState* dst_ = st.up(std::move(big));
      int64_t* dsp = st.up(std::move(sp));
      {
        ProfScope ps("pivqr_large", 0, 0, s);
        launch_pivqr_init(dst_, dsp, ns, nbig, s);
        for (int t = 0; t < maxcap; ++t) {
          launch_pivqr_pick(dst_, nbig, t, s);
          launch_pivqr_apply(dst_, dsp, ns, nbig, t, s);
        }
      }
      H2ULV_HIP(hipGetLastError());
      std::vector<int32_t> hf(2 * (size_t)nb + 2);
      H2ULV_HIP(hipMemcpyAsync(hf.data(), flg, hf.size() * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
      H2ULV_HIP(hipStreamSynchronize(s));
      // E = R11^-1 R12 by triangular blocks
      for (int i : bigid) lf.k[i] = hf[2 * i + 1];
      for (int i = 0; i < nb; ++i) {
        bool isbig = m[i] > BIG;
        offE[i + 1] = offE[i] + (isbig ? (int64_t)lf.k[i] * (m[i] - lf.k[i]) : 0);
      }
      Ebuf.alloc(std::max<int64_t>(offE[nb], 1) * sizeof(double));
      std::vector<TriRhs> sys;
      for (int i : bigid) {
        int ki = lf.k[i];
        if (ki == 0 || ki == m[i]) continue;
        double* PQi = PQ.as<double>() + offSq[i];
        sys.push_back(TriRhs{PQi, m[i], ki, PQi + (int64_t)ki * m[i], m[i],
                             Ebuf.as<double>() + offE[i], ki, m[i] - ki});
      }
      trsm_upper(st, sys);
      std::vector<int32_t> hk(2);
      for (int i : bigid) {
        hk[0] = lf.k[i];
        H2ULV_HIP(hipMemcpyAsync(kd.as<int32_t>() + i, hk.data(), sizeof(int32_t),
                                 hipMemcpyHostToDevice, s));
        H2ULV_HIP(hipStreamSynchronize(s));
      }
    }
    tick("c_pivqr");
    st.sync();
  }
  Z.reset();
  check_dup();
  // ranks and pivots to the host
  {
    std::vector<int32_t> hk(nb), hp(cand_off[nb]);
    H2ULV_HIP(hipMemcpyAsync(hk.data(), kd.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (cand_off[nb] > 0)
      H2ULV_HIP(hipMemcpyAsync(hp.data(), pivd.p, cand_off[nb] * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    H2ULV_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nb; ++i) {
      lf.k[i] = (m[i] == 0) ? 0 : hk[i];
      piv[i].assign(hp.begin() + cand_off[i], hp.begin() + cand_off[i + 1]);
      lf.sk[i].resize(lf.k[i]);
      for (int t = 0; t < lf.k[i]; ++t) lf.sk[i][t] = lf.cand[i][piv[i][t]];
    }
  }
  std::vector<int>& k = lf.k;
  // W', W = T-hat W', QR -> U, T
  lf.offU.assign(nb + 1, 0);
  lf.offT.assign(nb + 1, 0);
  std::vector<int64_t> offW(nb + 1, 0);
  for (int i = 0; i < nb; ++i) {
    lf.offU[i + 1] = lf.offU[i] + (int64_t)m[i] * m[i];
    lf.offT[i + 1] = lf.offT[i] + (int64_t)k[i] * k[i];
    offW[i + 1] = offW[i] + (int64_t)m[i] * k[i];
  }
  lf.U.alloc(std::max<int64_t>(lf.offU[nb], 1) * sizeof(double));
  lf.Tt.alloc(std::max<int64_t>(lf.offT[nb], 1) * sizeof(double));
  {
    DBuf Wp(std::max<int64_t>(offW[nb], 1) * sizeof(double));
    DBuf W(std::max<int64_t>(offW[nb], 1) * sizeof(double));
    std::vector<WpItem> wi;
    for (int i = 0; i < nb; ++i) {
      if (k[i] == 0) continue;
      const bool isbig = m[i] > BIG;
      const double* E = isbig ? Ebuf.as<double>() + offE[i]
                              : PQ.as<double>() + offSq[i] + (int64_t)k[i] * m[i];
      wi.push_back(WpItem{pivd.as<int32_t>() + cand_off[i], E,
                          (upper ? Wp.as<double>() : W.as<double>()) + offW[i],
                          isbig ? std::max(k[i], 1) : m[i], m[i], m[i], k[i]});
    }
    int nw = (int)wi.size();
    WpItem* dwi = st.up(std::move(wi));
    launch_wprime(dwi, nw, s);
    H2ULV_HIP(hipGetLastError());
    if (upper) {
      const LevelFactor& ch = F.levels[lev + 1];
      GemmBatch<double> g;
      for (int i = 0; i < nb; ++i) {
        if (k[i] == 0) continue;
        int k1 = ch.k[2 * i], k2 = ch.k[2 * i + 1];
        double* Wi = W.as<double>() + offW[i];
        const double* Wpi = Wp.as<double>() + offW[i];
        if (k1 > 0)
          g.one(Wi, m[i], k1, k[i], k1, ch.Tt.as<double>() + ch.offT[2 * i], k1, false, Wpi, m[i],
                false);
        if (k2 > 0)
          g.one(Wi + k1, m[i], k2, k[i], k2, ch.Tt.as<double>() + ch.offT[2 * i + 1], k2, false,
                Wpi + k1, m[i], false);
      }
      g.run(st);
    }
    std::vector<QrW> qs;
    for (int i = 0; i < nb; ++i) {
      if (m[i] == 0) continue;
      qs.push_back(QrW{W.as<double>() + offW[i], m[i], k[i], lf.U.as<double>() + lf.offU[i],
                       lf.Tt.as<double>() + lf.offT[i]});
      flops_basis += 4.0 * m[i] * (double)k[i] * k[i] + 4.0 * (double)m[i] * m[i] * k[i];
    }
    batched_qr_basis(st, qs);
    st.sync();
  }
  PQ.reset();
  pivd.reset();
  Ebuf.reset();
  tick("c_basis_qr");

  // new skeleton blocks of this level: near pairs then far pairs
  shat_near_off.assign(nnear + 1, 0);
  shat_far_off.assign(nfar + 1, 0);
  int64_t tot = 0;
  for (int i = 0; i < nb; ++i)
    for (int64_t e = np[i]; e < np[i + 1]; ++e) {
      shat_near_off[e] = tot;
      tot += (int64_t)k[i] * k[ni[e]];
    }
  for (int i = 0; i < nb; ++i)
    for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
      shat_far_off[e] = tot;
      tot += (int64_t)k[i] * k[fi[e]];
    }
  Shat.alloc(std::max<int64_t>(tot, 1) * sizeof(double));
  double* Sh = Shat.as<double>();
  shat_lev = lev;

  // ---- (d) low-rank couplings --------------------------------------------
  {
    std::vector<int64_t> skoff(nb + 1, 0);
    std::vector<int64_t> skall;
    for (int i = 0; i < nb; ++i) {
      skoff[i + 1] = skoff[i] + k[i];
      skall.insert(skall.end(), lf.sk[i].begin(), lf.sk[i].end());
    }
    const int64_t* dsk = st.up(std::move(skall));
    std::vector<int64_t> kcoff(nfar + 1, 0);
    for (int i = 0; i < nb; ++i)
      for (int64_t e = fp[i]; e < fp[i + 1]; ++e) kcoff[e + 1] = kcoff[e] + (int64_t)k[i] * k[fi[e]];
    double* Kc = st.scratch<double>(std::max<int64_t>(kcoff[nfar], 1));
    double* Tmp = st.scratch<double>(std::max<int64_t>(kcoff[nfar], 1));
    KgenBatch kb;
    for (int i = 0; i < nb; ++i)
      for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
        int j = fi[e];
        if (k[i] == 0 || k[j] == 0) continue;
        kb.add(dsk + skoff[i], k[i], dsk + skoff[j], k[j], Kc + kcoff[e], k[i]);
        kevals += (double)k[i] * k[j];
        flops_couple += 2.0 * k[i] * (double)k[j] * k[j] + 2.0 * k[i] * (double)k[i] * k[j];
      }
    kb.run(st, F.pts.as<double>(), kf, dup);
    // tmp = Kc T_j^T ; S = T_i tmp
    if (!mixed) {
      GemmBatch<double> g1, g2;
      for (int i = 0; i < nb; ++i)
        for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
          int j = fi[e];
          if (k[i] == 0 || k[j] == 0) continue;
          g1.one(Tmp + kcoff[e], k[i], k[i], k[j], k[j], Kc + kcoff[e], k[i], false,
                 lf.Tt.as<double>() + lf.offT[j], k[j], true);
          g2.one(Sh + shat_far_off[e], k[i], k[i], k[j], k[i], lf.Tt.as<double>() + lf.offT[i],
                 k[i], false, Tmp + kcoff[e], k[i], false);
        }
      g1.run(st);
      g2.run(st);
    } else {
      DBuf Kc32 = to_f32(Kc, kcoff[nfar], s);
      DBuf T32 = to_f32(lf.Tt.as<double>(), lf.offT[nb], s);
      DBuf Tmp32(std::max<int64_t>(kcoff[nfar], 1) * sizeof(float));
      const float* Tf = T32.as<float>();
      GemmBatch<float> g1;
      GemmBatch<float, double> g2;
      for (int i = 0; i < nb; ++i)
        for (int64_t e = fp[i]; e < fp[i + 1]; ++e) {
          int j = fi[e];
          if (k[i] == 0 || k[j] == 0) continue;
          g1.one(Tmp32.as<float>() + kcoff[e], k[i], k[i], k[j], k[j],
                 Kc32.as<float>() + kcoff[e], k[i], false, Tf + lf.offT[j], k[j], true);
          g2.one(Sh + shat_far_off[e], k[i], k[i], k[j], k[i], Tf + lf.offT[i], k[i], false,
                 Tmp32.as<float>() + kcoff[e], k[i], false);
        }
      g1.run(st);
      g2.run(st);
      st.sync();
    }
    st.sync();
  }

  tick("d_couple");
  // ---- (e) rotation and (f) elimination ------------------------------------
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
  DBuf U32;
  {
    // off-diagonal near blocks: S_ij = U^S_i^T D_ij U^S_j
    std::vector<int64_t> toff(nnear + 1, 0);
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) toff[e + 1] = toff[e] + (int64_t)m[i] * k[ni[e]];
    if (mixed) U32 = to_f32(lf.U.as<double>(), lf.offU[nb], s);
    for (int i = 0; i < nb; ++i)
      for (int64_t e = np[i]; e < np[i + 1]; ++e) {
        int j = ni[e];
        if (j == i || k[i] == 0 || k[j] == 0) continue;
        flops_rotate += 2.0 * m[i] * (double)m[j] * k[j] + 2.0 * k[i] * (double)m[i] * k[j];
      }
    if (!mixed) {
      double* Tmp = st.scratch<double>(std::max<int64_t>(toff[nnear], 1));
      GemmBatch<double> g1, g2;
      const double* U = lf.U.as<double>();
      for (int i = 0; i < nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e) {
          int j = ni[e];
          if (j == i || k[i] == 0 || k[j] == 0) continue;
          g1.one(Tmp + toff[e], m[i], m[i], k[j], m[j], Dp + Doff[e], m[i], false, U + lf.offU[j],
                 m[j], false);
          g2.one(Sh + shat_near_off[e], k[i], k[i], k[j], m[i], U + lf.offU[i], m[i], true,
                 Tmp + toff[e], m[i], false);
        }
      g1.run(st);
      g2.run(st);
    } else {
      float* Tmp = st.scratch<float>(std::max<int64_t>(toff[nnear], 1));
      GemmBatch<float> g1;
      GemmBatch<float, double> g2;
      const float* U = U32.as<float>();
      const float* D32p = D32.as<float>();
      for (int i = 0; i < nb; ++i)
        for (int64_t e = np[i]; e < np[i + 1]; ++e) {
          int j = ni[e];
          if (j == i || k[i] == 0 || k[j] == 0) continue;
          g1.one(Tmp + toff[e], m[i], m[i], k[j], m[j], D32p + Doff[e], m[i], false,
                 U + lf.offU[j], m[j], false);
          g2.one(Sh + shat_near_off[e], k[i], k[i], k[j], m[i], U + lf.offU[i], m[i], true,
                 Tmp + toff[e], m[i], false);
        }
      g1.run(st);
      g2.run(st);
    }
    st.sync();
  }
  {
    // diagonal: S_ii = U_i^T D_ii U_i
    DBuf S(std::max<int64_t>(offSq[nb], 1) * sizeof(double));
    for (int i = 0; i < nb; ++i)
      if (m[i] > 0) flops_rotate += 4.0 * std::pow((double)m[i], 3);
    if (!mixed) {
      DBuf Tmp(std::max<int64_t>(offSq[nb], 1) * sizeof(double));
      GemmBatch<double> g1, g2;
      const double* U = lf.U.as<double>();
      for (int i = 0; i < nb; ++i) {
        if (m[i] == 0) continue;
        g1.one(Tmp.as<double>() + offSq[i], m[i], m[i], m[i], m[i], Dblk(i, i), m[i], false,
               U + lf.offU[i], m[i], false);
        g2.one(S.as<double>() + offSq[i], m[i], m[i], m[i], m[i], U + lf.offU[i], m[i], true,
               Tmp.as<double>() + offSq[i], m[i], false);
      }
      g1.run(st);
      g2.run(st);
      st.sync();
    } else {
      DBuf Tmp(std::max<int64_t>(offSq[nb], 1) * sizeof(float));
      GemmBatch<float> g1;
      GemmBatch<float, double> g2;
      const float* U = U32.as<float>();
      const float* D32p = D32.as<float>();
      for (int i = 0; i < nb; ++i) {
        if (m[i] == 0) continue;
        int64_t e = csr_find(np, ni, i, i);
        g1.one(Tmp.as<float>() + offSq[i], m[i], m[i], m[i], m[i], D32p + Doff[e], m[i], false,
               U + lf.offU[i], m[i], false);
        g2.one(S.as<double>() + offSq[i], m[i], m[i], m[i], m[i], U + lf.offU[i], m[i], true,
               Tmp.as<float>() + offSq[i], m[i], false);
      }
      g1.run(st);
      g2.run(st);
      st.sync();
    }
    D.reset();
    D32.reset();
    U32.reset();
    tick("e_rotate");
    // S^RR inverse, X = S^RR^-1 S^RS, S^SR copy, Schur update into the new diagonal block
    DBuf RRw(std::max<int64_t>(lf.offR[nb], 1) * sizeof(double));
    CopyBatch cb, cs, css;
    std::vector<SqMat> mats;
    std::vector<int> who;
    for (int i = 0; i < nb; ++i) {
      int r = m[i] - k[i], ki = k[i];
      const double* Si = S.as<double>() + offSq[i];
      if (r > 0) {
        cb.add(Si + ki + (int64_t)ki * m[i], m[i], RRw.as<double>() + lf.offR[i], r, r, r);
        mats.push_back(SqMat{RRw.as<double>() + lf.offR[i], r, r,
                             lf.Sinv.as<double>() + lf.offR[i], r});
        who.push_back(i);
        if (ki > 0)
          cs.add(Si + (int64_t)ki * m[i], m[i], lf.SSR.as<double>() + lf.offX[i], ki, ki, r);
        flops_elim += 2.0 / 3.0 * r * (double)r * r + 2.0 * ki * (double)r * r +
                      2.0 * ki * (double)ki * r;
      }
      if (ki > 0) {
        int64_t e = csr_find(np, ni, i, i);
        css.add(Si, m[i], Sh + shat_near_off[e], ki, ki, ki);
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
      for (double v : hl) F.stats.logabsdet += v;
    }
    GemmBatch<double> g1, g2;
    for (int i = 0; i < nb; ++i) {
      int r = m[i] - k[i], ki = k[i];
      if (r == 0 || ki == 0) continue;
      const double* Si = S.as<double>() + offSq[i];
      g1.one(lf.Xs.as<double>() + lf.offX[i], r, r, ki, r, lf.Sinv.as<double>() + lf.offR[i], r,
             false, Si + ki, m[i], false);
    }
    g1.run(st);
    if (!mixed) {
      for (int i = 0; i < nb; ++i) {
        int r = m[i] - k[i], ki = k[i];
        if (r == 0 || ki == 0) continue;
        int64_t e = csr_find(np, ni, i, i);
        g2.one(Sh + shat_near_off[e], ki, ki, ki, r, lf.SSR.as<double>() + lf.offX[i], ki, false,
               lf.Xs.as<double>() + lf.offX[i], r, false, -1.0, 1.0);
      }
      g2.run(st);
    } else {
      DBuf SSR32 = to_f32(lf.SSR.as<double>(), lf.offX[nb], s);
      DBuf X32 = to_f32(lf.Xs.as<double>(), lf.offX[nb], s);
      GemmBatch<float, double> g3;
      for (int i = 0; i < nb; ++i) {
        int r = m[i] - k[i], ki = k[i];
        if (r == 0 || ki == 0) continue;
        int64_t e = csr_find(np, ni, i, i);
        g3.one(Sh + shat_near_off[e], ki, ki, ki, r, SSR32.as<float>() + lf.offX[i], ki, false,
               X32.as<float>() + lf.offX[i], r, false, -1.0, 1.0);
      }
      g3.run(st);
      st.sync();
    }
    st.sync();
  }
  tick("f_elim");
  // next level's candidate rows
  if (lev > 1) {
    LevelFactor& pa = F.levels[lev - 1];
    pa.cand.assign(nb / 2, {});
    for (int p = 0; p < nb / 2; ++p) {
      pa.cand[p] = lf.sk[2 * p];
      pa.cand[p].insert(pa.cand[p].end(), lf.sk[2 * p + 1].begin(), lf.sk[2 * p + 1].end());
    }
  }
}

void Factorizer::root() {
  Stage st(s);
  const int L = F.tree.L;
  int m0;
  DBuf D0;
  if (L == 0) {
    m0 = (int)F.n;
    D0.alloc((size_t)m0 * m0 * sizeof(double));
    KgenBatch kb;
    std::vector<int64_t> pv(F.tree.perm);
    const int64_t* dp = st.up(std::move(pv));
    kb.add(dp, m0, dp, m0, D0.as<double>(), m0);
    kevals += (double)m0 * m0;
    kb.run(st, F.pts.as<double>(), kf, dup);
    st.sync();
    check_dup();
  } else {
    const std::vector<int>& k = F.levels[1].k;
    m0 = k[0] + k[1];
    D0.alloc(std::max<size_t>((size_t)m0 * m0, 1) * sizeof(double));
    CopyBatch cb;
    int ro = 0;
    for (int a = 0; a < 2; ++a) {
      int co = 0;
      for (int b = 0; b < 2; ++b) {
        int64_t ld;
        const double* src = shat_block(1, a, b, &ld);
        cb.add(src, std::max<int64_t>(ld, 1), D0.as<double>() + ro + (int64_t)co * m0, m0, k[a],
               k[b]);
        co += k[b];
      }
      ro += k[a];
    }
    cb.run(st);
    st.sync();
    Shat.reset();
  }
  F.m_root = m0;
  F.root_inv.alloc(std::max<size_t>((size_t)m0 * m0, 1) * sizeof(double));
  if (m0 > 0) {
    std::vector<SqMat> mats{SqMat{D0.as<double>(), m0, m0, F.root_inv.as<double>(), m0}};
    int32_t* info = nullptr;
    batched_inverse(st, mats, &info, nullptr, nullptr);
    std::vector<MatDesc> ds(1);
    ds[0].A = D0.as<double>();
    ds[0].lda = m0;
    ds[0].m = m0;
    double* ld = st.scratch<double>(1);
    MatDesc* dd = st.up(std::move(ds));
    launch_logdet(dd, 1, ld, s);
    double hl = 0;
    H2ULV_HIP(hipMemcpyAsync(&hl, ld, sizeof(double), hipMemcpyDeviceToHost, s));
    check_info(info, 1, s, "the root block");
    F.stats.logabsdet += hl;
    flops_root += 2.0 / 3.0 * std::pow((double)m0, 3);
  }
  st.sync();
}

// ---------------------------------------------------------------------------
// solve: forward sweep over levels, root, backward sweep (Sec. II-B)
// ---------------------------------------------------------------------------
static void solve_impl(const h2ulv_factor& F, double* b, int nrhs, int64_t ldb, hipStream_t s) {
  Stage st(s);
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
    g.run(st);
    launch_permute_rows(x, n, b, ldb, F.perm.as<int64_t>(), n, nrhs, 1, s);
    st.sync();
    return;
  }
  // per-level RHS blocks: rhs[lev] holds m_i x nrhs per box (ld m_i); the leaf
  // level reads bt directly.
  std::vector<std::vector<int64_t>> moff(L + 1), woff(L + 1);
  std::vector<double*> rhs(L + 1, nullptr), cbuf(L + 1, nullptr), wbuf(L + 1, nullptr),
      xbuf(L + 1, nullptr);
  for (int lev = 1; lev <= L; ++lev) {
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
  for (int lev = L; lev >= 1; --lev) {
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
    g1.run(st);
    g2.run(st);
    g3.run(st);
    // gather c^S of both children into the parent's rhs
    CopyBatch cb;
    if (lev > 1) {
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
  // root
  const LevelFactor& l1 = F.levels[1];
  int m0 = F.m_root, k1 = l1.k[0];
  double* b0 = st.scratch<double>(std::max<int64_t>((int64_t)m0 * nrhs, 1));
  double* x0 = st.scratch<double>(std::max<int64_t>((int64_t)m0 * nrhs, 1));
  {
    CopyBatch cb;
    cb.add(cbuf[1] + moff[1][0], l1.m[0], b0, m0, k1, nrhs);
    cb.add(cbuf[1] + moff[1][1], l1.m[1], b0 + k1, m0, l1.k[1], nrhs);
    cb.run(st);
    GemmBatch<double> g;
    g.one(x0, m0, m0, nrhs, m0, F.root_inv.as<double>(), m0, false, b0, m0, false);
    g.run(st);
  }
  // backward
  for (int lev = 1; lev <= L; ++lev) {
    const LevelFactor& lf = F.levels[lev];
    GemmBatch<double> g1, g2;
    for (int i = 0; i < lf.nb; ++i) {
      int mi = lf.m[i], ki = lf.k[i], r = mi - ki;
      if (mi == 0) continue;
      // skeleton part of the solution from the parent
      const double* xs;
      int64_t ldxs;
      if (lev == 1) {
        xs = x0 + (i == 0 ? 0 : k1);
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
      if (ki > 0) g2.term(lf.U.as<double>() + lf.offU[i], mi, false, xs, ldxs, false, ki);
      if (r > 0)
        g2.term(lf.U.as<double>() + lf.offU[i] + (int64_t)ki * mi, mi, false, wi, r, false, r);
    }
    g1.run(st);
    g2.run(st);
  }
  launch_permute_rows(bt, n, b, ldb, F.perm.as<int64_t>(), n, nrhs, 1, s);
  H2ULV_HIP(hipGetLastError());
  st.sync();
}

static h2ulv_factor* factorize_impl(const double* pts, int64_t n, const h2ulv_params* params,
                                    hipStream_t s) {
  validate_params(params);
  if (!pts) fail(H2ULV_ERR_INVALID_ARG, "pts is NULL");
  if (n < 1) fail(H2ULV_ERR_INVALID_ARG, "n must be >= 1");
  if (n > ((int64_t)1 << 31) - 1) fail(H2ULV_ERR_INVALID_ARG, "n too large");
  double t0 = now_s();
  std::vector<double> hp(n * 3);
  H2ULV_HIP(hipMemcpyAsync(hp.data(), pts, n * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  for (double v : hp)
    if (!std::isfinite(v)) fail(H2ULV_ERR_INVALID_ARG, "non-finite point coordinate");
  auto F = std::make_unique<h2ulv_factor>();
  F->p = *params;
  F->n = n;
  F->tree = build_tree(hp.data(), n, params->leaf_size);
  F->lists = build_lists(F->tree, params->eta);
  double t1 = now_s();
  F->pts.alloc(n * 3 * sizeof(double));
  H2ULV_HIP(hipMemcpyAsync(F->pts.p, pts, n * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  F->perm.alloc(n * sizeof(int64_t));
  H2ULV_HIP(hipMemcpyAsync(F->perm.p, F->tree.perm.data(), n * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  mem_stats().peak = mem_stats().live;
  Factorizer fz(*F, s);
  fz.run();
  H2ULV_HIP(hipStreamSynchronize(s));
  double t2 = now_s();
  h2ulv_stats& st = F->stats;
  st.levels = F->tree.L;
  st.n = n;
  st.root_size = F->m_root;
  int mx = 0;
  for (auto& lf : F->levels)
    for (int x : lf.k) mx = std::max(mx, x);
  st.max_rank = mx;
  st.flops_fill = fz.flops_fill;
  st.flops_basis = fz.flops_basis;
  st.flops_couple = fz.flops_couple;
  st.flops_rotate = fz.flops_rotate;
  st.flops_elim = fz.flops_elim;
  st.flops_root = fz.flops_root;
  st.kernel_evals = fz.kevals;
  st.time_setup_s = t1 - t0;
  st.time_factor_s = t2 - t0;
  st.device_bytes = (double)mem_stats().peak;
  return F.release();
}

static void matvec_impl(const h2ulv_factor& F, const double* x, int64_t ldx, double* y,
                        int64_t ldy, int nrhs, hipStream_t s) {
  launch_matvec(F.pts.as<double>(), F.n, kfn(F.p), x, ldx, y, ldy, nrhs, s);
  H2ULV_HIP(hipGetLastError());
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
  solve_impl(F, x, nrhs, ldx, s);
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
    solve_impl(F, r.as<double>(), nrhs, n, s);
    launch_axpy_cols(x, ldx, r.as<double>(), n, n, nrhs, s);
    H2ULV_HIP(hipGetLastError());
  }
  g_last_error = "refinement did not reach the tolerance";
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
  return H2ULV_OK;
}

h2ulv_status h2ulv_factorize(const double* pts, int64_t n, const h2ulv_params* params,
                             void* stream, h2ulv_factor** out) {
  if (!out) {
    g_last_error = "out is NULL";
    return H2ULV_ERR_INVALID_ARG;
  }
  *out = nullptr;
  return guarded([&] { *out = factorize_impl(pts, n, params, (hipStream_t)stream); });
}

h2ulv_status h2ulv_factorize_batch(int32_t nprob, const double* const* pts, const int64_t* n,
                                   const h2ulv_params* params, void* stream,
                                   h2ulv_factor** out) {
  if (nprob < 1 || !pts || !n || !out) {
    g_last_error = "bad batch arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  for (int p = 0; p < nprob; ++p) out[p] = nullptr;
  h2ulv_status st = guarded([&] {
    for (int p = 0; p < nprob; ++p) out[p] = factorize_impl(pts[p], n[p], params, (hipStream_t)stream);
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
  return guarded([&] { solve_impl(*f, b, nrhs, ldb, (hipStream_t)stream); });
}

h2ulv_status h2ulv_matvec_exact(const h2ulv_factor* f, const double* x, int64_t ldx, double* y,
                                int64_t ldy, int32_t nrhs, void* stream) {
  if (!f || !x || !y || nrhs < 1 || ldx < f->n || ldy < f->n) {
    g_last_error = "bad matvec arguments";
    return H2ULV_ERR_INVALID_ARG;
  }
  return guarded([&] { matvec_impl(*f, x, ldx, y, ldy, nrhs, (hipStream_t)stream); });
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
    out = refine_impl(*f, b, ldb, x, ldx, nrhs, rtol, max_iter, iters, relres,
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

h2ulv_status h2ulv_get_ranks(const h2ulv_factor* f, int32_t lev, int32_t* m, int32_t* k) {
  if (!f || lev < 1 || lev > f->tree.L) {
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
  if (!f || !sk || lev < 1 || lev > f->tree.L || box < 0 || box >= (1 << lev)) {
    g_last_error = "bad level or box";
    return H2ULV_ERR_INVALID_ARG;
  }
  const auto& v = f->levels[lev].sk[box];
  std::copy(v.begin(), v.end(), sk);
  return H2ULV_OK;
}

h2ulv_status h2ulv_get_basis(const h2ulv_factor* f, int32_t lev, int32_t box, double* U) {
  if (!f || !U || lev < 1 || lev > f->tree.L || box < 0 || box >= (1 << lev)) {
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
    s->tree = build_tree(pts, n, params->leaf_size);
    s->lists = build_lists(s->tree, params->eta);
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

const char* h2ulv_status_string(h2ulv_status s) {
  switch (s) {
    case H2ULV_OK: return "ok";
    case H2ULV_ERR_INVALID_ARG: return "invalid argument";
    case H2ULV_ERR_OOM: return "out of memory";
    case H2ULV_ERR_HIP: return "HIP runtime error";
    case H2ULV_ERR_SINGULAR: return "singular block";
    case H2ULV_ERR_DUPLICATE_POINTS: return "duplicate points";
    case H2ULV_ERR_NOT_CONVERGED: return "refinement not converged";
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
  });
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
