// Host setup of the sweep: binary cluster tree and near/far block lists.
//
// The paper factorizes level by level over a full binary tree of boxes
// (Sec. III-D) and uses strong admissibility: a block is low-rank only when its
// two boxes are well separated, otherwise it is kept dense (Sec. I, II-D).
// The paper does not fix the partitioner or the admissibility formula; this
// library uses
//   * a k-d split along the widest bounding-box axis (lowest axis on ties),
//     points stably ordered by (coordinate, original index), left child gets
//     floor(n/2); depth L = smallest integer with leaf * 2^L >= N; or, for
//     point clouds on surfaces, a balanced 2-means bisection (Sec. V clusters
//     the boundary-element points with k-means, the cluster count a power of
//     two);
//   * box centre = bounding-box midpoint, radius = half its diagonal;
//   * (i, j) admissible iff |c_i - c_j| > eta (r_i + r_j), decided for the
//     children of every near pair of the parent level (root: near to itself).
// Geometry is computed with plain (non-contracted) double arithmetic.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "h2ulv_internal.h"

namespace h2ulv {

int tree_depth(int64_t n, int leaf) {
  int L = 0;
  while ((int64_t)leaf * ((int64_t)1 << L) < n) ++L;
  return L;
}

static void bbox(const double* pts, const int64_t* idx, int64_t cnt, double lo[3], double hi[3]) {
  for (int c = 0; c < 3; ++c) {
    lo[c] = pts[idx[0] * 3 + c];
    hi[c] = lo[c];
  }
  for (int64_t a = 1; a < cnt; ++a)
    for (int c = 0; c < 3; ++c) {
      double v = pts[idx[a] * 3 + c];
      if (v < lo[c]) lo[c] = v;
      if (v > hi[c]) hi[c] = v;
    }
}

// Balanced 2-means bisection of the points p[0..cnt) (reordered in place):
// start from the k-d split (order by coordinate of the widest axis, then index;
// the first floor(cnt/2) points form cluster 0), then up to 10 Lloyd steps:
// centroids as plain sums over each cluster's points in ascending index order
// divided by the count, every point keyed by |x - c0|^2 - |x - c1|^2, the
// floor(cnt/2) smallest keys (ties by index) form cluster 0; stop when
// cluster 0 no longer changes.  The final order is the last (key, index) order.
static void kmeans_split(const double* pts, int64_t* p, int64_t cnt, int axis) {
  const int64_t half = cnt / 2;
  std::vector<std::pair<double, int64_t>> key(cnt);
  for (int64_t u = 0; u < cnt; ++u) key[u] = {pts[p[u] * 3 + axis], p[u]};
  std::sort(key.begin(), key.end());
  std::vector<int64_t> c0(half), prev;
  for (int64_t u = 0; u < half; ++u) c0[u] = key[u].second;
  std::sort(c0.begin(), c0.end());
  for (int it = 0; it < 10; ++it) {
    std::vector<int64_t> c1;
    c1.reserve(cnt - half);
    for (int64_t u = half; u < cnt; ++u) c1.push_back(key[u].second);
    std::sort(c1.begin(), c1.end());
    double m0[3] = {0, 0, 0}, m1[3] = {0, 0, 0};
    for (int64_t q : c0)
      for (int c = 0; c < 3; ++c) m0[c] = m0[c] + pts[q * 3 + c];
    for (int64_t q : c1)
      for (int c = 0; c < 3; ++c) m1[c] = m1[c] + pts[q * 3 + c];
    for (int c = 0; c < 3; ++c) {
      m0[c] = m0[c] / (double)c0.size();
      m1[c] = m1[c] / (double)c1.size();
    }
    for (int64_t u = 0; u < cnt; ++u) {
      const int64_t q = key[u].second;
      double a0 = pts[q * 3] - m0[0], a1 = pts[q * 3 + 1] - m0[1], a2 = pts[q * 3 + 2] - m0[2];
      double b0 = pts[q * 3] - m1[0], b1 = pts[q * 3 + 1] - m1[1], b2 = pts[q * 3 + 2] - m1[2];
      double d0 = a0 * a0;
      d0 = d0 + a1 * a1;
      d0 = d0 + a2 * a2;
      double d1 = b0 * b0;
      d1 = d1 + b1 * b1;
      d1 = d1 + b2 * b2;
      key[u].first = d0 - d1;
    }
    std::sort(key.begin(), key.end());
    prev.swap(c0);
    c0.assign(half, 0);
    for (int64_t u = 0; u < half; ++u) c0[u] = key[u].second;
    std::sort(c0.begin(), c0.end());
    if (c0 == prev) break;
  }
  for (int64_t u = 0; u < cnt; ++u) p[u] = key[u].second;
}

Tree build_tree(const double* pts, int64_t n, int leaf, int partition) {
  Tree t;
  t.n = n;
  t.L = tree_depth(n, leaf);
  t.perm.resize(n);
  std::iota(t.perm.begin(), t.perm.end(), (int64_t)0);
  std::vector<std::pair<int64_t, int64_t>> ranges{{0, n}};
  for (int lev = 0; lev <= t.L; ++lev) {
    const size_t nb = ranges.size();
    t.start.emplace_back(nb);
    t.end.emplace_back(nb);
    t.centre.emplace_back(3 * nb);
    t.radius.emplace_back(nb);
    std::vector<std::pair<int64_t, int64_t>> next(lev < t.L ? 2 * nb : 0);
    // boxes of a level are independent; each split orders its range by
    // (coordinate, index) along the widest axis.  Only the last split's order
    // survives (every level re-orders the ranges of the previous one), so the
    // earlier splits only partition at the median.
    parallel_for((int64_t)nb, 1, [&](int64_t b) {
      const int64_t a0 = ranges[b].first, a1 = ranges[b].second;
      t.start[lev][b] = a0;
      t.end[lev][b] = a1;
      double lo[3], hi[3];
      bbox(pts, t.perm.data() + a0, a1 - a0, lo, hi);
      double d[3];
      for (int c = 0; c < 3; ++c) {
        t.centre[lev][3 * b + c] = 0.5 * (lo[c] + hi[c]);
        d[c] = hi[c] - lo[c];
      }
      double sq = d[0] * d[0];
      sq = sq + d[1] * d[1];
      sq = sq + d[2] * d[2];
      t.radius[lev][b] = 0.5 * std::sqrt(sq);
      if (lev < t.L) {
        int axis = 0;
        if (d[1] > d[axis]) axis = 1;
        if (d[2] > d[axis]) axis = 2;
        int64_t* p = t.perm.data() + a0;
        const int64_t cnt = a1 - a0;
        const int64_t half = cnt / 2;
        if (partition == 1 && cnt >= 2) {
          kmeans_split(pts, p, cnt, axis);
        } else {
          std::vector<std::pair<double, int64_t>> key(cnt);
          for (int64_t u = 0; u < cnt; ++u) key[u] = {pts[p[u] * 3 + axis], p[u]};
          if (lev + 1 == t.L)
            std::sort(key.begin(), key.end());
          else if (half > 0)
            std::nth_element(key.begin(), key.begin() + half, key.end());
          for (int64_t u = 0; u < cnt; ++u) p[u] = key[u].second;
        }
        next[2 * b] = {a0, a0 + half};
        next[2 * b + 1] = {a0 + half, a1};
      }
    });
    ranges.swap(next);
  }
  return t;
}

Lists build_lists(const Tree& t, double eta) {
  Lists ls;
  ls.near_ptr.push_back({0, 1});
  ls.near_idx.push_back({0});
  ls.far_ptr.push_back({0, 0});
  ls.far_idx.push_back({});
  for (int lev = 1; lev <= t.L; ++lev) {
    int64_t nb = (int64_t)1 << lev;
    std::vector<std::vector<int32_t>> nl(nb), fl(nb);
    const std::vector<double>& c = t.centre[lev];
    const std::vector<double>& r = t.radius[lev];
    const std::vector<int64_t>& pp = ls.near_ptr[lev - 1];
    const std::vector<int32_t>& pi = ls.near_idx[lev - 1];
    for (int64_t p = 0; p < nb / 2; ++p)
      for (int64_t e = pp[p]; e < pp[p + 1]; ++e) {
        int64_t q = pi[e];
        for (int64_t i = 2 * p; i < 2 * p + 2; ++i)
          for (int64_t j = 2 * q; j < 2 * q + 2; ++j) {
            double d0 = c[3 * i] - c[3 * j], d1 = c[3 * i + 1] - c[3 * j + 1],
                   d2 = c[3 * i + 2] - c[3 * j + 2];
            double s = d0 * d0;
            s = s + d1 * d1;
            s = s + d2 * d2;
            double dist = std::sqrt(s);
            if (dist > eta * (r[i] + r[j]))
              fl[i].push_back((int32_t)j);
            else
              nl[i].push_back((int32_t)j);
          }
      }
    std::vector<int64_t> np(nb + 1, 0), fp(nb + 1, 0);
    std::vector<int32_t> ni, fi;
    for (int64_t i = 0; i < nb; ++i) {
      std::sort(nl[i].begin(), nl[i].end());
      std::sort(fl[i].begin(), fl[i].end());
      ni.insert(ni.end(), nl[i].begin(), nl[i].end());
      fi.insert(fi.end(), fl[i].begin(), fl[i].end());
      np[i + 1] = (int64_t)ni.size();
      fp[i + 1] = (int64_t)fi.size();
    }
    ls.near_ptr.push_back(std::move(np));
    ls.near_idx.push_back(std::move(ni));
    ls.far_ptr.push_back(std::move(fp));
    ls.far_idx.push_back(std::move(fi));
  }
  return ls;
}

bool separate_bases(const h2ulv_params& p) { return p.bases == 1 || p.kernel == H2ULV_ADVECTION; }

Lists build_flat_lists(const Tree& t, double eta) {
  // one level of boxes, the leaves, every pair classified directly (no
  // hierarchy); the levels above hold empty lists, the root level its box
  Lists ls;
  ls.near_ptr.push_back({0, 1});
  ls.near_idx.push_back({0});
  ls.far_ptr.push_back({0, 0});
  ls.far_idx.push_back({});
  for (int lev = 1; lev < t.L; ++lev) {
    ls.near_ptr.emplace_back(((size_t)1 << lev) + 1, 0);
    ls.near_idx.emplace_back();
    ls.far_ptr.emplace_back(((size_t)1 << lev) + 1, 0);
    ls.far_idx.emplace_back();
  }
  if (t.L == 0) return ls;
  const int64_t nb = (int64_t)1 << t.L;
  const std::vector<double>& c = t.centre[t.L];
  const std::vector<double>& r = t.radius[t.L];
  std::vector<std::vector<int32_t>> nl(nb), fl(nb);
  parallel_for(nb, 16, [&](int64_t i) {
    for (int64_t j = 0; j < nb; ++j) {
      double d0 = c[3 * i] - c[3 * j], d1 = c[3 * i + 1] - c[3 * j + 1],
             d2 = c[3 * i + 2] - c[3 * j + 2];
      double s = d0 * d0;
      s = s + d1 * d1;
      s = s + d2 * d2;
      if (std::sqrt(s) > eta * (r[i] + r[j]))
        fl[i].push_back((int32_t)j);
      else
        nl[i].push_back((int32_t)j);
    }
  });
  std::vector<int64_t> np(nb + 1, 0), fp(nb + 1, 0);
  std::vector<int32_t> ni, fi;
  for (int64_t i = 0; i < nb; ++i) {
    ni.insert(ni.end(), nl[i].begin(), nl[i].end());
    fi.insert(fi.end(), fl[i].begin(), fl[i].end());
    np[i + 1] = (int64_t)ni.size();
    fp[i + 1] = (int64_t)fi.size();
  }
  ls.near_ptr.push_back(std::move(np));
  ls.near_idx.push_back(std::move(ni));
  ls.far_ptr.push_back(std::move(fp));
  ls.far_idx.push_back(std::move(fi));
  return ls;
}

Lists build_structure_lists(const Tree& t, const h2ulv_params& p) {
  return p.structure == 1 ? build_flat_lists(t, p.eta) : build_lists(t, p.eta);
}

bool Lists::is_near(int lev, int32_t i, int32_t j) const {
  const int32_t* b = near_idx[lev].data() + near_ptr[lev][i];
  const int32_t* e = near_idx[lev].data() + near_ptr[lev][i + 1];
  return std::binary_search(b, e, j);
}

void validate_params(const h2ulv_params* p) {
  if (!p) fail(H2ULV_ERR_INVALID_ARG, "params is NULL");
  if (p->struct_size != (int32_t)sizeof(h2ulv_params))
    fail(H2ULV_ERR_INVALID_ARG, "params.struct_size mismatch (use h2ulv_params_default)");
  if (p->kernel != H2ULV_LAPLACE && p->kernel != H2ULV_YUKAWA && p->kernel != H2ULV_ADVECTION)
    fail(H2ULV_ERR_INVALID_ARG, "unknown kernel");
  if (p->kernel == H2ULV_ADVECTION) {
    // decay in every direction: b.(x - y) <= |b| r <= alpha r
    for (double v : p->drift)
      if (!std::isfinite(v)) fail(H2ULV_ERR_INVALID_ARG, "drift must be finite");
    double b2 = p->drift[0] * p->drift[0];
    b2 = b2 + p->drift[1] * p->drift[1];
    b2 = b2 + p->drift[2] * p->drift[2];
    if (!(std::sqrt(b2) <= p->alpha))
      fail(H2ULV_ERR_INVALID_ARG, "the advection kernel needs alpha >= |drift|");
  }
  if (p->sketch_fallback != 0 && p->sketch_fallback != 1)
    fail(H2ULV_ERR_INVALID_ARG, "sketch_fallback must be 0 or 1");
  if (p->sketch_min_level < 0)
    fail(H2ULV_ERR_INVALID_ARG, "sketch_min_level must be >= 0");
  if (p->bases != 0 && p->bases != 1)
    fail(H2ULV_ERR_INVALID_ARG, "bases must be 0 (by kernel) or 1 (separate)");
  if (separate_bases(*p) &&
      (p->structure != 0 || p->precision != H2ULV_FP64 || p->rank_model))
    fail(H2ULV_ERR_INVALID_ARG,
         "separate row and column bases need structure 0, precision FP64 and no rank model");
  if (!std::isfinite(p->alpha) || !std::isfinite(p->diag))
    fail(H2ULV_ERR_INVALID_ARG, "alpha and diag must be finite");
  if (!(p->eta >= 0) || !std::isfinite(p->eta)) fail(H2ULV_ERR_INVALID_ARG, "eta must be >= 0");
  if (p->leaf_size < 2) fail(H2ULV_ERR_INVALID_ARG, "leaf_size must be >= 2");
  if (p->rank_cap < 0) fail(H2ULV_ERR_INVALID_ARG, "rank_cap must be >= 0");
  if (!(p->tol >= 0) || !std::isfinite(p->tol)) fail(H2ULV_ERR_INVALID_ARG, "tol must be >= 0");
  if (p->far_sample < 0) fail(H2ULV_ERR_INVALID_ARG, "far_sample must be >= 0");
  if (p->precision != H2ULV_FP64 && p->precision != H2ULV_MIXED)
    fail(H2ULV_ERR_INVALID_ARG, "unknown precision");
  if (p->oversample < 0) fail(H2ULV_ERR_INVALID_ARG, "oversample must be >= 0");
  if (p->fill_in != 0 && p->fill_in != 1) fail(H2ULV_ERR_INVALID_ARG, "fill_in must be 0 or 1");
  if (p->partition != 0 && p->partition != 1)
    fail(H2ULV_ERR_INVALID_ARG, "partition must be 0 (k-d) or 1 (k-means)");
  if (p->structure != 0 && p->structure != 1)
    fail(H2ULV_ERR_INVALID_ARG, "structure must be 0 (H^2) or 1 (flat BLR^2)");
  if (p->fill_in == 0 && p->rank_model)
    fail(H2ULV_ERR_INVALID_ARG, "fill_in = 0 must not be combined with a rank model");
}

}  // namespace h2ulv
