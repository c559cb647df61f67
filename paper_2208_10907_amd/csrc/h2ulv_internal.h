// Internal declarations of the H^2-ULV library (not part of the C-ABI).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/h2ulv.h"

namespace h2ulv {

// Error carried from deep inside the library to the ABI boundary.
struct Error : std::runtime_error {
  h2ulv_status status;
  Error(h2ulv_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(h2ulv_status s, const std::string& m) { throw Error(s, m); }

// fn(i) for i in [0, n) on up to 16 host threads (the calling thread takes
// part); iterations are handed out in blocks of `grain`.  fn must not throw.
template <class Fn>
void parallel_for(int64_t n, int64_t grain, Fn&& fn) {
  if (n <= 0) return;
  const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
  const int64_t nt = std::min<int64_t>({16, hw, (n + grain - 1) / grain});
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next(0);
  auto work = [&]() {
    for (;;) {
      const int64_t b = next.fetch_add(grain);
      if (b >= n) break;
      const int64_t e = std::min(n, b + grain);
      for (int64_t i = b; i < e; ++i) fn(i);
    }
  };
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int64_t t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------------------
// Cluster tree (binary k-d tree, Sec. III-D) and strong-admissibility lists.
// ---------------------------------------------------------------------------
struct Tree {
  int L = 0;
  int64_t n = 0;
  std::vector<int64_t> perm;                       // tree position -> point index
  std::vector<std::vector<int64_t>> start, end;    // [lev][box] position range
  std::vector<std::vector<double>> centre;         // [lev][3*box]
  std::vector<std::vector<double>> radius;         // [lev][box]
  int64_t box_size(int lev, int64_t i) const { return end[lev][i] - start[lev][i]; }
};

struct Lists {
  // CSR per level; rows sorted ascending
  std::vector<std::vector<int64_t>> near_ptr, far_ptr;
  std::vector<std::vector<int32_t>> near_idx, far_idx;
  bool is_near(int lev, int32_t i, int32_t j) const;
};

int tree_depth(int64_t n, int leaf);
Tree build_tree(const double* pts, int64_t n, int leaf, int partition);
Lists build_lists(const Tree& t, double eta);
// flat BLR^2 lists: the leaf level only (upper levels empty)
Lists build_flat_lists(const Tree& t, double eta);
// separate row and column bases (nonsymmetric kernel, or asked for)
bool separate_bases(const h2ulv_params& p);
// the lists of the structure params.structure selects
Lists build_structure_lists(const Tree& t, const h2ulv_params& p);
void validate_params(const h2ulv_params* p);

}  // namespace h2ulv
