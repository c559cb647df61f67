// Internal declarations of the H^2-ULV library (not part of the C-ABI).
#pragma once

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/h2ulv.h"

namespace h2ulv {

// Error carried from deep inside the library to the ABI boundary.
struct Error : std::runtime_error {
  h2ulv_status status;
  Error(h2ulv_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(h2ulv_status s, const std::string& m) { throw Error(s, m); }

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
Tree build_tree(const double* pts, int64_t n, int leaf);
Lists build_lists(const Tree& t, double eta);
void validate_params(const h2ulv_params* p);

}  // namespace h2ulv
