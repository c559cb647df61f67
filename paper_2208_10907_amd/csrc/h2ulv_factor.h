// Factor storage and the batched level driver (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "h2ulv_dense.h"

namespace h2ulv {

struct SolveGraph;  // a solve recorded in a HIP graph (h2ulv_api.cpp)

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
  // learned ranks: features (nb x 16), predicted rank, sketch columns, outcome
  std::vector<float> feat;
  std::vector<int> khat, ell, sk_state;
};

double now_s();
KernelFn kfn(const h2ulv_params& p);

// Capacity, in doubles, of the per-GPU array that holds the partial sums of
// the allocation-free exact matvec.
int64_t matvec_noalloc_capacity();

// Sketch probes and the acceptance slack of the learned-rank basis step.
constexpr int SKETCH_PROBES = 8;
constexpr double SKETCH_SLACK = 10.0;

// The 16 rank-model features of box i at level lev (see h2ulv_get_features).
void box_features(const h2ulv_factor& F, int lev, int i, int m, int ntargets,
                  int64_t ncols, double child_ratio, float* out);

// Factorize several problems (same parameters) with shared batched launches.
// pts[p] are device pointers (n[p] x 3 row-major).  On error nothing is returned
// (the exception carries the status).
std::vector<h2ulv_factor*> factorize_many(const std::vector<const double*>& pts,
                                          const std::vector<int64_t>& n,
                                          const h2ulv_params& params, hipStream_t s);

}  // namespace h2ulv

struct h2ulv_factor {
  h2ulv_params p{};
  int64_t n = 0;
  std::vector<double> hpts;  // host copy of the points (tree geometry, features)
  h2ulv::Tree tree;
  h2ulv::Lists lists;
  h2ulv::DBuf pts;   // device copy of the points (n x 3)
  h2ulv::DBuf perm;  // device tree permutation
  std::vector<h2ulv::LevelFactor> levels;  // index = level (0 unused)
  h2ulv::DBuf root_inv;
  int m_root = 0;
  h2ulv_stats stats{};
  // the caller's allocator of the factorization (has_alloc), used again for the
  // temporaries of later calls on this factor
  h2ulv_allocator alloc{};
  bool has_alloc = false;
  // separate row and column bases: the column side of the factorization, the
  // row bases of the transposed matrix (its levels hold V, T_V and the column
  // skeletons in U, Tt and sk; its elimination fields stay empty)
  std::unique_ptr<h2ulv_factor> colview;
  // solves recorded in HIP graphs, one per right-hand-side count (refinement
  // repeats the solve); destroyed first
  mutable std::mutex graph_mu;
  mutable std::vector<std::shared_ptr<h2ulv::SolveGraph>> solve_graphs;
};

struct h2ulv_rankmodel {
  h2ulv::DBuf theta, m, v;  // float parameters and Adam moments (device)
  int64_t step = 0;         // Adam steps taken
};

namespace h2ulv {
// Exact y = A x like the allocating matvec (same split and summation order),
// with the partial sums in the per-GPU array; fails with INVALID_ARG when they
// need more than matvec_noalloc_capacity() doubles.  Allocates nothing and does
// not synchronise the stream.
void matvec_noalloc(const h2ulv_factor& F, const double* x, int64_t ldx, double* y, int64_t ldy,
                    int nrhs, hipStream_t s);
}  // namespace h2ulv
