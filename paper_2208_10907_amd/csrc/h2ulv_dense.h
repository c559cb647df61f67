// Batched dense building blocks (internal).
#pragma once

#include "h2ulv_batch.h"

namespace h2ulv {

// Triangular system with several right-hand sides: X = T^-1 B.
struct TriRhs {
  const double* T;
  int64_t ldt;
  int m;
  double* B;  // destroyed
  int64_t ldb;
  double* X;  // result
  int64_t ldx;
  int ncols;
};

struct SqMat {
  double* A;  // m x m, overwritten (LU factors) where noted
  int64_t lda;
  int m;
  double* inv;  // result
  int64_t ldinv;
};

struct QrW {
  double* W;  // m x k (ld m), overwritten
  int m, k;
  double* U;  // m x m (ld m) result
  double* T;  // k x k (ld k) result
};

// Tall (or short) matrix factored in place by blocked Householder QR; on
// return its upper triangle (rows < min(h, m)) holds R.
struct TallQr {
  double* A;
  int64_t lda;
  int h;  // rows
  int m;  // columns
};

void batched_qr_R(Stage& st, const std::vector<TallQr>& ms);
void trsm_lower_unit(Stage& st, const std::vector<TriRhs>& sys);
void trsm_upper(Stage& st, const std::vector<TriRhs>& sys);
void batched_lu(Stage& st, const std::vector<SqMat>& mats, int32_t* ipiv, int32_t* info,
                const std::vector<int64_t>& ipiv_off);
void batched_inverse(Stage& st, const std::vector<SqMat>& mats, int32_t** info_out,
                     int32_t** ipiv_out, std::vector<int64_t>* ipiv_off_out);
void batched_triu_inverse(Stage& st, const std::vector<SqMat>& mats);
void batched_qr_basis(Stage& st, const std::vector<QrW>& ws);

}  // namespace h2ulv
