// Device-kernel descriptors and launchers of the H^2-ULV library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2ulv {

struct KernelFn {
  int kind;      // 0 Laplace 1/r, 1 Yukawa exp(-alpha r)/r, 2 exp(b.(x - y) - alpha r)/r
  double alpha;
  double diag;   // value where row point == column point
  double b[3];   // drift of kind 2
};

// out[a + b*ld] = K(x[rows[a]], x[cols[b]])   (a < m, b < n)
struct KgenItem {
  const int64_t* rows;
  const int64_t* cols;
  double* out;
  int64_t ld;
  int32_t m, n;
  int32_t tr;   // 1: entries of the transposed kernel, K(x[cols[b]], x[rows[a]])
  int32_t pad;
};

// C = beta C + alpha * sum_t op(A_t) op(B_t); op(A) is M x K, op(B) is K x N.
template <typename T>
struct GemmItem {
  T* C;
  int64_t ldc;
  int32_t M, N;
  int32_t t0, nt;  // term range in the term table
  double alpha, beta;
};
template <typename T>
struct GemmTerm {
  const T* A;
  const T* B;
  int64_t lda, ldb;
  int32_t K;
  int32_t flags;  // bit0: op(A) = A^T, bit1: op(B) = B^T
};

// C = alpha sum_{s < S} P_s + beta C with P_s = P + s M N (M x N, ld M): the
// partial products of a GEMM item whose K range was split over S workgroups.
template <typename T>
struct SplitKItem {
  T* C;
  int64_t ldc;
  const T* P;
  int32_t M, N, S;
  double alpha, beta;
};

// One square (or tall, for QR) matrix per box for the factorization kernels.
struct MatDesc {
  double* A;
  int64_t lda;
  int32_t m;      // rows
  int32_t n;      // columns
  int32_t* ipiv;  // LU pivots (m entries), or QR pivots / work
  double* aux;    // QR: tau (n) ; LU: unused
  double* V;      // QR: explicit reflector block (ld = m), panel columns
  double* Tf;     // QR: block-reflector T factors, nb x nb per panel
  int32_t* info;  // per-matrix flag (singular / status)
  int32_t panel_ws;  // QR: V and Tf hold only the current panel
  int32_t pad;
};

// Generic batched 2-D copy: dst[i + j*ldd] = alpha * src(i, j) (+ beta dst)
// src(i, j) = src[i + j*lds] or src[j + i*lds] when trans.
struct CopyItem {
  const double* src;
  double* dst;
  int64_t lds, ldd;
  int32_t rows, cols;
  int32_t trans;
  int32_t pad;
};

// Column-pivoted QR with exact norms of one matrix (row interpolative decomposition).
struct PivQrItem {
  double* A;        // m x n, overwritten by R (upper part)
  int64_t lda;
  int32_t m, n;     // the pivoted QR acts on the n columns of this m x n matrix
  int32_t* piv;     // out: n column pivots
  int32_t* kout;    // out: rank
  double* diag;     // out: |R_tt| for t < min(m,n) (0 beyond the last step)
  double* work;     // n doubles: column norms
  double tol;
  int32_t cap;      // effective cap (>= 1), min(m, n, cap)
  int32_t pad;
};

// Column-pivoted QR of one large matrix spread over many workgroups, one step
// per pair of launches (pick/reflect, then apply/renormalise).
struct PivQrState {
  double* A;       // m x n, in place
  int64_t lda;
  int32_t m;       // rows
  int32_t n;       // columns (the pivoted ones)
  int32_t cap;     // steps allowed: at most min(m, n)
  int32_t pad;
  double* nrm;     // n column norms
  int32_t* piv;    // n pivots
  double* scal;    // [0] tau of the current step, [1] threshold tol |R_00|
  int32_t* flags;  // [0] stopped, [1] rank k so far
  double tol;
};

// Dense P^T from LU interchanges (ipiv == nullptr gives the identity).
struct PermItem {
  const int32_t* ipiv;
  double* out;
  int64_t ld;
  int32_t m;
  int32_t pad;
};

// Row-ID matrix W' from pivots and E = R11^-1 R12 (k x (m-k)).
struct WpItem {
  const int32_t* piv;
  const double* E;  // E(t, s) at E[t + s * ldE], s < m - k
  double* W;        // m x k, ld ldW
  int64_t ldE, ldW;
  int32_t m, k;
};

// Launchers (all asynchronous on `s`).  Device descriptor arrays must be
// resident on the device.
void launch_kgen(const KgenItem* items, const int64_t* tile_ptr, int64_t ntiles, int nitems,
                 const double* pts, KernelFn kf, int* dup_flag, hipStream_t s);
// TI: operand / MFMA type (f64 or f32, accumulation in that type); TC: type of C.
// Tile shapes tm x tn: 64 x 64, 64 x 128, 128 x 64, 128 x 128, 32 x 128.
template <typename TI, typename TC>
void launch_gemm(const GemmItem<TC>* items, const GemmTerm<TI>* terms, const int64_t* tile_ptr,
                 int64_t ntiles, int nitems, int tm, int tn, hipStream_t s);
template <typename T>
void launch_splitk_reduce(const SplitKItem<T>* items, const int64_t* tile_ptr, int64_t ntiles,
                          int nitems, hipStream_t s);
// Products with N <= GEMV_MAXN columns and B not transposed, on the vector
// units; tiles of 64 rows (tile_ptr: per-item prefix of ceil(M / 64)).
constexpr int GEMV_MAXN = 4;
void launch_gemv(const GemmItem<double>* items, const GemmTerm<double>* terms,
                 const int64_t* tile_ptr, int64_t ntiles, int nitems, hipStream_t s);
// maxrows: largest m - j0 over the matrices (selects the register-resident panel)
void launch_lu_panel(const MatDesc* d, int nmat, int j0, int nb, int maxrows, hipStream_t s);
void launch_lu_swap_trsm(const MatDesc* d, const int64_t* slab_ptr, int64_t nslabs, int nmat,
                         int j0, int nb, hipStream_t s);
void launch_trinv_diag(const MatDesc* d, const int64_t* blk_ptr, int64_t nblk, int nmat, int nb,
                       int upper, double* out, const int64_t* out_off, hipStream_t s);
// maxrows: largest m - j0 over the matrices (selects the register-resident panel)
void launch_qr_panel(const MatDesc* d, int nmat, int j0, int nb, int maxrows, hipStream_t s);
void launch_pivqr_init(const PivQrState* st, const int64_t* slab_ptr, int64_t nslabs, int n,
                       hipStream_t s);
void launch_pivqr_pick(const PivQrState* st, int n, int t, hipStream_t s);
// maxcols: largest column count over the n matrices
void launch_pivqr_apply(const PivQrState* st, int n, int maxcols, int t, hipStream_t s);
void launch_pivqr(const PivQrItem* items, int nitems, hipStream_t s);
void launch_copy(const CopyItem* items, const int64_t* tile_ptr, int64_t ntiles, int nitems,
                 double alpha, double beta, hipStream_t s);
void launch_perm_matrix(const PermItem* items, const int64_t* slab_ptr, int64_t nslabs,
                        int nitems, hipStream_t s);
void launch_wprime(const WpItem* items, int nitems, hipStream_t s);
void launch_zero_lower(const CopyItem* items, int nitems, hipStream_t s);
void launch_logdet(const MatDesc* d, int nmat, double* out, hipStream_t s);
// Exact y = A x.  work: matvec_work_words(n, nrhs) doubles for the partial sums
// of split source ranges (nullptr: one range per target block)
int64_t matvec_work_words(int64_t n, int nrhs);
void launch_matvec(const double* pts, int64_t n, KernelFn kf, const double* x, int64_t ldx,
                   double* y, int64_t ldy, int nrhs, double* work, hipStream_t s);
void launch_convert_d2f(const double* src, float* dst, int64_t count, hipStream_t s);
void launch_convert_f2d(const float* src, double* dst, int64_t count, hipStream_t s);
void launch_resid_norms(const double* b, int64_t ldb, const double* ax, int64_t ldax, double* r,
                        int64_t ldr, int64_t n, int nrhs, double* rnorm2, double* bnorm2,
                        hipStream_t s);
// C = A^T B (M x N, N <= 8) for a long inner dimension n; partial holds
// GRAM_CHUNKS * M * N doubles.  Deterministic.
constexpr int GRAM_CHUNKS = 256;
void launch_gram(const double* A, int64_t lda, int M, const double* B, int64_t ldb, int N,
                 int64_t n, double* C, int64_t ldc, double* partial, hipStream_t s);
void launch_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                     double* partial, int nblk, double* out, hipStream_t s);
void launch_scale_inv_norm(double* dst, const double* src, const double* nrm2, int64_t n,
                           hipStream_t s);
void launch_axpy_cols(double* x, int64_t ldx, const double* d, int64_t ldd, int64_t n, int nrhs,
                      hipStream_t s);
void launch_permute_rows(const double* src, int64_t lds, double* dst, int64_t ldd,
                         const int64_t* perm, int64_t n, int nrhs, int inverse, hipStream_t s);

}  // namespace h2ulv
