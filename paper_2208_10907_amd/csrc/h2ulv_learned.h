// Kernels of the learned-rank variant of the basis step (internal): Gaussian
// sketch matrices, the randomized error probe, and the rank MLP.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2ulv {

// Rank MLP: 16 features -> 3 hidden layers of 64 (ReLU) -> 1 output.  One flat
// float array: W1 (64 x 16 row-major), b1, W2 (64 x 64), b2, W3, b3, w4, b4.
constexpr int MLP_NF = 16;
constexpr int MLP_W = 64;
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_W * MLP_NF;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_W;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_W * MLP_W;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_W;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_W * MLP_W;
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + MLP_W;
constexpr int MLP_OFF_B4 = MLP_OFF_W4 + MLP_W;
constexpr int MLP_NPARAM = MLP_OFF_B4 + 1;
constexpr int MLP_TILE = 32;  // samples per workgroup

// SplitMix64 (Steele, Lea, Flood 2014) read at position c of the stream that
// starts at state `key`; Gaussian deviate number i from positions 2i, 2i+1.
uint64_t sm64_at(uint64_t key, uint64_t c);
// Key of stream `id` at level `lev`: position (lev << 40) | id of the seed's stream.
uint64_t sketch_key(uint64_t seed, int lev, uint64_t id);
// Sketch rows are keyed by point: stream STREAM_FAR for far-field columns,
// STREAM_FILL for fill-in columns.
constexpr uint64_t STREAM_BASE = (uint64_t)1 << 39;
constexpr uint64_t STREAM_FAR = 0;
constexpr uint64_t STREAM_FILL = 1;

// dst(r, c) = deviate number c * stride + (idx[r] - sub) of `key` (column-major,
// ld): the sketch row of point idx[r] - sub among `stride` points
struct GaussItem {
  double* dst;
  int64_t ld;
  const int64_t* idx;
  int64_t sub;
  int64_t stride;
  uint64_t key;
  int32_t rows, cols;
};
// dst(:, j) = src(:, idx[j])   (rows x cols)
struct GatherItem {
  const double* src;
  int64_t lds;
  double* dst;
  int64_t ldd;
  const int32_t* idx;
  int32_t rows, cols;
};
// out[0] = sum of squares of A (rows x cols), out[1] = largest column sum of squares
struct NormItem {
  const double* A;
  int64_t lda;
  double* out;
  int32_t rows, cols;
};

void launch_gauss(const GaussItem* items, const int64_t* tile_ptr, int64_t ntiles, int nitems,
                  hipStream_t s);
void launch_gather_cols(const GatherItem* items, const int64_t* tile_ptr, int64_t ntiles,
                        int nitems, hipStream_t s);
void launch_norms(const NormItem* items, int nitems, hipStream_t s);

// y[s] = MLP(feat[s, :])   (feat: n x 16 row-major)
void launch_mlp_forward(const float* theta, const float* feat, int64_t n, float* y,
                        hipStream_t s);
// Per-workgroup partial gradients of mean (y - t)^2 (partial: nblk x NPARAM) and
// partial losses (nblk); nblk = ceil(n / MLP_TILE).
void launch_mlp_grad(const float* theta, const float* feat, const float* target, int64_t n,
                     float* partial, float* partial_loss, hipStream_t s);
// grad[p] = sum over blocks of partial[b, p]; loss[0] = sum of partial losses
void launch_mlp_reduce(const float* partial, const float* partial_loss, int64_t nblk, float* grad,
                       float* loss, hipStream_t s);
// Adam (Kingma & Ba 2015, Algorithm 1); bc1 = 1 - beta1^t, bc2 = 1 - beta2^t
void launch_adam(float* theta, float* m, float* v, const float* grad, int n, float lr, float beta1,
                 float beta2, float eps, float bc1, float bc2, hipStream_t s);

}  // namespace h2ulv
