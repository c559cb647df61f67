// Kernels of the learned-rank variant of the basis step: Gaussian sketch
// matrices from a counter-based generator, the gather / norm kernels of the
// randomized error probe, and the rank MLP's forward, gradient and Adam update.
#include "h2ulv_learned.h"

#include <cmath>

namespace h2ulv {

namespace {

// SplitMix64 output function (Steele, Lea and Flood 2014).
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Position c of the stream starting at state `key`: c + 1 increments.
__host__ __device__ __forceinline__ uint64_t sm64_pos(uint64_t key, uint64_t c) {
  return sm64_mix(key + (c + 1ull) * 0x9E3779B97F4A7C15ull);
}

// Box-Muller (cosine branch): u1 in (0, 1] from position 2i, u2 in [0, 1) from 2i + 1.
__device__ __forceinline__ double gauss_at(uint64_t key, uint64_t i) {
  const uint64_t x1 = sm64_pos(key, 2ull * i);
  const uint64_t x2 = sm64_pos(key, 2ull * i + 1ull);
  const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

__device__ __forceinline__ int find_tile_item(const int64_t* ptr, int n, int64_t tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

uint64_t sm64_at(uint64_t key, uint64_t c) { return sm64_pos(key, c); }

uint64_t sketch_key(uint64_t seed, int lev, uint64_t id) {
  return sm64_pos(seed, ((uint64_t)lev << 40) | id);
}

// ---------------------------------------------------------------------------
// Gaussian sketch rows of points, 64 x 64 tiles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gauss_kernel(const GaussItem* __restrict__ items,
                                                    const int64_t* __restrict__ tile_ptr,
                                                    int nitems) {
  const int64_t tile = blockIdx.x;
  const int id = find_tile_item(tile_ptr, nitems, tile);
  const GaussItem it = items[id];
  const int64_t t = tile - tile_ptr[id];
  const int tr = (it.rows + 63) / 64;
  const int r0 = (int)(t % tr) * 64, c0 = (int)(t / tr) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = r0 + (e & 63), c = c0 + (e >> 6);
    if (r < it.rows && c < it.cols)
      it.dst[r + (int64_t)c * it.ld] =
          gauss_at(it.key, (uint64_t)c * (uint64_t)it.stride + (uint64_t)(it.idx[r] - it.sub));
  }
}

void launch_gauss(const GaussItem* items, const int64_t* tile_ptr, int64_t ntiles, int nitems,
                  hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(gauss_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, items, tile_ptr,
                     nitems);
}

// ---------------------------------------------------------------------------
// Column gather, 64 x 64 tiles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gather_cols_kernel(const GatherItem* __restrict__ items,
                                                          const int64_t* __restrict__ tile_ptr,
                                                          int nitems) {
  const int64_t tile = blockIdx.x;
  const int id = find_tile_item(tile_ptr, nitems, tile);
  const GatherItem it = items[id];
  const int64_t t = tile - tile_ptr[id];
  const int tr = (it.rows + 63) / 64;
  const int r0 = (int)(t % tr) * 64, c0 = (int)(t / tr) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = r0 + (e & 63), c = c0 + (e >> 6);
    if (r < it.rows && c < it.cols)
      it.dst[r + (int64_t)c * it.ldd] = it.src[r + (int64_t)it.idx[c] * it.lds];
  }
}

void launch_gather_cols(const GatherItem* items, const int64_t* tile_ptr, int64_t ntiles,
                        int nitems, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, items,
                     tile_ptr, nitems);
}

// ---------------------------------------------------------------------------
// Sum of squares and largest column sum of squares, one workgroup per item
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void norms_kernel(const NormItem* __restrict__ items) {
  __shared__ double s_sum[256];
  __shared__ double s_max[256];
  const NormItem it = items[blockIdx.x];
  double tot = 0.0, mx = 0.0;
  for (int c = threadIdx.x; c < it.cols; c += 256) {
    const double* a = it.A + (int64_t)c * it.lda;
    double s = 0.0;
    for (int r = 0; r < it.rows; ++r) s += a[r] * a[r];
    tot += s;
    mx = fmax(mx, s);
  }
  s_sum[threadIdx.x] = tot;
  s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
      s_max[threadIdx.x] = fmax(s_max[threadIdx.x], s_max[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    it.out[0] = s_sum[0];
    it.out[1] = s_max[0];
  }
}

void launch_norms(const NormItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(norms_kernel, dim3(nitems), dim3(256), 0, s, items);
}

// ---------------------------------------------------------------------------
// Rank MLP.  A workgroup of 256 threads takes MLP_TILE = 32 samples; the
// activations of every layer stay in LDS.  Hidden layer outputs are computed
// by the thread pair (neuron o = lane, sample s = wave + 4 j): the weight is
// read once per input and broadcast against the samples held in LDS.
// ---------------------------------------------------------------------------
namespace {

constexpr int NS = MLP_TILE;
constexpr int PER = NS / 4;  // samples per thread in the layer loops

struct MlpLds {
  float a0[NS][MLP_NF];
  float a1[NS][MLP_W];
  float a2[NS][MLP_W];
  float a3[NS][MLP_W];
  float y[NS];
  float dy[NS];
  float da[NS][MLP_W];
  float db[NS][MLP_W];
  float red[4];
};

template <int IN>
__device__ __forceinline__ void dense_relu(const float* __restrict__ W, const float* __restrict__ b,
                                           const float (*in)[IN], float (*out)[MLP_W]) {
  const int o = threadIdx.x & 63, w = threadIdx.x >> 6;
  float acc[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) acc[j] = b[o];
  for (int i = 0; i < IN; ++i) {
    const float wi = W[o * IN + i];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc[j] += wi * in[w + 4 * j][i];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) out[w + 4 * j][o] = fmaxf(acc[j], 0.0f);
}

// Forward pass of one tile; on return L.y holds the outputs (0 for padding).
__device__ void mlp_tile_forward(const float* __restrict__ th, const float* __restrict__ feat,
                                 int64_t n, int64_t s0, MlpLds& L) {
  for (int e = threadIdx.x; e < NS * MLP_NF; e += 256) {
    const int s = e / MLP_NF, f = e % MLP_NF;
    L.a0[s][f] = (s0 + s < n) ? feat[(s0 + s) * MLP_NF + f] : 0.0f;
  }
  __syncthreads();
  dense_relu<MLP_NF>(th + MLP_OFF_W1, th + MLP_OFF_B1, L.a0, L.a1);
  __syncthreads();
  dense_relu<MLP_W>(th + MLP_OFF_W2, th + MLP_OFF_B2, L.a1, L.a2);
  __syncthreads();
  dense_relu<MLP_W>(th + MLP_OFF_W3, th + MLP_OFF_B3, L.a2, L.a3);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float w4 = th[MLP_OFF_W4 + lane];
  for (int j = 0; j < PER; ++j) {
    const int s = w + 4 * j;
    const float v = wave_sum_f(w4 * L.a3[s][lane]);
    if (lane == 0) L.y[s] = v + th[MLP_OFF_B4];
  }
  __syncthreads();
}

// delta of the layer below: out[s][i] = (sum_o W[o][i] d[s][o]) * (a[s][i] > 0)
__device__ __forceinline__ void back_delta(const float* __restrict__ W, const float (*d)[MLP_W],
                                           const float (*a)[MLP_W], float (*out)[MLP_W]) {
  const int i = threadIdx.x & 63, w = threadIdx.x >> 6;
  float acc[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) acc[j] = 0.0f;
  for (int o = 0; o < MLP_W; ++o) {
    const float wo = W[o * MLP_W + i];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc[j] += wo * d[w + 4 * j][o];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int s = w + 4 * j;
    out[s][i] = a[s][i] > 0.0f ? acc[j] : 0.0f;
  }
}

// weight gradient of one layer: g[o][i] = sum_s d[s][o] a[s][i]; bias g[o] = sum_s d[s][o]
template <int IN>
__device__ __forceinline__ void weight_grad(const float (*d)[MLP_W], const float (*a)[IN],
                                            float* __restrict__ gW, float* __restrict__ gb) {
  for (int e = threadIdx.x; e < MLP_W * IN; e += 256) {
    const int o = e / IN, i = e % IN;
    float acc = 0.0f;
    for (int s = 0; s < NS; ++s) acc += d[s][o] * a[s][i];
    gW[e] = acc;
  }
  if (threadIdx.x < MLP_W) {
    float acc = 0.0f;
    for (int s = 0; s < NS; ++s) acc += d[s][threadIdx.x];
    gb[threadIdx.x] = acc;
  }
}

}  // namespace

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ th,
                                                          const float* __restrict__ feat,
                                                          int64_t n, float* __restrict__ y) {
  __shared__ MlpLds L;
  const int64_t s0 = (int64_t)blockIdx.x * NS;
  mlp_tile_forward(th, feat, n, s0, L);
  if (threadIdx.x < NS && s0 + threadIdx.x < n) y[s0 + threadIdx.x] = L.y[threadIdx.x];
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ th,
                                                       const float* __restrict__ feat,
                                                       const float* __restrict__ target,
                                                       int64_t n, float* __restrict__ partial,
                                                       float* __restrict__ partial_loss) {
  __shared__ MlpLds L;
  const int64_t s0 = (int64_t)blockIdx.x * NS;
  mlp_tile_forward(th, feat, n, s0, L);
  float* g = partial + (int64_t)blockIdx.x * MLP_NPARAM;
  const float inv_n = 1.0f / (float)n;
  // dL/dy and the tile's loss
  if (threadIdx.x < 64) {  // all of wave 0; its first NS lanes hold the samples
    const int s = threadIdx.x;
    float r = 0.0f;
    if (s < NS && s0 + s < n) r = L.y[s] - target[s0 + s];
    if (s < NS) L.dy[s] = 2.0f * r * inv_n;
    const float v = wave_sum_f(r * r * inv_n);
    if (s == 0) partial_loss[blockIdx.x] = v;
  }
  __syncthreads();
  // output layer
  if (threadIdx.x < MLP_W) {
    float acc = 0.0f;
    for (int s = 0; s < NS; ++s) acc += L.dy[s] * L.a3[s][threadIdx.x];
    g[MLP_OFF_W4 + threadIdx.x] = acc;
  }
  if (threadIdx.x == 0) {
    float acc = 0.0f;
    for (int s = 0; s < NS; ++s) acc += L.dy[s];
    g[MLP_OFF_B4] = acc;
  }
  {
    const int o = threadIdx.x & 63, w = threadIdx.x >> 6;
    const float w4 = th[MLP_OFF_W4 + o];
    for (int j = 0; j < PER; ++j) {
      const int s = w + 4 * j;
      L.da[s][o] = L.a3[s][o] > 0.0f ? L.dy[s] * w4 : 0.0f;  // delta of layer 3
    }
  }
  __syncthreads();
  weight_grad<MLP_W>(L.da, L.a2, g + MLP_OFF_W3, g + MLP_OFF_B3);
  back_delta(th + MLP_OFF_W3, L.da, L.a2, L.db);  // delta of layer 2
  __syncthreads();
  weight_grad<MLP_W>(L.db, L.a1, g + MLP_OFF_W2, g + MLP_OFF_B2);
  back_delta(th + MLP_OFF_W2, L.db, L.a1, L.da);  // delta of layer 1 (da is free again)
  __syncthreads();
  weight_grad<MLP_NF>(L.da, L.a0, g + MLP_OFF_W1, g + MLP_OFF_B1);
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial,
                                                         const float* __restrict__ partial_loss,
                                                         int64_t nblk, float* __restrict__ grad,
                                                         float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < MLP_NPARAM) {
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += partial[b * MLP_NPARAM + p];
    grad[p] = (float)acc;
  } else if (p == MLP_NPARAM) {
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += partial_loss[b];
    loss[0] = (float)acc;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ th, float* __restrict__ m,
                                                   float* __restrict__ v,
                                                   const float* __restrict__ g, int n, float lr,
                                                   float b1, float b2, float eps, float bc1,
                                                   float bc2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  th[p] -= lr * (mp / bc1) / (sqrtf(vp / bc2) + eps);
}

void launch_mlp_forward(const float* theta, const float* feat, int64_t n, float* y,
                        hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)((n + NS - 1) / NS);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(nb), dim3(256), 0, s, theta, feat, n, y);
}

void launch_mlp_grad(const float* theta, const float* feat, const float* target, int64_t n,
                     float* partial, float* partial_loss, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)((n + NS - 1) / NS);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(256), 0, s, theta, feat, target, n, partial,
                     partial_loss);
}

void launch_mlp_reduce(const float* partial, const float* partial_loss, int64_t nblk, float* grad,
                       float* loss, hipStream_t s) {
  const unsigned nb = (unsigned)((MLP_NPARAM + 1 + 255) / 256);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3(nb), dim3(256), 0, s, partial, partial_loss, nblk,
                     grad, loss);
}

void launch_adam(float* theta, float* m, float* v, const float* grad, int n, float lr, float beta1,
                 float beta2, float eps, float bc1, float bc2, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, m, v,
                     grad, n, lr, beta1, beta2, eps, bc1, bc2);
}

}  // namespace h2ulv
