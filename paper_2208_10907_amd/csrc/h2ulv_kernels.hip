// HIP kernels of the H^2-ULV sweep for CDNA4 (gfx950).
//
// Every kernel is batched: one launch covers every box (or block pair) of a
// tree level, since the boxes of a level are independent of each other once
// the fill-ins are inside the shared bases (Sec. III-C, III-D of the paper).
// Descriptor tables live in device memory; tiles are mapped to items by a
// binary search over a prefix-sum table so that uneven block sizes share one
// launch.  All matrices are column-major.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "h2ulv_kernels.h"

namespace h2ulv {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_item(const int64_t* ptr, int n, int64_t tile) {
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

// K(x, y) with d = x - y, r2 = |d|^2 > 0; sgn = -1 evaluates K(y, x)
__device__ __forceinline__ double kernel_value(const KernelFn& kf, double r2, double dx,
                                               double dy, double dz, double sgn) {
  double r = sqrt(r2);
  if (kf.kind == 0) return 1.0 / r;
  if (kf.kind == 1) return exp(-kf.alpha * r) / r;
  const double bd = sgn * (kf.b[0] * dx + kf.b[1] * dy + kf.b[2] * dz);
  return exp(bd - kf.alpha * r) / r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum over 256 threads (4 waves); every thread gets the result.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0] + sh[1] + sh[2] + sh[3];
  return s;
}

// Block-wide sum over NW waves; every thread gets the result (same order in
// every thread).
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) s += sh[q];
  return s;
}

// ---------------------------------------------------------------------------
// Kernel-matrix generation (dense near blocks, far-field samples, skeleton
// couplings).  Tile 64 x 64, 256 threads; writes coalesced along rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void kgen_kernel(const KgenItem* __restrict__ items,
                                                   const int64_t* __restrict__ tile_ptr,
                                                   int nitems, const double* __restrict__ pts,
                                                   KernelFn kf, int* dup_flag) {
  int64_t tile = blockIdx.x;
  int id = find_item(tile_ptr, nitems, tile);
  KgenItem it = items[id];
  int64_t local = tile - tile_ptr[id];
  int tm = (it.m + 63) >> 6;
  int ti = (int)(local % tm), tj = (int)(local / tm);
  int a = ti * 64 + (threadIdx.x & 63);
  int b0 = tj * 64 + (threadIdx.x >> 6);
  if (a >= it.m) return;
  int64_t ra = it.rows[a];
  double xa = pts[3 * ra], ya = pts[3 * ra + 1], za = pts[3 * ra + 2];
  const double sgn = it.tr ? -1.0 : 1.0;
  bool dup = false;
  for (int q = 0; q < 16; ++q) {
    int b = b0 + 4 * q;
    if (b >= it.n) break;
    int64_t cb = it.cols[b];
    double v;
    if (cb == ra) {
      v = kf.diag;
    } else {
      double dx = xa - pts[3 * cb], dy = ya - pts[3 * cb + 1], dz = za - pts[3 * cb + 2];
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) {
        dup = true;
        v = 0.0;
      } else {
        v = kernel_value(kf, r2, dx, dy, dz, sgn);
      }
    }
    it.out[a + (int64_t)b * it.ld] = v;
  }
  if (dup) *dup_flag = 1;
}

void launch_kgen(const KgenItem* items, const int64_t* tile_ptr, int64_t ntiles, int nitems,
                 const double* pts, KernelFn kf, int* dup_flag, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(kgen_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, items, tile_ptr,
                     nitems, pts, kf, dup_flag);
}

// ---------------------------------------------------------------------------
// Grouped GEMM on the matrix cores.
// MFMA 16x16x4 operand layout (one value per lane): A(i, k) with i = lane % 16,
// k = lane / 16; B(k, j) with j = lane % 16, k = lane / 16.  Accumulator element
// r of lane l holds D(row, l % 16) with row = 4 r + l / 16 for the f64
// instruction and row = 4 (l / 16) + r for the f32 one (checked on gfx950).
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Load through a global (address space 1) pointer: operand pointers read from
// descriptor tables are generic, and generic (flat) loads also count against
// the LDS wait counter, which would make every LDS wait of the GEMM wait for
// the next tile's global loads as well.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch; each XCD has its own L2).
// Within every block of 8 G consecutive tiles, the G consecutive tiles of chunk
// x go to XCD x: neighbouring tiles of an item (the same column band of B)
// then share that XCD's L2, while all XCDs still advance through the tiles
// together.  Tiles past the last whole block keep their index.
template <int G>
__device__ __forceinline__ int64_t xcd_chunk_tile(int64_t b, int64_t n) {
  const int64_t full = n / (8 * G) * (8 * G);
  if (b >= full) return b;
  const int64_t q = b / (8 * G), r = b % (8 * G);
  return q * (8 * G) + (r % 8) * G + r / 8;
}

// C = beta C + alpha sum_t op(A_t) op(B_t) for a batch of items of any size.
// A workgroup (4 waves, 2 x 2, each a (TM/2) x (TN/2) block of 16 x 16 MFMA
// accumulators) owns a TM x TN tile of one item (found
// by binary search over the tile prefix table) and runs over the flattened
// sequence of 16-deep K tiles of all the item's terms.  The K tiles are staged
// through two LDS buffers: the next tile is loaded from global memory into
// registers while the MFMAs consume the current one, then stored into the other
// buffer, with one barrier per tile; the A/B fragments of the next 4-deep step
// are read from LDS before the MFMAs of the current step.  Interior tiles load
// without bounds checks.
template <typename T, typename TC, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmItem<TC>* __restrict__ items,
                                                    const GemmTerm<T>* __restrict__ terms,
                                                    const int64_t* __restrict__ tile_ptr,
                                                    int nitems) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int BM = TM / 32, BN = TN / 32;
  constexpr int LA = TM / 16, LB = TN / 16;
  __shared__ T As[2][16][TM + 4];
  __shared__ T Bs[2][16][TN + 4];
  const int64_t tile = xcd_chunk_tile<4>(blockIdx.x, gridDim.x);
  const int id = find_item(tile_ptr, nitems, tile);
  const GemmItem<TC> it = items[id];
  const int64_t local = tile - tile_ptr[id];
  const int tm = (it.M + TM - 1) / TM;
  const int row0 = (int)(local % tm) * TM, col0 = (int)(local / tm) * TN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w & 1, wc = w >> 1;
  const bool rows_in = row0 + TM <= it.M, cols_in = col0 + TN <= it.N;
  v4 acc[BM][BN];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) acc[a][b] = v4{0, 0, 0, 0};
  T ra[LA], rb[LB];
  auto load = [&](const GemmTerm<T>& tt, int k0) {
    const bool kin = k0 + 16 <= tt.K;
    if (!(tt.flags & 1)) {
      const int i = tid % TM, kb = tid / TM;
      const T* p = tt.A + (row0 + i) + (int64_t)(k0 + kb) * tt.lda;
      if (rows_in && kin) {
#pragma unroll
        for (int r = 0; r < LA; ++r) ra[r] = gload(p + (int64_t)((256 / TM) * r) * tt.lda);
      } else {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
          const int kk = kb + (256 / TM) * r, gi = row0 + i, gk = k0 + kk;
          ra[r] = (gi < it.M && gk < tt.K) ? gload(tt.A + gi + (int64_t)gk * tt.lda) : T(0);
        }
      }
    } else {
      const int kk = tid & 15, ib = tid >> 4;
      const T* p = tt.A + (k0 + kk) + (int64_t)(row0 + ib) * tt.lda;
      if (rows_in && kin) {
#pragma unroll
        for (int r = 0; r < LA; ++r) ra[r] = gload(p + (int64_t)(16 * r) * tt.lda);
      } else {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
          const int i = ib + 16 * r, gi = row0 + i, gk = k0 + kk;
          ra[r] = (gi < it.M && gk < tt.K) ? gload(tt.A + gk + (int64_t)gi * tt.lda) : T(0);
        }
      }
    }
    if (!(tt.flags & 2)) {
      const int kk = tid & 15, jb = tid >> 4;
      const T* p = tt.B + (k0 + kk) + (int64_t)(col0 + jb) * tt.ldb;
      if (cols_in && kin) {
#pragma unroll
        for (int r = 0; r < LB; ++r) rb[r] = gload(p + (int64_t)(16 * r) * tt.ldb);
      } else {
#pragma unroll
        for (int r = 0; r < LB; ++r) {
          const int j = jb + 16 * r, gj = col0 + j, gk = k0 + kk;
          rb[r] = (gj < it.N && gk < tt.K) ? gload(tt.B + gk + (int64_t)gj * tt.ldb) : T(0);
        }
      }
    } else {
      const int j = tid % TN, kb = tid / TN;
      const T* p = tt.B + (col0 + j) + (int64_t)(k0 + kb) * tt.ldb;
      if (cols_in && kin) {
#pragma unroll
        for (int r = 0; r < LB; ++r) rb[r] = gload(p + (int64_t)((256 / TN) * r) * tt.ldb);
      } else {
#pragma unroll
        for (int r = 0; r < LB; ++r) {
          const int kk = kb + (256 / TN) * r, gj = col0 + j, gk = k0 + kk;
          rb[r] = (gj < it.N && gk < tt.K) ? gload(tt.B + gj + (int64_t)gk * tt.ldb) : T(0);
        }
      }
    }
  };
  auto store = [&](const GemmTerm<T>& tt, int buf) {
    if (!(tt.flags & 1)) {
      const int i = tid % TM, kb = tid / TM;
#pragma unroll
      for (int r = 0; r < LA; ++r) As[buf][kb + (256 / TM) * r][i] = ra[r];
    } else {
      const int kk = tid & 15, ib = tid >> 4;
#pragma unroll
      for (int r = 0; r < LA; ++r) As[buf][kk][ib + 16 * r] = ra[r];
    }
    if (!(tt.flags & 2)) {
      const int kk = tid & 15, jb = tid >> 4;
#pragma unroll
      for (int r = 0; r < LB; ++r) Bs[buf][kk][jb + 16 * r] = rb[r];
    } else {
      const int j = tid % TN, kb = tid / TN;
#pragma unroll
      for (int r = 0; r < LB; ++r) Bs[buf][kb + (256 / TN) * r][j] = rb[r];
    }
  };
  int t = it.t0;
  const int tend = it.t0 + it.nt;
  while (t < tend && terms[t].K <= 0) ++t;
  if (t < tend) {
    // the current term's descriptor stays in registers; the table is read again
    // only when the K loop moves on to the next term
    GemmTerm<T> tc = terms[t];
    int k0 = 0, cur = 0;
    load(tc, k0);
    store(tc, 0);
    __syncthreads();
    for (;;) {
      int tn = t, kn = k0 + 16;
      GemmTerm<T> tx = tc;
      if (kn >= tc.K) {
        kn = 0;
        ++tn;
        while (tn < tend && terms[tn].K <= 0) ++tn;
        if (tn < tend) tx = terms[tn];
      }
      const bool more = tn < tend;
      if (more) load(tx, kn);
      T av[2][BM], bv[2][BN];
      {
        const int kk = lane >> 4;
#pragma unroll
        for (int a = 0; a < BM; ++a) av[0][a] = As[cur][kk][(TM / 2) * wr + 16 * a + (lane & 15)];
#pragma unroll
        for (int b = 0; b < BN; ++b) bv[0][b] = Bs[cur][kk][(TN / 2) * wc + 16 * b + (lane & 15)];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (s < 3) {
          const int kk = 4 * (s + 1) + (lane >> 4);
#pragma unroll
          for (int a = 0; a < BM; ++a)
            av[(s + 1) & 1][a] = As[cur][kk][(TM / 2) * wr + 16 * a + (lane & 15)];
#pragma unroll
          for (int b = 0; b < BN; ++b)
            bv[(s + 1) & 1][b] = Bs[cur][kk][(TN / 2) * wc + 16 * b + (lane & 15)];
        }
#pragma unroll
        for (int a = 0; a < BM; ++a)
#pragma unroll
          for (int b = 0; b < BN; ++b) acc[a][b] = Mfma<T>::mac(av[s & 1][a], bv[s & 1][b], acc[a][b]);
      }
      if (!more) break;
      store(tx, cur ^ 1);
      __syncthreads();
      cur ^= 1;
      t = tn;
      k0 = kn;
      tc = tx;
    }
  }
  const TC alpha = (TC)it.alpha, beta = (TC)it.beta;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + (TM / 2) * wr + 16 * bi + Mfma<T>::row(lane, r);
        const int col = col0 + (TN / 2) * wc + 16 * bj + (lane & 15);
        if (row < it.M && col < it.N) {
          TC v = alpha * (TC)acc[bi][bj][r];
          TC* c = it.C + row + (int64_t)col * it.ldc;
          if (beta != TC(0)) v += beta * (*c);
          *c = v;
        }
      }
}

template <typename TI, typename TC>
void launch_gemm(const GemmItem<TC>* items, const GemmTerm<TI>* terms, const int64_t* tile_ptr,
                 int64_t ntiles, int nitems, int tm, int tn, hipStream_t s) {
  if (ntiles <= 0) return;
  const dim3 g((unsigned)ntiles), b(256);
  if (tm == 32)  // 32 x 128 tiles for batches whose items have M <= 32
    hipLaunchKernelGGL((gemm_kernel<TI, TC, 32, 128>), g, b, 0, s, items, terms, tile_ptr, nitems);
  else if (tm == 128 && tn == 128)
    hipLaunchKernelGGL((gemm_kernel<TI, TC, 128, 128>), g, b, 0, s, items, terms, tile_ptr, nitems);
  else if (tm == 128)
    hipLaunchKernelGGL((gemm_kernel<TI, TC, 128, 64>), g, b, 0, s, items, terms, tile_ptr, nitems);
  else if (tn == 128)
    hipLaunchKernelGGL((gemm_kernel<TI, TC, 64, 128>), g, b, 0, s, items, terms, tile_ptr, nitems);
  else
    hipLaunchKernelGGL((gemm_kernel<TI, TC, 64, 64>), g, b, 0, s, items, terms, tile_ptr, nitems);
}
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const SplitKItem<T>* __restrict__ items,
                                                            const int64_t* __restrict__ tile_ptr,
                                                            int nitems) {
  const int64_t tile = blockIdx.x;
  const int id = find_item(tile_ptr, nitems, tile);
  const SplitKItem<T> it = items[id];
  const int64_t local = tile - tile_ptr[id];
  const int tmr = (it.M + 63) / 64;
  const int r = (int)(local % tmr) * 64 + (threadIdx.x & 63);
  const int c0 = (int)(local / tmr) * 64 + (threadIdx.x >> 6);
  if (r >= it.M) return;
  const int64_t mn = (int64_t)it.M * it.N;
  for (int c = c0; c < min(it.N, (int)(local / tmr) * 64 + 64); c += 4) {
    const T* p = it.P + r + (int64_t)c * it.M;
    T acc = 0;
    for (int sp = 0; sp < it.S; ++sp) acc += p[sp * mn];
    T* cp = it.C + r + (int64_t)c * it.ldc;
    T v = (T)it.alpha * acc;
    if (it.beta != 0.0) v += (T)it.beta * (*cp);
    *cp = v;
  }
}

// ---------------------------------------------------------------------------
// Products with at most GEMV_MAXN right-hand columns (the solve's vectors):
// C = beta C + alpha sum_t op(A_t) B_t with B_t not transposed.  This is
// matrix-vector work, bound by reading A once from HBM, so it runs on the
// vector units: one 256-thread workgroup per 64 rows of an item.
//   op(A) = A (column-major M x K): lane = row, wave = k mod 4, four columns of
//     A in flight per wave (each a coalesced 64-row segment);
//   op(A) = A^T (row i of op(A) contiguous): wave w takes rows 16w..16w+15,
//     four at a time, lanes over k, then a wave sum per row and column.
// Per-wave partial sums meet in LDS and are added in wave order (deterministic).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gemv_kernel(const GemmItem<double>* __restrict__ items,
                                                   const GemmTerm<double>* __restrict__ terms,
                                                   const int64_t* __restrict__ tile_ptr,
                                                   int nitems) {
  __shared__ double red[4][64][GEMV_MAXN];
  const int64_t tile = blockIdx.x;
  const int id = find_item(tile_ptr, nitems, tile);
  const GemmItem<double> it = items[id];
  const int i0 = (int)(tile - tile_ptr[id]) * 64;
  const int M = it.M, N = it.N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < GEMV_MAXN; ++j) red[w][lane][j] = 0.0;  // this wave's slots only
  double acc[GEMV_MAXN];
#pragma unroll
  for (int j = 0; j < GEMV_MAXN; ++j) acc[j] = 0.0;
  for (int t = it.t0; t < it.t0 + it.nt; ++t) {
    const GemmTerm<double> tt = terms[t];
    const int K = tt.K;
    if (!(tt.flags & 1)) {
      const int i = i0 + lane;
      if (i < M) {
        const double* a = tt.A + i;
        int k = w;
        for (; k + 12 < K; k += 16) {
          double av[4], bv[4][GEMV_MAXN];
#pragma unroll
          for (int q = 0; q < 4; ++q) av[q] = gload(a + (int64_t)(k + 4 * q) * tt.lda);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < GEMV_MAXN; ++j)
              bv[q][j] = j < N ? gload(tt.B + (k + 4 * q) + (int64_t)j * tt.ldb) : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < GEMV_MAXN; ++j) acc[j] = fma(av[q], bv[q][j], acc[j]);
        }
        for (; k < K; k += 4) {
          const double av = gload(a + (int64_t)k * tt.lda);
#pragma unroll
          for (int j = 0; j < GEMV_MAXN; ++j)
            acc[j] = fma(av, j < N ? gload(tt.B + k + (int64_t)j * tt.ldb) : 0.0, acc[j]);
        }
      }
    } else {
      for (int g = 0; g < 4; ++g) {  // rows 16w + 4g .. 16w + 4g + 3
        const int rl = 16 * w + 4 * g;
        double pr[4][GEMV_MAXN];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < GEMV_MAXN; ++j) pr[q][j] = 0.0;
        for (int k = lane; k < K; k += 64) {
          double bv[GEMV_MAXN];
#pragma unroll
          for (int j = 0; j < GEMV_MAXN; ++j)
            bv[j] = j < N ? gload(tt.B + k + (int64_t)j * tt.ldb) : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = i0 + rl + q;
            const double av = i < M ? gload(tt.A + k + (int64_t)i * tt.lda) : 0.0;
#pragma unroll
            for (int j = 0; j < GEMV_MAXN; ++j) pr[q][j] = fma(av, bv[j], pr[q][j]);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < GEMV_MAXN; ++j) {
            const double v = wave_sum(pr[q][j]);
            if (lane == 0) red[w][rl + q][j] += v;
          }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < GEMV_MAXN; ++j) red[w][lane][j] += acc[j];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int r = threadIdx.x, i = i0 + r;
    if (i < M) {
      for (int j = 0; j < N; ++j) {
        const double sum = ((red[0][r][j] + red[1][r][j]) + red[2][r][j]) + red[3][r][j];
        double* cp = it.C + i + (int64_t)j * it.ldc;
        double v = it.alpha * sum;
        if (it.beta != 0.0) v += it.beta * (*cp);
        *cp = v;
      }
    }
  }
}

void launch_gemv(const GemmItem<double>* items, const GemmTerm<double>* terms,
                 const int64_t* tile_ptr, int64_t ntiles, int nitems, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(gemv_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, items, terms, tile_ptr,
                     nitems);
}

template <typename T>
void launch_splitk_reduce(const SplitKItem<T>* items, const int64_t* tile_ptr, int64_t ntiles,
                          int nitems, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3((unsigned)ntiles), dim3(256), 0, s, items,
                     tile_ptr, nitems);
}
template void launch_splitk_reduce<double>(const SplitKItem<double>*, const int64_t*, int64_t, int,
                                           hipStream_t);
template void launch_splitk_reduce<float>(const SplitKItem<float>*, const int64_t*, int64_t, int,
                                          hipStream_t);

template void launch_gemm<double, double>(const GemmItem<double>*, const GemmTerm<double>*,
                                          const int64_t*, int64_t, int, int, int, hipStream_t);
template void launch_gemm<float, float>(const GemmItem<float>*, const GemmTerm<float>*,
                                        const int64_t*, int64_t, int, int, int, hipStream_t);
template void launch_gemm<float, double>(const GemmItem<double>*, const GemmTerm<float>*,
                                         const int64_t*, int64_t, int, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Blocked LU with partial pivoting (Sec. II-B Eq. lu: LU of S^RR; also the
// diagonal blocks D_kk of the fill-in step, Sec. III-B, and the root).
// Panel kernel: one workgroup per matrix factors columns [j0, j0+w) of rows
// [j0, m): pivot = largest |a| (lowest row on ties), row swap inside the
// panel, scaling and rank-1 updates of the panel.  Row swaps outside the panel,
// the U12 triangular solve and the trailing GEMM are separate launches.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lu_panel_kernel(const MatDesc* __restrict__ ds, int j0,
                                                       int nb) {
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  const MatDesc d = ds[blockIdx.x];
  const int m = d.m;
  if (m <= j0) return;
  const int w = min(nb, m - j0);
  double* A = d.A;
  const int64_t lda = d.lda;
  const int tid = threadIdx.x;
  for (int jj = 0; jj < w; ++jj) {
    const int col = j0 + jj;
    double best = -1.0;
    int bi = m;
    for (int r = col + tid; r < m; r += 256) {
      double v = fabs(A[r + (int64_t)col * lda]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
    red_v[tid] = best;
    red_i[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        double vo = red_v[tid + s];
        int io = red_i[tid + s];
        if (vo > red_v[tid] || (vo == red_v[tid] && io < red_i[tid])) {
          red_v[tid] = vo;
          red_i[tid] = io;
        }
      }
      __syncthreads();
    }
    int p = red_i[0];
    double pv = red_v[0];
    __syncthreads();
    if (!(pv > 0.0) || !isfinite(pv) || p >= m) {
      if (tid == 0 && *d.info == 0) *d.info = col + 1;
      p = col;
    }
    if (tid == 0) d.ipiv[col] = p;
    if (p != col) {
      for (int c = j0 + tid; c < j0 + w; c += 256) {
        double t0 = A[col + (int64_t)c * lda];
        A[col + (int64_t)c * lda] = A[p + (int64_t)c * lda];
        A[p + (int64_t)c * lda] = t0;
      }
    }
    __syncthreads();
    const double inv = 1.0 / A[col + (int64_t)col * lda];
    for (int r = col + 1 + tid; r < m; r += 256) {
      double l = A[r + (int64_t)col * lda] * inv;
      A[r + (int64_t)col * lda] = l;
      for (int c = col + 1; c < j0 + w; ++c)
        A[r + (int64_t)c * lda] -= l * A[col + (int64_t)c * lda];
    }
    __syncthreads();
  }
}

// The same panel factorization with the panel held in registers: 1024 threads,
// logical row r of the panel in thread r % 1024, slot r / 1024 (at most
// LUP_RPT * 1024 rows).  Columns are taken in groups of LUP_G, left-looking: a
// group is loaded once, updated by the L columns left of it (unit-lower solve
// of its top rows, then one product for the rest), factored with partial
// pivoting in registers (lowest row on ties) and written back.  Interchanges
// are not applied to the other panel columns as they happen: the kernel keeps
// the row permutation in LDS (logical row r lives in memory row perm[r] for
// every panel column) and puts the moved rows in place once, at the end.
// Same pivots, factors and info as lu_panel_kernel up to the summation order
// of the updates.
constexpr int LUP_RPT = 4;
constexpr int LUP_G = 4;
constexpr int LUP_THREADS = 1024;
constexpr int LUP_MAXROWS = LUP_RPT * LUP_THREADS;
constexpr int LUP_KB = 4;  // L columns per batch of loads in the update
static_assert(LUP_G % LUP_KB == 0, "group width must be a multiple of the load batch");

__global__ __launch_bounds__(LUP_THREADS) void lu_panel_reg_kernel(const MatDesc* __restrict__ ds,
                                                                   int j0, int nb) {
  __shared__ double s_u[64 * LUP_G];
  __shared__ double s_prow[LUP_G], s_crow[LUP_G];
  __shared__ double s_wv[LUP_THREADS / 64];
  __shared__ int s_wi[LUP_THREADS / 64];
  __shared__ int s_piv[64];
  __shared__ int s_perm[LUP_MAXROWS];
  const MatDesc d = ds[blockIdx.x];
  const int m = d.m;
  if (m <= j0) return;
  const int w = min(nb, m - j0);
  const int h = m - j0;
  const int64_t lda = d.lda;
  double* P = d.A + j0 + (int64_t)j0 * lda;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int r = tid; r < h; r += LUP_THREADS) s_perm[r] = r;
  __syncthreads();
  int info_col = 0;  // first singular column (1-based), thread 0 only
  for (int g0 = 0; g0 < w; g0 += LUP_G) {
    const int gw = min(LUP_G, w - g0);
    // memory rows of this thread's logical rows (the permutation is only
    // changed inside the column loop below)
    int pr[LUP_RPT];
#pragma unroll
    for (int i = 0; i < LUP_RPT; ++i) {
      const int r = tid + LUP_THREADS * i;
      pr[i] = r < h ? s_perm[r] : 0;
    }
    double x[LUP_RPT][LUP_G];
#pragma unroll
    for (int i = 0; i < LUP_RPT; ++i) {
      const int r = tid + LUP_THREADS * i;
#pragma unroll
      for (int c = 0; c < LUP_G; ++c)
        x[i][c] = (r < h && c < gw) ? gload(P + pr[i] + (int64_t)(g0 + c) * lda) : 0.0;
    }
    if (g0 > 0) {
      // top rows: U = L11^-1 A_top with L11 = P(0:g0, 0:g0), unit lower (one wave,
      // the columns of the group side by side)
      if (tid < g0) {
#pragma unroll
        for (int c = 0; c < LUP_G; ++c) s_u[tid + 64 * c] = x[0][c];
      }
      __syncthreads();
      if (wv == 0) {
        const bool top = lane < g0;
        double val[LUP_G];
#pragma unroll
        for (int c = 0; c < LUP_G; ++c) val[c] = top ? s_u[lane + 64 * c] : 0.0;
        const double* lrow = P + (top ? s_perm[lane] : 0);
        for (int k = 0; k < g0 - 1; ++k) {
          const bool below = top && lane > k;
          const double l = below ? gload(lrow + (int64_t)k * lda) : 0.0;
#pragma unroll
          for (int c = 0; c < LUP_G; ++c) {
            const double uk = __shfl(val[c], k, 64);
            if (below) val[c] -= l * uk;
          }
        }
        if (top) {
#pragma unroll
          for (int c = 0; c < LUP_G; ++c)
            if (c < gw) s_u[lane + 64 * c] = val[c];
        }
      }
      __syncthreads();
      if (tid < g0) {
#pragma unroll
        for (int c = 0; c < LUP_G; ++c) x[0][c] = s_u[tid + 64 * c];
      }
      // rows g0..h-1: A -= L(:, 0:g0) U, LUP_KB columns of L per batch of loads
      for (int k0 = 0; k0 < g0; k0 += LUP_KB) {
        double l[LUP_RPT][LUP_KB];
#pragma unroll
        for (int i = 0; i < LUP_RPT; ++i) {
          const int r = tid + LUP_THREADS * i;
          const bool ok = r >= g0 && r < h;
#pragma unroll
          for (int kk = 0; kk < LUP_KB; ++kk)
            l[i][kk] = ok ? gload(P + pr[i] + (int64_t)(k0 + kk) * lda) : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < LUP_KB; ++kk) {
          double u[LUP_G];
#pragma unroll
          for (int c = 0; c < LUP_G; ++c) u[c] = s_u[k0 + kk + 64 * c];
#pragma unroll
          for (int i = 0; i < LUP_RPT; ++i) {
            const int r = tid + LUP_THREADS * i;
            if (r >= g0 && r < h) {
#pragma unroll
              for (int c = 0; c < LUP_G; ++c) x[i][c] -= l[i][kk] * u[c];
            }
          }
        }
      }
    }
    // Two barriers per column: s_wv / s_wi are read before the second, and
    // s_prow / s_crow are read before the next column's first, so neither is
    // written again while a thread may still read it.
#pragma unroll
    for (int jj = 0; jj < LUP_G; ++jj) {
      if (jj >= gw) break;
      const int col = g0 + jj;
      double best = -1.0;
      int bi = h;
#pragma unroll
      for (int i = 0; i < LUP_RPT; ++i) {
        const int r = tid + LUP_THREADS * i;
        if (r >= col && r < h) {
          const double v = fabs(x[i][jj]);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double vo = __shfl_xor(best, off, 64);
        const int io = __shfl_xor(bi, off, 64);
        if (vo > best || (vo == best && io < bi)) {
          best = vo;
          bi = io;
        }
      }
      if (lane == 0) {
        s_wv[wv] = best;
        s_wi[wv] = bi;
      }
      __syncthreads();
      best = s_wv[0];
      bi = s_wi[0];
      for (int q = 1; q < LUP_THREADS / 64; ++q) {
        const double vo = s_wv[q];
        const int io = s_wi[q];
        if (vo > best || (vo == best && io < bi)) {
          best = vo;
          bi = io;
        }
      }
      int p = bi;
      if (!(best > 0.0) || !isfinite(best) || p >= h) {
        if (tid == 0 && info_col == 0) info_col = j0 + col + 1;
        p = col;
      }
      // rows col and p: col < 64 lives in thread col, slot 0
      const int pt = p % LUP_THREADS, ps = p / LUP_THREADS;
      if (tid == pt) {
#pragma unroll
        for (int i = 0; i < LUP_RPT; ++i)
          if (i == ps) {
#pragma unroll
            for (int c = 0; c < LUP_G; ++c) s_prow[c] = x[i][c];
          }
      }
      if (tid == col) {
#pragma unroll
        for (int c = 0; c < LUP_G; ++c) s_crow[c] = x[0][c];
      }
      if (tid == 0) {
        s_piv[col] = p;
        if (p != col) {
          const int t0 = s_perm[col];
          s_perm[col] = s_perm[p];
          s_perm[p] = t0;
        }
      }
      __syncthreads();
      if (p != col) {
        if (tid == pt) {
#pragma unroll
          for (int i = 0; i < LUP_RPT; ++i)
            if (i == ps) {
#pragma unroll
              for (int c = 0; c < LUP_G; ++c) x[i][c] = s_crow[c];
            }
        }
        if (tid == col) {
#pragma unroll
          for (int c = 0; c < LUP_G; ++c) x[0][c] = s_prow[c];
        }
      }
      const double inv = 1.0 / s_prow[jj];
#pragma unroll
      for (int i = 0; i < LUP_RPT; ++i) {
        const int r = tid + LUP_THREADS * i;
        if (r > col && r < h) {
          const double l = x[i][jj] * inv;
          x[i][jj] = l;
#pragma unroll
          for (int c = jj + 1; c < LUP_G; ++c) x[i][c] -= l * s_prow[c];
        }
      }
    }
    // write the group back to the memory rows of the logical rows as they are now
#pragma unroll
    for (int i = 0; i < LUP_RPT; ++i) {
      const int r = tid + LUP_THREADS * i;
      if (r < h) {
        const int q = s_perm[r];
#pragma unroll
        for (int c = 0; c < LUP_G; ++c)
          if (c < gw) P[q + (int64_t)(g0 + c) * lda] = x[i][c];
      }
    }
    __syncthreads();
  }
  // put the moved rows in place: logical row r <- memory row perm[r], LUP_G
  // columns at a time (all loads of a batch before any of its stores)
  int src[LUP_RPT];
  bool moved = false;
#pragma unroll
  for (int i = 0; i < LUP_RPT; ++i) {
    const int r = tid + LUP_THREADS * i;
    src[i] = r < h ? s_perm[r] : r;
    moved = moved || src[i] != r;
  }
  for (int c0 = 0; c0 < w; c0 += LUP_G) {
    double v[LUP_RPT][LUP_G];
    if (moved) {
#pragma unroll
      for (int i = 0; i < LUP_RPT; ++i) {
        const int r = tid + LUP_THREADS * i;
#pragma unroll
        for (int c = 0; c < LUP_G; ++c)
          v[i][c] = (src[i] != r && c0 + c < w) ? gload(P + src[i] + (int64_t)(c0 + c) * lda)
                                                 : 0.0;
      }
    }
    __syncthreads();
    if (moved) {
#pragma unroll
      for (int i = 0; i < LUP_RPT; ++i) {
        const int r = tid + LUP_THREADS * i;
        if (src[i] != r) {
#pragma unroll
          for (int c = 0; c < LUP_G; ++c)
            if (c0 + c < w) P[r + (int64_t)(c0 + c) * lda] = v[i][c];
        }
      }
    }
  }
  for (int c = tid; c < w; c += LUP_THREADS) d.ipiv[j0 + c] = j0 + s_piv[c];
  if (tid == 0 && info_col != 0 && *d.info == 0) *d.info = info_col;
}

void launch_lu_panel(const MatDesc* d, int nmat, int j0, int nb, int maxrows, hipStream_t s) {
  if (nmat <= 0) return;
  if (maxrows <= LUP_MAXROWS && nb <= 64)
    hipLaunchKernelGGL(lu_panel_reg_kernel, dim3(nmat), dim3(LUP_THREADS), 0, s, d, j0, nb);
  else
    hipLaunchKernelGGL(lu_panel_kernel, dim3(nmat), dim3(256), 0, s, d, j0, nb);
}

// Row swaps of panel [j0, j0+w) applied to every column outside the panel, then
// U12 = L11^-1 A12 for the columns right of the panel (L11 unit lower, in LDS).
// One wave per slab of 64 columns; slab_ptr: per-matrix prefix of slab counts.
__global__ __launch_bounds__(64) void lu_swap_trsm_kernel(const MatDesc* __restrict__ ds,
                                                          const int64_t* __restrict__ slab_ptr,
                                                          int nmat, int j0, int nb) {
  __shared__ double L11[64][65];
  __shared__ double X[64][65];
  int64_t slab = blockIdx.x;
  int id = find_item(slab_ptr, nmat, slab);
  const MatDesc d = ds[id];
  const int m = d.m;
  if (m <= j0) return;
  const int w = min(nb, m - j0);
  const int64_t lda = d.lda;
  double* A = d.A;
  const int lane = threadIdx.x;
  // stage L11 (global loads, which cannot alias the LDS stores, so they stay in flight together)
#pragma unroll 16
  for (int c = 0; c < w; ++c)
    if (lane < w) L11[lane][c] = gload(A + (j0 + lane) + (int64_t)(j0 + c) * lda);
  __syncthreads();
  const int c = (int)(slab - slab_ptr[id]) * 64 + lane;
  if (c >= m || (c >= j0 && c < j0 + w)) return;
  double* col = A + (int64_t)c * lda;
  for (int jj = 0; jj < w; ++jj) {
    int p = d.ipiv[j0 + jj];
    if (p != j0 + jj) {
      double t0 = col[j0 + jj];
      col[j0 + jj] = col[p];
      col[p] = t0;
    }
  }
  if (c >= j0 + w) {
    // forward substitution with the unit lower L11; each lane keeps its column
    // in its own LDS column (no cross-lane traffic, no barrier)
#pragma unroll 16
    for (int r = 0; r < w; ++r) X[r][lane] = gload(col + j0 + r);
    for (int l = 0; l < w; ++l) {
      const double xl = X[l][lane];
      for (int r = l + 1; r < w; ++r) X[r][lane] -= L11[r][l] * xl;
    }
    for (int r = 0; r < w; ++r) col[j0 + r] = X[r][lane];
  }
}

void launch_lu_swap_trsm(const MatDesc* d, const int64_t* slab_ptr, int64_t nslabs, int nmat,
                         int j0, int nb, hipStream_t s) {
  if (nslabs <= 0) return;
  hipLaunchKernelGGL(lu_swap_trsm_kernel, dim3((unsigned)nslabs), dim3(64), 0, s, d, slab_ptr,
                     nmat, j0, nb);
}

// Inverse of the nb x nb diagonal blocks of a triangular factor, for
// triangular solves by blocks (X_j = inv(T_jj) * B_j followed by a GEMM update).
// upper = 0: unit lower (LU's L); upper = 1: upper with its diagonal.
// Output block b of matrix id at out + out_off[id] + b * nb * nb (ld nb),
// zero outside the triangle.  One wave per (matrix, block).
__global__ __launch_bounds__(64) void trinv_diag_kernel(const MatDesc* __restrict__ ds,
                                                        const int64_t* __restrict__ blk_ptr,
                                                        int nmat, int nb, int upper,
                                                        double* __restrict__ out,
                                                        const int64_t* __restrict__ out_off) {
  __shared__ double Tm[64][65];
  __shared__ double X[64][65];
  int64_t blk = blockIdx.x;
  int id = find_item(blk_ptr, nmat, blk);
  const MatDesc d = ds[id];
  const int b = (int)(blk - blk_ptr[id]);
  const int o = b * nb;
  const int w = min(nb, d.m - o);
  if (w <= 0) return;
  const int lane = threadIdx.x;
  for (int c = 0; c < w; ++c)
    for (int r = lane; r < w; r += 64) Tm[r][c] = d.A[(o + r) + (int64_t)(o + c) * d.lda];
  __syncthreads();
  const int j = lane;
  if (j < w) {
    for (int i = 0; i < w; ++i) X[i][j] = 0.0;
    if (!upper) {
      X[j][j] = 1.0;
      for (int i = j + 1; i < w; ++i) {
        double s = 0.0;
        for (int l = j; l < i; ++l) s += Tm[i][l] * X[l][j];
        X[i][j] = -s;
      }
    } else {
      X[j][j] = 1.0 / Tm[j][j];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int l = i + 1; l <= j; ++l) s += Tm[i][l] * X[l][j];
        X[i][j] = -s / Tm[i][i];
      }
    }
  }
  __syncthreads();
  double* dst = out + out_off[id] + (int64_t)b * nb * nb;
  for (int c = 0; c < nb; ++c)
    for (int r = lane; r < nb; r += 64) dst[r + (int64_t)c * nb] = (r < w && c < w) ? X[r][c] : 0.0;
}

void launch_trinv_diag(const MatDesc* d, const int64_t* blk_ptr, int64_t nblk, int nmat, int nb,
                       int upper, double* out, const int64_t* out_off, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(trinv_diag_kernel, dim3((unsigned)nblk), dim3(64), 0, s, d, blk_ptr, nmat,
                     nb, upper, out, out_off);
}

// ---------------------------------------------------------------------------
// Householder panel (LAPACK dgeqrf convention: beta = -sign(alpha) |(alpha, x)|,
// tau = (beta - alpha) / beta, v = x / (alpha - beta), tau = 0 when x = 0).
// One workgroup per matrix factors columns [j0, j0+w) of rows [j0, m), writes
// the explicit reflectors into V (column jj of the panel holds v with a unit
// entry at row j0+jj and zeros above), tau into aux, and the upper-triangular
// block-reflector factor T (H_0 ... H_{w-1} = I - V T V^T) into Tf (nb x nb).
// The trailing columns are updated afterwards by GEMMs.
// ---------------------------------------------------------------------------
template <int NW>
__global__ __launch_bounds__(64 * NW) void qr_panel_kernel(const MatDesc* __restrict__ ds, int j0,
                                                            int nb) {
  constexpr int NT = 64 * NW;
  __shared__ double sh[NW];
  __shared__ double s_tau, s_scale;
  __shared__ double dots[64];
  const MatDesc d = ds[blockIdx.x];
  const int m = d.m, n = d.n;
  if (n <= j0 || m <= j0) return;
  const int w = min(nb, min(n, m) - j0);
  double* A = d.A;
  const int64_t lda = d.lda;
  double* V = d.panel_ws ? d.V : d.V + (int64_t)j0 * m;  // panel reflectors, ld = m
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int jj = 0; jj < w; ++jj) {
    const int col = j0 + jj;
    double* a = A + (int64_t)col * lda;
    double part = 0.0, part1 = 0.0;
    int rr = col + 1 + tid;
    for (; rr + NT < m; rr += 2 * NT) {
      part += a[rr] * a[rr];
      part1 += a[rr + NT] * a[rr + NT];
    }
    for (; rr < m; rr += NT) part += a[rr] * a[rr];
    double xn2 = block_sum<NW>(part + part1, sh);
    double alpha = a[col];
    if (tid == 0) {
      if (xn2 == 0.0) {
        s_tau = 0.0;
        s_scale = 0.0;
        d.aux[col] = 0.0;
      } else {
        double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        s_tau = (beta - alpha) / beta;
        s_scale = 1.0 / (alpha - beta);
        d.aux[col] = s_tau;
        a[col] = beta;
      }
    }
    __syncthreads();
    const double tau = s_tau, scale = s_scale;
    double* v = V + (int64_t)jj * m;
    for (int r = tid; r < m; r += NT) {
      double val;
      if (r < col)
        val = 0.0;
      else if (r == col)
        val = 1.0;
      else {
        val = a[r] * scale;
        a[r] = val;
      }
      v[r] = val;
    }
    __syncthreads();
    if (tau != 0.0) {
      // apply H = I - tau v v^T to the panel columns right of col: one wave per column
      for (int c = col + 1 + wv; c < j0 + w; c += NW) {
        double* ac = A + (int64_t)c * lda;
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
        int r = col + lane;
        for (; r + 192 < m; r += 256) {
          p0 += v[r] * ac[r];
          p1 += v[r + 64] * ac[r + 64];
          p2 += v[r + 128] * ac[r + 128];
          p3 += v[r + 192] * ac[r + 192];
        }
        for (; r < m; r += 64) p0 += v[r] * ac[r];
        double wsum = wave_sum((p0 + p1) + (p2 + p3)) * tau;
        r = col + lane;
        for (; r + 192 < m; r += 256) {
          ac[r] -= wsum * v[r];
          ac[r + 64] -= wsum * v[r + 64];
          ac[r + 128] -= wsum * v[r + 128];
          ac[r + 192] -= wsum * v[r + 192];
        }
        for (; r < m; r += 64) ac[r] -= wsum * v[r];
      }
    }
    __syncthreads();
  }
  // T factor (forward, columnwise): T[jj][jj] = tau_jj,
  // T[0:jj, jj] = -tau_jj T[0:jj, 0:jj] (V[:, 0:jj]^T v_jj)
  double* Tf = d.panel_ws ? d.Tf : d.Tf + (int64_t)(j0 / nb) * nb * nb;
  for (int e = tid; e < nb * nb; e += NT) Tf[e] = 0.0;
  __syncthreads();
  for (int jj = 0; jj < w; ++jj) {
    const double tau = d.aux[j0 + jj];
    const double* vj = V + (int64_t)jj * m;
    for (int l = wv; l < jj; l += NW) {
      const double* vl = V + (int64_t)l * m;
      double p = 0.0, q = 0.0;
      int r = j0 + jj + lane;
      for (; r + 64 < m; r += 128) {
        p += vl[r] * vj[r];
        q += vl[r + 64] * vj[r + 64];
      }
      for (; r < m; r += 64) p += vl[r] * vj[r];
      p = wave_sum(p + q);
      if (lane == 0) dots[l] = p;
    }
    __syncthreads();
    if (tid < jj) {
      double s = 0.0;
      for (int l = tid; l < jj; ++l) s += Tf[tid + (int64_t)l * nb] * dots[l];
      Tf[tid + (int64_t)jj * nb] = -tau * s;
    }
    if (tid == 0) Tf[jj + (int64_t)jj * nb] = tau;
    __syncthreads();
  }
}

// The same Householder panel with each group of QRP_G columns staged in LDS
// (at most QRP_MAXROWS rows from row j0; panel width at most 32), 16 waves.
// Left-looking over the groups: a group is loaded once, the panel's earlier
// reflectors are applied to it as a block (A_g -= V T^T V^T A_g), its columns
// are factored in LDS, and it is written back with its explicit reflectors;
// the T columns of the group come from V^T v.  Products with earlier
// reflectors are taken by one wave per reflector (lanes over rows, four rows
// per lane in flight, then a wave sum); the norm and the dot products of the
// column being factored are taken by all 16 waves.
constexpr int QRP_G = 4;
constexpr int QRP_MAXROWS = 4096;
constexpr int QRP_RPT = QRP_MAXROWS / 1024;  // rows per thread

__global__ __launch_bounds__(1024) void qr_panel_lds_kernel(const MatDesc* __restrict__ ds, int j0,
                                                            int nb) {
  __shared__ double s_a[QRP_G * QRP_MAXROWS];  // group column c at s_a + c * QRP_MAXROWS
  __shared__ double s_y[32 * QRP_G], s_z[32 * QRP_G];
  __shared__ double s_T[32][33];
  __shared__ double s_red[16][QRP_G];  // per-wave partial sums
  __shared__ double s_dot[QRP_G];
  __shared__ double s_sc[3];  // tau, scale, beta of the current column
  const MatDesc d = ds[blockIdx.x];
  const int m = d.m, n = d.n;
  if (n <= j0 || m <= j0) return;
  const int w = min(nb, min(n, m) - j0);
  const int h = m - j0;
  const int64_t lda = d.lda;
  double* P = d.A + j0 + (int64_t)j0 * lda;  // P(r, c) = P[r + c lda]
  double* V = d.panel_ws ? d.V : d.V + (int64_t)j0 * m;  // column c at V + c m, full rows
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < 32 * 33; e += 1024) (&s_T[0][0])[e] = 0.0;
  for (int g0 = 0; g0 < w; g0 += QRP_G) {
    const int gw = min(QRP_G, w - g0);
    {  // all loads of a thread before its LDS stores
      double x[QRP_RPT][QRP_G];
#pragma unroll
      for (int i = 0; i < QRP_RPT; ++i) {
        const int r = tid + 1024 * i;
#pragma unroll
        for (int c = 0; c < QRP_G; ++c)
          x[i][c] = (r < h && c < gw) ? gload(P + r + (int64_t)(g0 + c) * lda) : 0.0;
      }
#pragma unroll
      for (int i = 0; i < QRP_RPT; ++i) {
        const int r = tid + 1024 * i;
#pragma unroll
        for (int c = 0; c < QRP_G; ++c)
          if (r < h && c < gw) s_a[c * QRP_MAXROWS + r] = x[i][c];
      }
    }
    __syncthreads();
    if (g0 > 0) {
      // Y = V_p^T A_g: wave per reflector k (V_p(r, k) = 0 for r < k)
      for (int k = wv; k < g0; k += 16) {
        const double* vk = V + j0 + (int64_t)k * m;
        double acc[QRP_G] = {0.0, 0.0, 0.0, 0.0};
        int r = k + lane;
        for (; r + 192 < h; r += 256) {
          double vv[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) vv[q] = gload(vk + r + 64 * q);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < QRP_G; ++c) acc[c] += vv[q] * s_a[c * QRP_MAXROWS + r + 64 * q];
        }
        for (; r < h; r += 64) {
          const double vv = gload(vk + r);
#pragma unroll
          for (int c = 0; c < QRP_G; ++c) acc[c] += vv * s_a[c * QRP_MAXROWS + r];
        }
#pragma unroll
        for (int c = 0; c < QRP_G; ++c) {
          const double t = wave_sum(acc[c]);
          if (lane == 0) s_y[k * QRP_G + c] = t;
        }
      }
      __syncthreads();
      // Z = T^T Y
      if (tid < g0 * QRP_G) {
        const int k = tid / QRP_G, c = tid % QRP_G;
        double z = 0.0;
        for (int l = 0; l <= k; ++l) z += s_T[l][k] * s_y[l * QRP_G + c];
        s_z[tid] = z;
      }
      __syncthreads();
      // A_g -= V_p Z, thread per row, four reflectors per batch of loads
      for (int r = tid; r < h; r += 1024) {
        double acc[QRP_G] = {0.0, 0.0, 0.0, 0.0};
        const int kend = min(g0, r + 1);
        const double* vr = V + j0 + r;
        int k = 0;
        for (; k + 3 < kend; k += 4) {
          double vv[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) vv[q] = gload(vr + (int64_t)(k + q) * m);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < QRP_G; ++c) acc[c] += vv[q] * s_z[(k + q) * QRP_G + c];
        }
        for (; k < kend; ++k) {
          const double vv = gload(vr + (int64_t)k * m);
#pragma unroll
          for (int c = 0; c < QRP_G; ++c) acc[c] += vv * s_z[k * QRP_G + c];
        }
#pragma unroll
        for (int c = 0; c < QRP_G; ++c)
          if (c < gw) s_a[c * QRP_MAXROWS + r] -= acc[c];
      }
      __syncthreads();
    }
    // factor the group's columns
    for (int jj = 0; jj < gw; ++jj) {
      const int col = g0 + jj;
      double* a = s_a + jj * QRP_MAXROWS;
      {
        double part = 0.0;
        for (int r = col + 1 + tid; r < h; r += 1024) part += a[r] * a[r];
        part = wave_sum(part);
        if (lane == 0) s_red[wv][0] = part;
      }
      __syncthreads();
      if (tid == 0) {
        double xn2 = 0.0;
        for (int q = 0; q < 16; ++q) xn2 += s_red[q][0];
        const double alpha = a[col];
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (xn2 != 0.0) {
          beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        s_sc[0] = tau;
        s_sc[1] = scale;
        s_sc[2] = beta;
        s_T[col][col] = tau;
        d.aux[j0 + col] = tau;
      }
      __syncthreads();
      const double tau = s_sc[0], scale = s_sc[1];
      if (tau != 0.0) {
        for (int r = col + 1 + tid; r < h; r += 1024) a[r] *= scale;
        if (tid == 0) a[col] = s_sc[2];
      }
      __syncthreads();
      if (tau != 0.0 && jj + 1 < gw) {
        // dot_c = a_c(col) + sum_{r > col} v(r) a_c(r) for the later columns
        double pd[QRP_G] = {0.0, 0.0, 0.0, 0.0};
        for (int r = col + 1 + tid; r < h; r += 1024) {
          const double vr = a[r];
#pragma unroll
          for (int c = 0; c < QRP_G; ++c)
            if (c > jj && c < gw) pd[c] += vr * s_a[c * QRP_MAXROWS + r];
        }
        for (int c = jj + 1; c < gw; ++c) {
          const double t = wave_sum(pd[c]);
          if (lane == 0) s_red[wv][c] = t;
        }
        __syncthreads();
        if (tid > jj && tid < gw) {
          double dsum = 0.0;
          for (int q = 0; q < 16; ++q) dsum += s_red[q][tid];
          s_dot[tid] = dsum + s_a[tid * QRP_MAXROWS + col];
        }
        __syncthreads();
        for (int r = col + tid; r < h; r += 1024) {
          const double vr = r == col ? 1.0 : a[r];
          for (int c = jj + 1; c < gw; ++c) s_a[c * QRP_MAXROWS + r] -= tau * s_dot[c] * vr;
        }
        __syncthreads();
      }
    }
    // write the group back (R above and on the diagonal, v below) and its
    // explicit reflectors (zero above the unit entry, full rows)
    for (int c = 0; c < gw; ++c) {
      const int col = g0 + c;
      const double* ac = s_a + c * QRP_MAXROWS;
      double* vc = V + (int64_t)col * m;
      for (int r = tid; r < h; r += 1024) {
        P[r + (int64_t)col * lda] = ac[r];
        vc[j0 + r] = r < col ? 0.0 : (r == col ? 1.0 : ac[r]);
      }
      for (int r = tid; r < j0; r += 1024) vc[r] = 0.0;
    }
    // T columns of the group: T(0:k, k) = -tau_k T(0:k, 0:k) (V(:, 0:k)^T v_k);
    // wave per earlier column l, the group's own columns from LDS
    const int kmax = g0 + gw - 1;
    for (int l = wv; l < kmax; l += 16) {
      double acc[QRP_G] = {0.0, 0.0, 0.0, 0.0};
      const bool own = l >= g0;
      const double* vg = V + j0 + (int64_t)l * m;
      const double* vs = s_a + (own ? l - g0 : 0) * QRP_MAXROWS;
      int r = l + 1 + lane;
      for (; r + 192 < h; r += 256) {
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = own ? vs[r + 64 * q] : gload(vg + r + 64 * q);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rq = r + 64 * q;
#pragma unroll
          for (int c = 0; c < QRP_G; ++c) {
            const int k = g0 + c;
            if (c < gw && k > l && rq >= k)
              acc[c] += x[q] * (rq == k ? 1.0 : s_a[c * QRP_MAXROWS + rq]);
          }
        }
      }
      for (; r < h; r += 64) {
        const double x = own ? vs[r] : gload(vg + r);
#pragma unroll
        for (int c = 0; c < QRP_G; ++c) {
          const int k = g0 + c;
          if (c < gw && k > l && r >= k) acc[c] += x * (r == k ? 1.0 : s_a[c * QRP_MAXROWS + r]);
        }
      }
      // the unit entry of v_l at row l meets v_k(l) = 0 for k > l
#pragma unroll
      for (int c = 0; c < QRP_G; ++c) {
        const double t = wave_sum(acc[c]);
        if (lane == 0) s_y[l * QRP_G + c] = t;
      }
    }
    __syncthreads();
    for (int c = 0; c < gw; ++c) {  // column k needs T(0:k, 0:k): one column at a time
      const int k = g0 + c;
      if (tid < k) {
        double acc = 0.0;
        for (int l2 = tid; l2 < k; ++l2) acc += s_T[tid][l2] * s_y[l2 * QRP_G + c];
        s_T[tid][k] = -s_T[k][k] * acc;
      }
      __syncthreads();
    }
  }
  double* Tf = d.panel_ws ? d.Tf : d.Tf + (int64_t)(j0 / nb) * nb * nb;
  for (int e = tid; e < nb * nb; e += 1024) {
    const int l = e % nb, k = e / nb;
    Tf[e] = (l < w && k < w && l <= k) ? s_T[l][k] : 0.0;
  }
}

void launch_qr_panel(const MatDesc* d, int nmat, int j0, int nb, int maxrows, hipStream_t s) {
  if (nmat <= 0) return;
  if (maxrows <= QRP_MAXROWS && nb <= 32)
    hipLaunchKernelGGL(qr_panel_lds_kernel, dim3(nmat), dim3(1024), 0, s, d, j0, nb);
  else  // 16 waves: each step updates 16 trailing panel columns at once
    hipLaunchKernelGGL(qr_panel_kernel<16>, dim3(nmat), dim3(1024), 0, s, d, j0, nb);
}


// ---------------------------------------------------------------------------
// Column-pivoted Householder QR for the row interpolative decomposition
// (Sec. II-A: the shared basis from a column-pivoted QR), for matrices of at
// most PQ_MAXR rows and PQ_MAXR columns.  One workgroup of 16 waves per
// matrix; the matrix stays in global memory and every column is read by one
// wave (lanes over rows, coalesced), held in registers while it is updated.
// At step t the column of largest remaining norm (norms recomputed exactly
// after every step, lowest index on ties) is moved to position t; the step is
// taken only while that norm exceeds tol * |R_00| and t < cap.  Afterwards
// the leading k rows of R give E = R11^-1 R12, written over R12.
// ---------------------------------------------------------------------------
constexpr int PQ_MAXR = 512;
constexpr int PQ_REG = PQ_MAXR / 64;  // column values per lane
constexpr int PQ_WAVES = 16;

__global__ __launch_bounds__(1024) void pivqr_kernel(const PivQrItem* __restrict__ items) {
  __shared__ double s_nrm[PQ_MAXR];
  __shared__ int s_piv[PQ_MAXR];
  __shared__ double s_v[PQ_MAXR];
  __shared__ double s_wv[PQ_WAVES];
  __shared__ int s_wi[PQ_WAVES];
  __shared__ double s_tau;
  const PivQrItem it = items[blockIdx.x];
  const int m = it.m, n = it.n;
  double* A = it.A;
  const int64_t lda = it.lda;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int c = wv; c < n; c += PQ_WAVES) {
    const double* ac = A + (int64_t)c * lda;
    double sq = 0.0;
    for (int r = lane; r < m; r += 64) sq += ac[r] * ac[r];
    sq = wave_sum(sq);
    if (lane == 0) s_nrm[c] = sqrt(sq);
  }
  for (int c = tid; c < n; c += 64 * PQ_WAVES) s_piv[c] = c;
  for (int t = tid; t < min(m, n); t += 64 * PQ_WAVES) it.diag[t] = 0.0;
  __syncthreads();
  const int steps = min(m, min(n, it.cap));
  double thr = 0.0;
  int k = 0;
  for (int t = 0; t < steps; ++t) {
    // pivot: largest norm among columns t..n-1, lowest index on ties
    double best = -1.0;
    int bi = n;
    for (int c = t + tid; c < n; c += 64 * PQ_WAVES) {
      const double v = s_nrm[c];
      if (v > best) {
        best = v;
        bi = c;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double vo = __shfl_xor(best, off, 64);
      const int io = __shfl_xor(bi, off, 64);
      if (vo > best || (vo == best && io < bi)) {
        best = vo;
        bi = io;
      }
    }
    if (lane == 0) {
      s_wv[wv] = best;
      s_wi[wv] = bi;
    }
    __syncthreads();
    best = s_wv[0];
    bi = s_wi[0];
    for (int w = 1; w < PQ_WAVES; ++w) {
      const double vo = s_wv[w];
      const int io = s_wi[w];
      if (vo > best || (vo == best && io < bi)) {
        best = vo;
        bi = io;
      }
    }
    const double pn = best;
    const int p = bi;
    if (t == 0) thr = it.tol * pn;
    if (!(pn > thr) || !(pn > 0.0) || p >= n) break;  // same decision in every thread
    // swap columns t and p (all rows), norms and pivots
    double* at = A + (int64_t)t * lda;
    if (p != t) {
      double* ap = A + (int64_t)p * lda;
      for (int r = tid; r < m; r += 64 * PQ_WAVES) {
        const double x = at[r];
        at[r] = ap[r];
        ap[r] = x;
      }
      if (tid == 0) {
        const double x = s_nrm[t];
        s_nrm[t] = s_nrm[p];
        s_nrm[p] = x;
        const int q = s_piv[t];
        s_piv[t] = s_piv[p];
        s_piv[p] = q;
      }
    }
    __syncthreads();
    // reflector from column t, rows t..m-1 (first wave); v(t) = 1
    if (wv == 0) {
      double x[PQ_REG];
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) {
        const int r = t + 1 + lane + 64 * q;
        x[q] = r < m ? at[r] : 0.0;
        part += x[q] * x[q];
      }
      const double xn2 = wave_sum(part);
      const double alpha = at[t];
      double tau = 0.0, scale = 0.0;
      if (xn2 != 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        if (lane == 0) at[t] = beta;
      }
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) {
        const int r = t + 1 + lane + 64 * q;
        if (r < m) {
          const double v = x[q] * scale;
          if (tau != 0.0) at[r] = v;
          s_v[r] = v;
        }
      }
      if (lane == 0) {
        s_v[t] = 1.0;
        s_tau = tau;
        it.diag[t] = pn;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    // apply I - tau v v^T to columns c > t and recompute their norms below row
    // t; the wave's next column is loaded while the current one is processed
    double x[PQ_REG];
    {
      const int c = t + 1 + wv;
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) {
        const int r = t + lane + 64 * q;
        x[q] = (c < n && r < m) ? gload(A + (int64_t)c * lda + r) : 0.0;
      }
    }
    for (int c = t + 1 + wv; c < n; c += PQ_WAVES) {
      double* ac = A + (int64_t)c * lda;
      double xn[PQ_REG];
      const int cn = c + PQ_WAVES;
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) {
        const int r = t + lane + 64 * q;
        xn[q] = (cn < n && r < m) ? gload(A + (int64_t)cn * lda + r) : 0.0;
      }
      if (tau != 0.0) {
        double dot = 0.0;
#pragma unroll
        for (int q = 0; q < PQ_REG; ++q) {
          const int r = t + lane + 64 * q;
          if (r < m) dot += s_v[r] * x[q];
        }
        const double w = wave_sum(dot) * tau;
#pragma unroll
        for (int q = 0; q < PQ_REG; ++q) {
          const int r = t + lane + 64 * q;
          if (r < m) {
            x[q] -= w * s_v[r];
            ac[r] = x[q];
          }
        }
      }
      double sq = 0.0;
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) {
        const int r = t + lane + 64 * q;
        if (r > t && r < m) sq += x[q] * x[q];
      }
      sq = wave_sum(sq);
      if (lane == 0) s_nrm[c] = sqrt(sq);
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) x[q] = xn[q];
    }
    k = t + 1;
    __syncthreads();
  }
  if (tid == 0) *it.kout = k;
  for (int c = tid; c < n; c += 64 * PQ_WAVES) it.piv[c] = s_piv[c];
  // E = R11^-1 R12 over R12 (rows 0..k-1, columns k..n-1): each wave takes
  // PQ_NC columns at a time and solves them side by side, sharing the loads of
  // R (back substitution with the columns in registers: row r in lane r % 64,
  // register r / 64)
  constexpr int PQ_NC = 4;
  for (int c0 = k + wv; c0 < n; c0 += PQ_WAVES * PQ_NC) {
    double x[PQ_NC][PQ_REG];
#pragma unroll
    for (int j = 0; j < PQ_NC; ++j) {
      const int c = c0 + PQ_WAVES * j;
#pragma unroll
      for (int q = 0; q < PQ_REG; ++q) {
        const int r = lane + 64 * q;
        x[j][q] = (c < n && r < k) ? gload(A + (int64_t)c * lda + r) : 0.0;
      }
    }
#pragma unroll
    for (int q = PQ_REG - 1; q >= 0; --q) {
      const int top = min(64, k - 64 * q);  // rows of this register block
      for (int ii = top - 1; ii >= 0; --ii) {
        const int i = 64 * q + ii;
        const double* ri = A + (int64_t)i * lda;  // column i of R
        const double dg = gload(ri + i);
        double rv[PQ_REG];
#pragma unroll
        for (int q2 = 0; q2 <= q; ++q2) {
          const int r = lane + 64 * q2;
          rv[q2] = r < i ? gload(ri + r) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < PQ_NC; ++j) {
          const double xi = __shfl(x[j][q], ii, 64) / dg;
          if (lane == ii) x[j][q] = xi;
#pragma unroll
          for (int q2 = 0; q2 <= q; ++q2) {
            const int r = lane + 64 * q2;
            if (r < i) x[j][q2] -= xi * rv[q2];
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PQ_NC; ++j) {
      const int c = c0 + PQ_WAVES * j;
      if (c < n) {
        double* ac = A + (int64_t)c * lda;
#pragma unroll
        for (int q = 0; q < PQ_REG; ++q) {
          const int r = lane + 64 * q;
          if (r < k) ac[r] = x[j][q];
        }
      }
    }
  }
}

void launch_pivqr(const PivQrItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(pivqr_kernel, dim3(nitems), dim3(64 * PQ_WAVES), 0, s, items);
}


// ---------------------------------------------------------------------------
// Column-pivoted QR of large matrices over many workgroups.  Same decisions as
// the one-workgroup kernel (largest exact remaining norm, lowest index on ties,
// continue while it exceeds tol |R_00| and the cap allows), one step per pair
// of launches: pick (one workgroup per matrix: pivot search, column swap,
// reflector) and apply (one workgroup per trailing column: reflector update
// and exact norm of the column below the new row).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pivqr_init_kernel(const PivQrState* __restrict__ sts,
                                                         const int64_t* __restrict__ slab_ptr,
                                                         int n) {
  int64_t slab = blockIdx.x;
  int id = find_item(slab_ptr, n, slab);
  const PivQrState st = sts[id];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = (int)(slab - slab_ptr[id]) * 4 + w;
  if (c == 0 && threadIdx.x == 0) {
    st.flags[0] = 0;
    st.flags[1] = 0;
    st.scal[0] = 0.0;
    st.scal[1] = 0.0;
  }
  if (c >= st.n) return;
  const double* ac = st.A + (int64_t)c * st.lda;
  double p = 0.0;
  for (int r = lane; r < st.m; r += 64) p += ac[r] * ac[r];
  p = wave_sum(p);
  if (lane == 0) {
    st.nrm[c] = sqrt(p);
    st.piv[c] = c;
  }
}

void launch_pivqr_init(const PivQrState* st, const int64_t* slab_ptr, int64_t nslabs, int n,
                       hipStream_t s) {
  if (nslabs <= 0) return;
  hipLaunchKernelGGL(pivqr_init_kernel, dim3((unsigned)nslabs), dim3(256), 0, s, st, slab_ptr, n);
}

// One pivot step of a large box (one 1024-thread workgroup per box): pick the
// column of largest norm among t..n-1 (lowest index on ties), swap it into
// position t, form the reflector from its rows t..m-1 (scaled in place, R_tt
// written), and leave tau and the rank so far for the apply kernel.
__global__ __launch_bounds__(1024) void pivqr_pick_kernel(const PivQrState* __restrict__ sts,
                                                          int t) {
  __shared__ double s_wv[16];
  __shared__ int s_wi[16];
  __shared__ double sh[16];
  const PivQrState st = sts[blockIdx.x];
  const int m = st.m, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ncol = st.n;
  // the stop flag, the threshold and the first PK_NV candidate norms of this
  // thread are loaded together (reading them is harmless for a stopped box)
  constexpr int PK_NV = 4;
  const int stopped = st.flags[0];
  const double thr_prev = st.scal[1];
  double nv[PK_NV];
#pragma unroll
  for (int i = 0; i < PK_NV; ++i) {
    const int c = t + tid + 1024 * i;
    nv[i] = c < ncol ? st.nrm[c] : -1.0;
  }
  if (stopped) return;
  if (t >= st.cap) {
    if (tid == 0) st.flags[0] = 1;
    return;
  }
  double best = -1.0;
  int bi = ncol;
#pragma unroll
  for (int i = 0; i < PK_NV; ++i) {
    const int c = t + tid + 1024 * i;
    if (c < ncol && nv[i] > best) {
      best = nv[i];
      bi = c;
    }
  }
  for (int c = t + tid + 1024 * PK_NV; c < ncol; c += 1024) {
    const double v = st.nrm[c];
    if (v > best) {
      best = v;
      bi = c;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double vo = __shfl_xor(best, off, 64);
    const int io = __shfl_xor(bi, off, 64);
    if (vo > best || (vo == best && io < bi)) {
      best = vo;
      bi = io;
    }
  }
  if (lane == 0) {
    s_wv[wv] = best;
    s_wi[wv] = bi;
  }
  __syncthreads();
  best = s_wv[0];
  bi = s_wi[0];
  for (int q = 1; q < 16; ++q) {
    const double vo = s_wv[q];
    const int io = s_wi[q];
    if (vo > best || (vo == best && io < bi)) {
      best = vo;
      bi = io;
    }
  }
  const double pn = best;
  const int p = bi;
  const double thr = (t == 0) ? st.tol * pn : thr_prev;
  if (!(pn > thr) || !(pn > 0.0) || p >= ncol) {  // same decision in every thread
    if (tid == 0) st.flags[0] = 1;
    return;
  }
  double* A = st.A;
  const int64_t lda = st.lda;
  double* at = A + (int64_t)t * lda;
  double* ap = A + (int64_t)p * lda;
  // Swap columns t and p.  Rows above t only move; rows below t are taken in
  // the same thread / row assignment as the sum of squares of the reflector,
  // their loads are issued together and their values stay in registers for
  // the scaling (the first PK_KEEP * 1024 of them).
  constexpr int PK_KEEP = 4;
  if (p != t) {
    for (int r = tid; r <= t && r < m; r += 1024) {
      const double x = gload(at + r), y = gload(ap + r);
      at[r] = y;
      ap[r] = x;
    }
  }
  double keep[PK_KEEP];
  double part = 0.0;
#pragma unroll
  for (int j = 0; j < PK_KEEP; ++j) {
    const int r = t + 1 + tid + 1024 * j;
    keep[j] = r < m ? gload(ap + r) : 0.0;  // the new column t (column p)
  }
  if (p != t) {
    double old[PK_KEEP];
#pragma unroll
    for (int j = 0; j < PK_KEEP; ++j) {
      const int r = t + 1 + tid + 1024 * j;
      old[j] = r < m ? gload(at + r) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < PK_KEEP; ++j) {
      const int r = t + 1 + tid + 1024 * j;
      if (r < m) {
        at[r] = keep[j];
        ap[r] = old[j];
      }
    }
  }
  // explicit fused multiply-adds in row order: contraction of a sum of
  // products may otherwise fuse either product
#pragma unroll
  for (int j = 0; j < PK_KEEP; ++j) part = fma(keep[j], keep[j], part);
  for (int r = t + 1 + tid + 1024 * PK_KEEP; r < m; r += 1024) {
    const double y = gload(ap + r);
    if (p != t) {
      const double x = gload(at + r);
      at[r] = y;
      ap[r] = x;
    }
    part = fma(y, y, part);
  }
  if (tid == 0 && p != t) {
    const double x = st.nrm[t];
    st.nrm[t] = st.nrm[p];
    st.nrm[p] = x;
    const int q = st.piv[t];
    st.piv[t] = st.piv[p];
    st.piv[p] = q;
  }
  const double xn2 = block_sum<16>(part, sh);  // its barriers also order the swap above
  const double alpha = at[t];
  double tau = 0.0, scale = 0.0;
  if (xn2 != 0.0) {
    const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  __syncthreads();  // every thread has read alpha before thread 0 overwrites it
  if (tau != 0.0) {
#pragma unroll
    for (int j = 0; j < PK_KEEP; ++j) {
      const int r = t + 1 + tid + 1024 * j;
      if (r < m) at[r] = keep[j] * scale;
    }
    for (int r = t + 1 + tid + 1024 * PK_KEEP; r < m; r += 1024) at[r] *= scale;
  }
  if (tid == 0) {
    if (tau != 0.0) at[t] = -copysign(sqrt(alpha * alpha + xn2), alpha);
    st.scal[0] = tau;
    if (t == 0) st.scal[1] = thr;
    st.flags[1] = t + 1;
  }
}

void launch_pivqr_pick(const PivQrState* st, int n, int t, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(pivqr_pick_kernel, dim3(n), dim3(1024), 0, s, st, t);
}

// Apply step: one PA_THREADS-thread workgroup per trailing column.  Workgroup
// b * per + q (per = widest trailing width) takes column t + 1 + q of matrix b.
// The column's rows below t stay in registers (PA_RPT per thread, the rest are
// read again) between the dot product with the reflector and the update, and
// the exact norm of the updated rows below t comes from the same registers.
constexpr int PA_THREADS = 256;
constexpr int PA_RPT = 8;

__global__ __launch_bounds__(PA_THREADS) void pivqr_apply_kernel(
    const PivQrState* __restrict__ sts, int per, int t) {
  __shared__ double sh[PA_THREADS / 64];
  const int b = (int)(blockIdx.x / (unsigned)per);
  const int q = (int)(blockIdx.x - (unsigned)b * (unsigned)per);
  const PivQrState st = sts[b];
  // stopped before or at this step: flags[1] is the rank, equal to t + 1 only
  // when step t was taken
  if (st.flags[1] != t + 1) return;
  const int c = t + 1 + q;
  if (c >= st.n) return;
  const int tid = threadIdx.x;
  const double tau = st.scal[0];
  const int m = st.m;
  const double* v = st.A + (int64_t)t * st.lda;
  double* ac = st.A + (int64_t)c * st.lda;
  const int r0 = t + 1 + tid;
  double x[PA_RPT];
#pragma unroll
  for (int j = 0; j < PA_RPT; ++j) {
    const int r = r0 + PA_THREADS * j;
    x[j] = r < m ? gload(ac + r) : 0.0;
  }
  if (tau != 0.0) {
    double vv[PA_RPT];
#pragma unroll
    for (int j = 0; j < PA_RPT; ++j) {
      const int r = r0 + PA_THREADS * j;
      vv[j] = r < m ? gload(v + r) : 0.0;
    }
    double p = 0.0;
#pragma unroll
    for (int j = 0; j < PA_RPT; ++j) p = fma(vv[j], x[j], p);
    for (int r = r0 + PA_THREADS * PA_RPT; r < m; r += PA_THREADS)
      p = fma(gload(v + r), gload(ac + r), p);
    const double dsum = block_sum<PA_THREADS / 64>(p, sh);
    const double wsum = (gload(ac + t) + dsum) * tau;
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < PA_RPT; ++j) {
      const int r = r0 + PA_THREADS * j;
      if (r < m) {
        const double y = x[j] - wsum * vv[j];
        __builtin_nontemporal_store(y, ac + r);
        s2 = fma(y, y, s2);
      }
    }
    for (int r = r0 + PA_THREADS * PA_RPT; r < m; r += PA_THREADS) {
      const double y = gload(ac + r) - wsum * gload(v + r);
      __builtin_nontemporal_store(y, ac + r);
      s2 = fma(y, y, s2);
    }
    s2 = block_sum<PA_THREADS / 64>(s2, sh);  // its first barrier: every thread has read ac[t]
    if (tid == 0) {
      ac[t] -= wsum;
      st.nrm[c] = sqrt(s2);
    }
  } else {
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < PA_RPT; ++j) s2 = fma(x[j], x[j], s2);
    for (int r = r0 + PA_THREADS * PA_RPT; r < m; r += PA_THREADS) {
      const double y = gload(ac + r);
      s2 = fma(y, y, s2);
    }
    s2 = block_sum<PA_THREADS / 64>(s2, sh);
    if (tid == 0) st.nrm[c] = sqrt(s2);
  }
}

void launch_pivqr_apply(const PivQrState* st, int n, int maxcols, int t, hipStream_t s) {
  const int64_t per = (int64_t)maxcols - t - 1;  // widest trailing width
  if (n <= 0 || per <= 0) return;
  hipLaunchKernelGGL(pivqr_apply_kernel, dim3((unsigned)(per * n)), dim3(PA_THREADS), 0, s, st,
                     (int)per, t);
}

// ---------------------------------------------------------------------------
// Batched 2-D copy / scaled accumulate (merges of skeleton blocks into the
// parent's dense blocks, quadrant extraction, packing).  Tile 64 x 64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void copy_kernel(const CopyItem* __restrict__ items,
                                                   const int64_t* __restrict__ tile_ptr,
                                                   int nitems, double alpha, double beta) {
  int64_t tile = blockIdx.x;
  int id = find_item(tile_ptr, nitems, tile);
  const CopyItem it = items[id];
  int64_t local = tile - tile_ptr[id];
  int tm = (it.rows + 63) >> 6;
  int i = (int)(local % tm) * 64 + (threadIdx.x & 63);
  int j0 = (int)(local / tm) * 64 + (threadIdx.x >> 6);
  if (i >= it.rows) return;
  for (int q = 0; q < 16; ++q) {
    int j = j0 + 4 * q;
    if (j >= it.cols) break;
    double v = it.trans ? it.src[j + (int64_t)i * it.lds] : it.src[i + (int64_t)j * it.lds];
    double* o = it.dst + i + (int64_t)j * it.ldd;
    double r = alpha * v;
    if (beta != 0.0) r += beta * (*o);
    *o = r;
  }
}

void launch_copy(const CopyItem* items, const int64_t* tile_ptr, int64_t ntiles, int nitems,
                 double alpha, double beta, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, items, tile_ptr,
                     nitems, alpha, beta);
}

// ---------------------------------------------------------------------------
// Exact matvec y = A x with A generated on the fly in float64 (residuals of the
// iterative refinement).  One thread per row; source points staged in LDS.
// ---------------------------------------------------------------------------
// 1/r to full double precision: the hardware reciprocal square root y (about 23
// correct bits, so e = 1 - r2 y^2 is below 2^-22) corrected by the series
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3): y (1 + e (1/2 + 3e/8)), whose
// truncation error is of order e^3 (below 2^-66).
__device__ __forceinline__ double inv_sqrt(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2 * y, y, 1.0);
  return fma(y, e * fma(0.375, e, 0.5), y);
}

// Sources t < cnt of the staged tile against the thread's two targets.  SELF:
// the tile holds target indices, whose self term (r^2 = 0) is excluded by a
// select; other tiles have r^2 > 0 throughout, since the points are distinct
// (a factorization rejects coinciding points).
template <int NR, int KIND, bool SELF>
__device__ __forceinline__ void matvec_tile(const double (*sp)[256], const double (*sx)[256],
                                            int cnt, const double* p0, const double* p1,
                                            const KernelFn& kf, double* a0, double* a1) {
  for (int t = 0; t < cnt; ++t) {
    const double sx0 = sp[0][t], sy0 = sp[1][t], sz0 = sp[2][t];
    const double dx0 = p0[0] - sx0, dy0 = p0[1] - sy0, dz0 = p0[2] - sz0;
    const double q0 = fma(dx0, dx0, fma(dy0, dy0, dz0 * dz0));
    const double dx1 = p1[0] - sx0, dy1 = p1[1] - sy0, dz1 = p1[2] - sz0;
    const double q1 = fma(dx1, dx1, fma(dy1, dy1, dz1 * dz1));
    double k0 = inv_sqrt(q0), k1 = inv_sqrt(q1);
    if (KIND == 1) {
      k0 *= exp(-kf.alpha * (q0 * k0));
      k1 *= exp(-kf.alpha * (q1 * k1));
    } else if (KIND == 2) {
      k0 *= exp(fma(kf.b[0], dx0, fma(kf.b[1], dy0, kf.b[2] * dz0)) - kf.alpha * (q0 * k0));
      k1 *= exp(fma(kf.b[0], dx1, fma(kf.b[1], dy1, kf.b[2] * dz1)) - kf.alpha * (q1 * k1));
    }
    if (SELF) {
      k0 = q0 > 0.0 ? k0 : 0.0;
      k1 = q1 > 0.0 ? k1 : 0.0;
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const double xs = sx[c][t];
      a0[c] = fma(k0, xs, a0[c]);
      a1[c] = fma(k1, xs, a1[c]);
    }
  }
}

// Exact y = A x with the matrix generated on the fly.  Each thread owns two
// target points (i and i + 256) and runs over the sources [js, je) staged in
// LDS, 256 at a time; only the tiles that hold target indices of the
// workgroup test for the self term.  The kernel kind is a template parameter
// (no branch in the inner loop).  With one source range the result
// y = diag x + sum is written directly; otherwise the range blockIdx.y writes
// its partial sums to part and matvec_reduce_kernel adds them in a fixed
// order.
template <int NR, int KIND>
__global__ __launch_bounds__(256) void matvec_kernel(const double* __restrict__ pts, int64_t n,
                                                     KernelFn kf, const double* __restrict__ x,
                                                     int64_t ldx, double* __restrict__ y,
                                                     int64_t ldy, double* __restrict__ part,
                                                     int64_t chunk) {
  __shared__ double sp[3][256];
  __shared__ double sx[NR][256];
  const int64_t i0 = (int64_t)blockIdx.x * 512 + threadIdx.x;
  const int64_t i1 = i0 + 256;
  const int64_t js = (int64_t)blockIdx.y * chunk, je = min(n, js + chunk);
  double p0[3] = {0, 0, 0}, p1[3] = {0, 0, 0};
  if (i0 < n)
    for (int d = 0; d < 3; ++d) p0[d] = pts[3 * i0 + d];
  if (i1 < n)
    for (int d = 0; d < 3; ++d) p1[d] = pts[3 * i1 + d];
  double a0[NR], a1[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) a0[c] = a1[c] = 0.0;
  for (int64_t j0 = js; j0 < je; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    __syncthreads();
    if (j < je) {
      for (int d = 0; d < 3; ++d) sp[d][threadIdx.x] = pts[3 * j + d];
#pragma unroll
      for (int c = 0; c < NR; ++c) sx[c][threadIdx.x] = x[j + c * ldx];
    } else {
      // padding entries (never read: the loop below stops at the last source)
      for (int d = 0; d < 3; ++d) sp[d][threadIdx.x] = 0.0;
#pragma unroll
      for (int c = 0; c < NR; ++c) sx[c][threadIdx.x] = 0.0;
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)256, je - j0);
    const int64_t ib = (int64_t)blockIdx.x * 512;  // targets [ib, ib + 512)
    if (j0 < ib + 512 && j0 + 256 > ib)
      matvec_tile<NR, KIND, true>(sp, sx, cnt, p0, p1, kf, a0, a1);
    else
      matvec_tile<NR, KIND, false>(sp, sx, cnt, p0, p1, kf, a0, a1);
  }
  if (part == nullptr) {
    if (i0 < n) {
#pragma unroll
      for (int c = 0; c < NR; ++c) y[i0 + c * ldy] = fma(kf.diag, x[i0 + c * ldx], a0[c]);
    }
    if (i1 < n) {
#pragma unroll
      for (int c = 0; c < NR; ++c) y[i1 + c * ldy] = fma(kf.diag, x[i1 + c * ldx], a1[c]);
    }
  } else {
    double* pp = part + (int64_t)blockIdx.y * NR * n;
    if (i0 < n) {
#pragma unroll
      for (int c = 0; c < NR; ++c) pp[i0 + c * n] = a0[c];
    }
    if (i1 < n) {
#pragma unroll
      for (int c = 0; c < NR; ++c) pp[i1 + c * n] = a1[c];
    }
  }
}

// Matrix-core form of the exact matvec for blocks of 4 or 8 columns.  The
// vector units evaluate one kernel entry per lane and the FP64 4x4x4 MFMA
// (four independent 4x4 blocks per wave) multiplies it into the columns, so
// the 8 multiply-adds per entry leave the vector pipe.  Operand layout of that
// instruction, lane l = 16 q + 4 b + p (q, b, p < 4):
//   A: block b, row p, k q     B: block b, column p, k q
//   D: block b, column p, row q
// A wave owns G groups of 16 targets; within a group, block b row p is target
// 4 b + p, so lane l evaluates K(target l & 15, source q) and all four blocks
// share the B operand x(source q, column p).  One step (a "chunk") consumes
// four staged sources.  Targets beyond n sit at (+1e30, 0, 0) and padding
// sources at (-1e30, 0, 0) with x = 0: every entry stays finite and only rows
// that are never written see them.  Accumulation order: per target, the
// sources of a chunk are summed by the instruction, chunks in ascending
// source order.
constexpr int MVM_G = 8;  // target groups of 16 per wave: 512 targets per workgroup

template <int KIND, bool SELF, int NB>
__device__ __forceinline__ void matvec_mfma_tile(const double (*sp)[4], const double (*sx)[8],
                                                 int cnt, const double* tx, const double* ty,
                                                 const double* tz, const KernelFn& kf,
                                                 double (*acc)[2]) {
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, col = lane & 3;
  for (int c0 = 0; c0 < cnt; c0 += 4) {
    const int src = c0 + q;
    const double sx0 = sp[src][0], sy0 = sp[src][1], sz0 = sp[src][2];
    const double b0 = sx[src][col];
    const double b1 = NB == 2 ? sx[src][4 + col] : 0.0;
#pragma unroll
    for (int g = 0; g < MVM_G; ++g) {
      const double dx = tx[g] - sx0, dy = ty[g] - sy0, dz = tz[g] - sz0;
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      double k = inv_sqrt(r2);
      if (KIND == 1)
        k *= exp(-kf.alpha * (r2 * k));
      else if (KIND == 2)
        k *= exp(fma(kf.b[0], dx, fma(kf.b[1], dy, kf.b[2] * dz)) - kf.alpha * (r2 * k));
      if (SELF) k = r2 > 0.0 ? k : 0.0;
      acc[g][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(k, b0, acc[g][0], 0, 0, 0);
      if (NB == 2) acc[g][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(k, b1, acc[g][1], 0, 0, 0);
    }
  }
}

template <int KIND, int NB>
__global__ __launch_bounds__(256) void matvec_mfma_kernel(const double* __restrict__ pts,
                                                          int64_t n, KernelFn kf,
                                                          const double* __restrict__ x,
                                                          int64_t ldx, double* __restrict__ y,
                                                          int64_t ldy, double* __restrict__ part,
                                                          int64_t chunk) {
  constexpr int NR = 4 * NB;
  constexpr int TPW = 16 * MVM_G;  // targets per wave
  __shared__ double sp[256][4];
  __shared__ double sx[256][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t tb = (int64_t)blockIdx.x * (4 * TPW);  // targets [tb, tb + 4 TPW)
  const int64_t tw = tb + (int64_t)wave * TPW;
  const int64_t js = (int64_t)blockIdx.y * chunk, je = min(n, js + chunk);
  double tx[MVM_G], ty[MVM_G], tz[MVM_G], acc[MVM_G][2];
#pragma unroll
  for (int g = 0; g < MVM_G; ++g) {
    const int64_t t = tw + 16 * g + (lane & 15);
    if (t < n) {
      tx[g] = pts[3 * t];
      ty[g] = pts[3 * t + 1];
      tz[g] = pts[3 * t + 2];
    } else {
      tx[g] = 1e30;
      ty[g] = 0.0;
      tz[g] = 0.0;
    }
    acc[g][0] = acc[g][1] = 0.0;
  }
  for (int64_t j0 = js; j0 < je; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    __syncthreads();
    if (j < je) {
      for (int d = 0; d < 3; ++d) sp[threadIdx.x][d] = pts[3 * j + d];
#pragma unroll
      for (int c = 0; c < NR; ++c) sx[threadIdx.x][c] = x[j + c * ldx];
    } else {
      sp[threadIdx.x][0] = -1e30;
      sp[threadIdx.x][1] = sp[threadIdx.x][2] = 0.0;
#pragma unroll
      for (int c = 0; c < NR; ++c) sx[threadIdx.x][c] = 0.0;
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)256, je - j0);
    if (j0 < tb + 4 * TPW && j0 + 256 > tb)
      matvec_mfma_tile<KIND, true, NB>(sp, sx, cnt, tx, ty, tz, kf, acc);
    else
      matvec_mfma_tile<KIND, false, NB>(sp, sx, cnt, tx, ty, tz, kf, acc);
  }
  // D lane 16 q + 4 b + p holds target 4 b + q of each group, column p (+4)
  const int col = lane & 3;
  const int trow = 4 * ((lane >> 2) & 3) + (lane >> 4);
#pragma unroll
  for (int g = 0; g < MVM_G; ++g) {
    const int64_t t = tw + 16 * g + trow;
    if (t >= n) continue;
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const int c = col + 4 * h;
      if (part == nullptr)
        y[t + c * ldy] = fma(kf.diag, x[t + c * ldx], acc[g][h]);
      else
        part[(int64_t)blockIdx.y * NR * n + c * n + t] = acc[g][h];
    }
  }
}

// Exact matvec of a symmetric kernel (Laplace, Yukawa) for blocks of 8
// columns, each unordered pair evaluated once.  The points are cut into tiles
// of 512; the pair of tiles {I, J} adds K(I, J) x_J to y_I and K(I, J)^T x_I to
// y_J.  One launch per diagonal (I = J, both orders, the self term excluded),
// then launches over cyclic offsets: workgroup I takes the tiles
// (I, (I + k) mod nb) for MVS_R consecutive offsets k (offset nb/2 of an even
// nb only for I < nb/2, so every unordered pair comes once).  The y_I sums stay
// in registers over a launch and are added to slot 0; the y_J sums of offset
// slot r go to slot 1 + r, which within a launch only workgroup J - k writes,
// so every sum is taken in a fixed order and the result is deterministic.
//   Inside a tile the 8 waves own 64 targets each (4 groups of 16).  y_I uses
// the FP64 4x4x4 MFMA as in matvec_mfma_kernel: lane 16 q + 4 b + p evaluates
// K(target 4 b + p of the group, source q of the step).  For y_J the same entry
// is the B operand of a second MFMA whose k index runs over targets: the lane
// takes the entry of lane 16 p + 4 b + q (the transposed 4x4 block), and the
// 4x4 result of block b holds that block's targets' contribution to (source p,
// column q + c0) for the columns c0..c0+3 of its A operand x(target 4 b + q,
// column c0 + p).  The first product (e0) of block b takes c0 = 4 (b & 1) and
// the second (e1) the other half, so e0 of block b and e1 of block b ^ 1 cover
// the same columns: one exchange adds that pair, a second adds block b ^ 2, and
// the lanes of blocks 0 and 1 add columns 0-3 and 4-7 to the tile's y_J
// accumulator in LDS (the blocks are summed as (0 + 1) + (2 + 3) either way).
// The 8 sub-blocks of 64 sources rotate among the waves, one step per sub-block
// with a barrier between steps, so no two waves add to one row at a time.
constexpr int MVS_TB = 512;         // points per tile
constexpr int MVS_R = 8;            // offsets per launch (slots of y_J sums)
constexpr int MVS_MIN_TILES = 512;  // the pair form from 512 tiles (n > 261632) on

template <int KIND, bool DIAG>
__global__ __launch_bounds__(512) void matvec_sym_kernel(const double* __restrict__ pts,
                                                         int64_t n, KernelFn kf,
                                                         const double* __restrict__ x,
                                                         int64_t ldx, double* __restrict__ Y,
                                                         int nb, int k0, int kmax) {
  __shared__ double sp[3][MVS_TB];
  __shared__ double sx[MVS_TB][8];
  __shared__ double sy[MVS_TB][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, b = (lane >> 2) & 3, p = lane & 3;
  const int I = blockIdx.x;
  const int64_t tw = (int64_t)I * MVS_TB + wave * 64;  // the wave's 64 targets
  double tx[4], ty[4], tz[4], xt[4][2], acc[4][2];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t t = tw + 16 * g + (lane & 15);
    if (t < n) {
      tx[g] = pts[3 * t];
      ty[g] = pts[3 * t + 1];
      tz[g] = pts[3 * t + 2];
    } else {
      tx[g] = 1e30;
      ty[g] = 0.0;
      tz[g] = 0.0;
    }
    const int64_t tq = tw + 16 * g + 4 * b + q;
    const int h0 = 4 * (b & 1);  // column half of this lane's first y_J product
    xt[g][0] = tq < n ? x[tq + (h0 + p) * ldx] : 0.0;
    xt[g][1] = tq < n ? x[tq + (4 - h0 + p) * ldx] : 0.0;
    acc[g][0] = acc[g][1] = 0.0;
  }
  const int ntile = DIAG ? 1 : MVS_R;
  for (int r = 0; r < ntile; ++r) {
    const int k = k0 + r;
    if (!DIAG) {
      if (k > kmax) break;
      if (2 * k == nb && I >= nb / 2) continue;
    }
    const int J = DIAG ? I : (I + k) % nb;
    const int64_t js = (int64_t)J * MVS_TB;
    __syncthreads();
    {
      const int t = threadIdx.x;
      const int64_t sidx = js + t;
      if (sidx < n) {
        for (int d = 0; d < 3; ++d) sp[d][t] = pts[3 * sidx + d];
#pragma unroll
        for (int c = 0; c < 8; ++c) sx[t][c] = x[sidx + c * ldx];
      } else {
        sp[0][t] = -1e30;
        sp[1][t] = sp[2][t] = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) sx[t][c] = 0.0;
      }
      if (!DIAG)
#pragma unroll
        for (int c = 0; c < 8; ++c) sy[t][c] = 0.0;
    }
    __syncthreads();
    for (int step = 0; step < 8; ++step) {
      const int sub = DIAG ? step : (wave + step) & 7;
      for (int c = 0; c < 16; ++c) {
        const int s0 = sub * 64 + 4 * c;
        const int src = s0 + q;
        const double sx0 = sp[0][src], sy0 = sp[1][src], sz0 = sp[2][src];
        const double b0 = sx[src][p], b1 = sx[src][4 + p];
        double e0 = 0.0, e1 = 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const double dx = tx[g] - sx0, dy = ty[g] - sy0, dz = tz[g] - sz0;
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          double kv = inv_sqrt(r2);
          if (KIND == 1) kv *= exp(-kf.alpha * (r2 * kv));
          if (DIAG) kv = r2 > 0.0 ? kv : 0.0;
          acc[g][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(kv, b0, acc[g][0], 0, 0, 0);
          acc[g][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(kv, b1, acc[g][1], 0, 0, 0);
          if (!DIAG) {
            const double kt = __shfl(kv, (p << 4) | (b << 2) | q, 64);
            e0 = __builtin_amdgcn_mfma_f64_4x4x4f64(xt[g][0], kt, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f64_4x4x4f64(xt[g][1], kt, e1, 0, 0, 0);
          }
        }
        if (!DIAG) {
          // e0 of block b and e1 of block b ^ 1 hold the same columns
          double s1 = e0 + __shfl_xor(e1, 4, 64);
          s1 += __shfl_xor(s1, 8, 64);
          if (b < 2) sy[s0 + p][4 * b + q] += s1;
        }
      }
      if (!DIAG) __syncthreads();
    }
    if (!DIAG) {
      const int t = threadIdx.x;
      const int64_t sidx = js + t;
      if (sidx < n) {
        double* Yr = Y + (int64_t)(1 + r) * 8 * n;
#pragma unroll
        for (int c = 0; c < 8; ++c) Yr[c * n + sidx] += sy[t][c];
      }
    }
  }
  // y_I sums: D lane 16 q + 4 b + p holds target 4 b + q of each group, column p (+4)
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t t = tw + 16 * g + 4 * b + q;
    if (t >= n) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = p + 4 * h;
      Y[c * n + t] = DIAG ? acc[g][h] : Y[c * n + t] + acc[g][h];
    }
  }
}

// Exact matvec of a symmetric kernel for one column, each unordered pair
// evaluated once: the one-column counterpart of matvec_sym_kernel (same tile
// pairs, launches, rotation and slots).  Lane 16 q + 4 b + p of a wave
// evaluates K(target 16 g + 4 b + q of the wave's 64, source p of the step) for
// the four target groups g.  y_I: a vector FMA with x of the lane's source; the
// four lanes of a target (p = 0..3) are added once, at the end of the launch.
// y_J: a vector FMA with x of the lane's target over the four groups, then four
// exchanges add the 16 lanes of each source (lane bits 2-5), and lanes 0-3 add
// the four sources' sums to the tile's y_J accumulator in LDS.  (The FP64 MFMA
// with x in one row of A, the entry as B, gave the same sums 3% slower: three
// of its four rows were zeros.)
template <int KIND, bool DIAG>
__global__ __launch_bounds__(512) void matvec_sym1_kernel(const double* __restrict__ pts,
                                                          int64_t n, KernelFn kf,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ Y, int nb, int k0,
                                                          int kmax) {
  __shared__ double sp[3][MVS_TB];
  __shared__ double sx[MVS_TB];
  __shared__ double sy[MVS_TB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, b = (lane >> 2) & 3, p = lane & 3;
  const int I = blockIdx.x;
  const int64_t tw = (int64_t)I * MVS_TB + wave * 64;  // the wave's 64 targets
  double tx[4], ty[4], tz[4], xa[4], acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t t = tw + 16 * g + 4 * b + q;
    if (t < n) {
      tx[g] = pts[3 * t];
      ty[g] = pts[3 * t + 1];
      tz[g] = pts[3 * t + 2];
    } else {
      tx[g] = 1e30;
      ty[g] = 0.0;
      tz[g] = 0.0;
    }
    xa[g] = t < n ? x[t] : 0.0;
    acc[g] = 0.0;
  }
  const int ntile = DIAG ? 1 : MVS_R;
  for (int r = 0; r < ntile; ++r) {
    const int k = k0 + r;
    if (!DIAG) {
      if (k > kmax) break;
      if (2 * k == nb && I >= nb / 2) continue;
    }
    const int J = DIAG ? I : (I + k) % nb;
    const int64_t js = (int64_t)J * MVS_TB;
    __syncthreads();
    {
      const int t = threadIdx.x;
      const int64_t sidx = js + t;
      if (sidx < n) {
        for (int d = 0; d < 3; ++d) sp[d][t] = pts[3 * sidx + d];
        sx[t] = x[sidx];
      } else {
        sp[0][t] = -1e30;
        sp[1][t] = sp[2][t] = 0.0;
        sx[t] = 0.0;
      }
      if (!DIAG) sy[t] = 0.0;
    }
    __syncthreads();
    for (int step = 0; step < 8; ++step) {
      const int sub = DIAG ? step : (wave + step) & 7;
      // unrolled 4 times (measured with the MFMA form of the y_J sums: 1.7%
      // faster than not unrolled, 20% faster than fully, whose 244 registers
      // halved the occupancy)
#pragma unroll 4
      for (int c = 0; c < 16; ++c) {
        const int s0 = sub * 64 + 4 * c;
        const int src = s0 + p;
        const double sx0 = sp[0][src], sy0 = sp[1][src], sz0 = sp[2][src];
        const double xs = sx[src];
        double e = 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const double dx = tx[g] - sx0, dy = ty[g] - sy0, dz = tz[g] - sz0;
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          double kv = inv_sqrt(r2);
          if (KIND == 1) kv *= exp(-kf.alpha * (r2 * kv));
          if (DIAG) kv = r2 > 0.0 ? kv : 0.0;
          acc[g] = fma(kv, xs, acc[g]);
          if (!DIAG) e = fma(kv, xa[g], e);
        }
        if (!DIAG) {
          e += __shfl_xor(e, 4, 64);
          e += __shfl_xor(e, 8, 64);
          e += __shfl_xor(e, 16, 64);
          e += __shfl_xor(e, 32, 64);
          if (lane < 4) sy[s0 + lane] += e;
        }
      }
      if (!DIAG) __syncthreads();
    }
    if (!DIAG) {
      const int t = threadIdx.x;
      const int64_t sidx = js + t;
      if (sidx < n) Y[(int64_t)(1 + r) * n + sidx] += sy[t];
    }
  }
  // y_I sums: the four source lanes of each target, (p0 + p1) + (p2 + p3)
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    double v = acc[g];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    const int64_t t = tw + 16 * g + 4 * b + q;
    if (p == 0 && t < n) Y[t] = DIAG ? v : Y[t] + v;
  }
}

__global__ void zero_kernel(double* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// y(i, c) = diag x(i, c) + sum over ranges s (in order) of part[s][c][i]
__global__ __launch_bounds__(256) void matvec_reduce_kernel(const double* __restrict__ part,
                                                            int nsplit, int nr, int64_t n,
                                                            double diag,
                                                            const double* __restrict__ x,
                                                            int64_t ldx, double* __restrict__ y,
                                                            int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nr) return;
  const int64_t i = e % n, c = e / n;
  double acc = 0.0;
  for (int q = 0; q < nsplit; ++q) acc += part[(int64_t)q * nr * n + c * n + i];
  y[i + c * ldy] = fma(diag, x[i + c * ldx], acc);
}

namespace {
constexpr int MV_MAX_SPLIT = 8;
// source ranges per launch: enough workgroups to fill the chip several times
int matvec_split(int64_t n) {
  const int64_t grid = (n + 511) / 512;
  if (n < 65536) return 1;
  return (int)std::max<int64_t>(1, std::min<int64_t>(MV_MAX_SPLIT, 4096 / grid));
}

// the pair forms (blocks of 8 columns, single columns): a symmetric kernel and
// at least MVS_MIN_TILES tiles
bool matvec_pairs(int64_t n, int kind) {
  return kind != 2 && (n + MVS_TB - 1) / MVS_TB >= MVS_MIN_TILES;
}

template <int KIND>
void matvec_sym_launch(const double* pts, int64_t n, KernelFn kf, const double* x, int64_t ldx,
                       double* y, int64_t ldy, double* work, hipStream_t s) {
  const int nb = (int)((n + MVS_TB - 1) / MVS_TB);
  const int kmax = nb / 2;
  const int64_t slots = (int64_t)MVS_R * 8 * n;
  hipLaunchKernelGGL(zero_kernel, dim3(2048), dim3(256), 0, s, work + 8 * n, slots);
  hipLaunchKernelGGL((matvec_sym_kernel<KIND, true>), dim3(nb), dim3(512), 0, s, pts, n, kf, x,
                     ldx, work, nb, 0, 0);
  for (int k0 = 1; k0 <= kmax; k0 += MVS_R)
    hipLaunchKernelGGL((matvec_sym_kernel<KIND, false>), dim3(nb), dim3(512), 0, s, pts, n, kf,
                       x, ldx, work, nb, k0, kmax);
  const int64_t tot = n * 8;
  hipLaunchKernelGGL(matvec_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     work, 1 + MVS_R, 8, n, kf.diag, x, ldx, y, ldy);
}

template <int KIND>
void matvec_sym1_launch(const double* pts, int64_t n, KernelFn kf, const double* x, int64_t ldx,
                        double* y, int64_t ldy, double* work, hipStream_t s) {
  const int nb = (int)((n + MVS_TB - 1) / MVS_TB);
  const int kmax = nb / 2;
  hipLaunchKernelGGL(zero_kernel, dim3(2048), dim3(256), 0, s, work + n, (int64_t)MVS_R * n);
  hipLaunchKernelGGL((matvec_sym1_kernel<KIND, true>), dim3(nb), dim3(512), 0, s, pts, n, kf, x,
                     work, nb, 0, 0);
  for (int k0 = 1; k0 <= kmax; k0 += MVS_R)
    hipLaunchKernelGGL((matvec_sym1_kernel<KIND, false>), dim3(nb), dim3(512), 0, s, pts, n, kf,
                       x, work, nb, k0, kmax);
  hipLaunchKernelGGL(matvec_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     work, 1 + MVS_R, 1, n, kf.diag, x, ldx, y, ldy);
}

template <int NR>
void matvec_launch(const double* pts, int64_t n, KernelFn kf, const double* x, int64_t ldx,
                   double* y, int64_t ldy, double* work, hipStream_t s) {
  if constexpr (NR == 1) {
    if (work && matvec_pairs(n, kf.kind)) {
      if (kf.kind == 0)
        matvec_sym1_launch<0>(pts, n, kf, x, ldx, y, ldy, work, s);
      else
        matvec_sym1_launch<1>(pts, n, kf, x, ldx, y, ldy, work, s);
      return;
    }
  }
  if constexpr (NR == 8) {
    if (work && matvec_pairs(n, kf.kind)) {
      if (kf.kind == 0)
        matvec_sym_launch<0>(pts, n, kf, x, ldx, y, ldy, work, s);
      else
        matvec_sym_launch<1>(pts, n, kf, x, ldx, y, ldy, work, s);
      return;
    }
  }
  const int ns = work ? matvec_split(n) : 1;
  const unsigned gx = (unsigned)((n + 511) / 512);
  const int64_t chunk = ns > 1 ? ((n + ns - 1) / ns + 255) / 256 * 256 : n;
  const int nsu = (int)((n + chunk - 1) / chunk);  // ranges actually used
  double* part = nsu > 1 ? work : nullptr;
  const dim3 grid(gx, (unsigned)std::max(nsu, 1));
  static_assert(4 * 16 * MVM_G == 512, "both matvec forms cover 512 targets per workgroup");
  if constexpr (NR == 8 || NR == 4) {
    constexpr int NB = NR / 4;
    if (kf.kind == 0)
      hipLaunchKernelGGL((matvec_mfma_kernel<0, NB>), grid, dim3(256), 0, s, pts, n, kf, x, ldx,
                         y, ldy, part, chunk);
    else if (kf.kind == 1)
      hipLaunchKernelGGL((matvec_mfma_kernel<1, NB>), grid, dim3(256), 0, s, pts, n, kf, x, ldx,
                         y, ldy, part, chunk);
    else
      hipLaunchKernelGGL((matvec_mfma_kernel<2, NB>), grid, dim3(256), 0, s, pts, n, kf, x, ldx,
                         y, ldy, part, chunk);
  } else {
    if (kf.kind == 0)
      hipLaunchKernelGGL((matvec_kernel<NR, 0>), grid, dim3(256), 0, s, pts, n, kf, x, ldx, y,
                         ldy, part, chunk);
    else if (kf.kind == 1)
      hipLaunchKernelGGL((matvec_kernel<NR, 1>), grid, dim3(256), 0, s, pts, n, kf, x, ldx, y,
                         ldy, part, chunk);
    else
      hipLaunchKernelGGL((matvec_kernel<NR, 2>), grid, dim3(256), 0, s, pts, n, kf, x, ldx, y,
                         ldy, part, chunk);
  }
  if (part) {
    const int64_t tot = n * NR;
    hipLaunchKernelGGL(matvec_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       part, nsu, NR, n, kf.diag, x, ldx, y, ldy);
  }
}
}  // namespace

int64_t matvec_work_words(int64_t n, int nrhs) {
  const int ns = matvec_split(n);
  int64_t w = ns > 1 ? (int64_t)ns * std::min(nrhs, 8) * n : 0;
  // the pair forms (blocks of 8 columns, single columns; a symmetric kernel):
  // sums of y_I and the MVS_R slots of y_J sums
  if (nrhs >= 8 && matvec_pairs(n, 0)) w = std::max<int64_t>(w, (int64_t)(1 + MVS_R) * 8 * n);
  if (nrhs % 4 != 0 && matvec_pairs(n, 0)) w = std::max<int64_t>(w, (int64_t)(1 + MVS_R) * n);
  return w;
}

void launch_matvec(const double* pts, int64_t n, KernelFn kf, const double* x, int64_t ldx,
                   double* y, int64_t ldy, int nrhs, double* work, hipStream_t s) {
  if (n <= 0) return;
  int c = 0;
  while (c < nrhs) {
    const int left = nrhs - c;
    const double* xc = x + (int64_t)c * ldx;
    double* yc = y + (int64_t)c * ldy;
    if (left >= 8) {
      matvec_launch<8>(pts, n, kf, xc, ldx, yc, ldy, work, s);
      c += 8;
    } else if (left >= 4) {
      matvec_launch<4>(pts, n, kf, xc, ldx, yc, ldy, work, s);
      c += 4;
    } else {
      matvec_launch<1>(pts, n, kf, xc, ldx, yc, ldy, work, s);
      c += 1;
    }
  }
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------
__global__ void d2f_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (float)s[i];
}
__global__ void f2d_kernel(const float* __restrict__ s, double* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (double)s[i];
}
void launch_convert_d2f(const double* src, float* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(d2f_kernel, dim3((unsigned)g), dim3(256), 0, s, src, dst, count);
}
void launch_convert_f2d(const float* src, double* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(f2d_kernel, dim3((unsigned)g), dim3(256), 0, s, src, dst, count);
}

// r = b - ax, per-column |r|^2 and |b|^2 (one workgroup per column).
__global__ __launch_bounds__(256) void resid_kernel(const double* __restrict__ b, int64_t ldb,
                                                    const double* __restrict__ ax, int64_t ldax,
                                                    double* __restrict__ r, int64_t ldr,
                                                    int64_t n, double* rn, double* bn) {
  __shared__ double sh[8];
  const int c = blockIdx.x;
  double pr = 0.0, pb = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double bv = b[i + c * ldb];
    double rv = bv - ax[i + c * ldax];
    r[i + c * ldr] = rv;
    pr += rv * rv;
    pb += bv * bv;
  }
  double sr = block_sum256(pr, sh);
  __syncthreads();
  double sb = block_sum256(pb, sh);
  if (threadIdx.x == 0) {
    rn[c] = sr;
    bn[c] = sb;
  }
}
void launch_resid_norms(const double* b, int64_t ldb, const double* ax, int64_t ldax, double* r,
                        int64_t ldr, int64_t n, int nrhs, double* rnorm2, double* bnorm2,
                        hipStream_t s) {
  hipLaunchKernelGGL(resid_kernel, dim3(nrhs), dim3(256), 0, s, b, ldb, ax, ldax, r, ldr, n,
                     rnorm2, bnorm2);
}

__global__ void axpy_cols_kernel(double* x, int64_t ldx, const double* d, int64_t ldd,
                                 int64_t n) {
  const int c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i + c * ldx] += d[i + c * ldd];
}
void launch_axpy_cols(double* x, int64_t ldx, const double* d, int64_t ldd, int64_t n, int nrhs,
                      hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(axpy_cols_kernel, dim3((unsigned)g, nrhs), dim3(256), 0, s, x, ldx, d, ldd,
                     n);
}

// C (M x N, ld ldc) = A^T B for a long inner dimension n (A n x M, B n x N,
// column-major), N <= 8.  Workgroup (chunk, group of 8 columns of A) sums the
// products over its contiguous rows into partial[chunk][j][i]; gram_sum_kernel
// adds the chunks in a fixed order (deterministic).
__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ A,
                                                           int64_t lda, int M,
                                                           const double* __restrict__ B,
                                                           int64_t ldb, int N, int64_t n,
                                                           double* __restrict__ partial) {
  __shared__ double sh[4][64];
  const int i0 = blockIdx.y * 8;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
  double acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    double av[8], bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bv[j] = j < N ? B[r + j * ldb] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) av[i] = i0 + i < M ? A[r + (int64_t)(i0 + i) * lda] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < 64; ++e) {
    const double v = wave_sum(acc[e >> 3][e & 7]);
    if (lane == 0) sh[wv][e] = v;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int e = threadIdx.x, i = e >> 3, j = e & 7;
    if (i0 + i < M && j < N)
      partial[((int64_t)blockIdx.x * N + j) * M + i0 + i] =
          (sh[0][e] + sh[1][e]) + (sh[2][e] + sh[3][e]);
  }
}

__global__ __launch_bounds__(256) void gram_sum_kernel(const double* __restrict__ partial,
                                                       int nchunk, int M, int N,
                                                       double* __restrict__ C, int64_t ldc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const int i = e % M, j = e / M;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[((int64_t)c * N + j) * M + i];
  C[i + (int64_t)j * ldc] = s;
}

void launch_gram(const double* A, int64_t lda, int M, const double* B, int64_t ldb, int N,
                 int64_t n, double* C, int64_t ldc, double* partial, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const dim3 grid(GRAM_CHUNKS, (unsigned)((M + 7) / 8));
  hipLaunchKernelGGL(gram_partial_kernel, grid, dim3(256), 0, s, A, lda, M, B, ldb, N, n,
                     partial);
  hipLaunchKernelGGL(gram_sum_kernel, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s,
                     partial, GRAM_CHUNKS, M, N, C, ldc);
}

// Several dot products with one vector: partial[b k + c] = sum over the rows of
// block b of V(r, c) w(r), c < k <= 32 (grid-stride rows, fixed block count),
// then out[c] = sum over blocks in a fixed order (deterministic).
__global__ __launch_bounds__(256) void multidot_kernel(const double* __restrict__ V, int64_t ldv,
                                                       int k, const double* __restrict__ w,
                                                       int64_t n, double* __restrict__ partial) {
  __shared__ double sh[4][32];
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
    const double wr = w[r];
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c < k) acc[c] = fma(V[r + c * ldv], wr, acc[c]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 32; ++c)
    if (c < k) {
      const double v = wave_sum(acc[c]);
      if (lane == 0) sh[wv][c] = v;
    }
  __syncthreads();
  if ((int)threadIdx.x < k)
    partial[(int64_t)blockIdx.x * k + threadIdx.x] =
        (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

__global__ void multidot_sum_kernel(const double* __restrict__ partial, int nblk, int k,
                                    double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * k + c];
  out[c] = s;
}

void launch_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                     double* partial, int nblk, double* out, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(multidot_kernel, dim3(nblk), dim3(256), 0, s, V, ldv, k, w, n, partial);
  hipLaunchKernelGGL(multidot_sum_kernel, dim3(1), dim3(32), 0, s, partial, nblk, k, out);
}

// dst = src / sqrt(nrm2[0])  (dst = src when nrm2[0] is zero)
__global__ void scale_inv_norm_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                      const double* __restrict__ nrm2, int64_t n) {
  const double d = nrm2[0];
  const double f = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] * f;
}

void launch_scale_inv_norm(double* dst, const double* src, const double* nrm2, int64_t n,
                           hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(scale_inv_norm_kernel, dim3((unsigned)g), dim3(256), 0, s, dst, src, nrm2, n);
}

// dst[t] = src[perm[t]] (inverse = 0) or dst[perm[t]] = src[t] (inverse = 1)
__global__ void permute_kernel(const double* src, int64_t lds, double* dst, int64_t ldd,
                               const int64_t* perm, int64_t n, int inverse) {
  const int c = blockIdx.y;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (!inverse)
      dst[t + c * ldd] = src[perm[t] + c * lds];
    else
      dst[perm[t] + c * ldd] = src[t + c * lds];
  }
}
void launch_permute_rows(const double* src, int64_t lds, double* dst, int64_t ldd,
                         const int64_t* perm, int64_t n, int nrhs, int inverse, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)g, nrhs), dim3(256), 0, s, src, lds, dst,
                     ldd, perm, n, inverse);
}

// ---------------------------------------------------------------------------
// P^T as a dense matrix from LU row interchanges (ipiv == nullptr: identity);
// one thread per column follows where the unit entry of that column moves.
// ---------------------------------------------------------------------------
__global__ void perm_matrix_kernel(const PermItem* __restrict__ items,
                                   const int64_t* __restrict__ slab_ptr, int nitems) {
  int64_t slab = blockIdx.x;
  int id = find_item(slab_ptr, nitems, slab);
  const PermItem it = items[id];
  const int c = (int)(slab - slab_ptr[id]) * 64 + threadIdx.x;
  if (c >= it.m) return;
  int pos = c;
  if (it.ipiv) {
    // B = P^T I where P^T applies the swaps (t, ipiv[t]) for t = 0..m-1 in order
    for (int t = 0; t < it.m; ++t) {
      int p = it.ipiv[t];
      if (p == t) continue;
      if (pos == t)
        pos = p;
      else if (pos == p)
        pos = t;
    }
  }
  double* col = it.out + (int64_t)c * it.ld;
  for (int r = 0; r < it.m; ++r) col[r] = (r == pos) ? 1.0 : 0.0;
}

void launch_perm_matrix(const PermItem* items, const int64_t* slab_ptr, int64_t nslabs,
                        int nitems, hipStream_t s) {
  if (nslabs <= 0) return;
  hipLaunchKernelGGL(perm_matrix_kernel, dim3((unsigned)nslabs), dim3(64), 0, s, items, slab_ptr,
                     nitems);
}

// W' (m x k) of the row ID: row piv[t] = e_t for t < k, row piv[k+s] = E[:, s]^T
// where E = R11^-1 R12 sits in rows 0..k-1, columns k.. of the pivoted-QR matrix.
__global__ void wprime_kernel(const WpItem* __restrict__ items) {
  const WpItem it = items[blockIdx.x];
  const int m = it.m, k = it.k;
  for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
    const int s = e / k, t = e % k;  // source row s of [I; E^T], column t
    double v;
    if (s < k)
      v = (s == t) ? 1.0 : 0.0;
    else
      v = it.E[t + (int64_t)(s - k) * it.ldE];
    it.W[it.piv[s] + (int64_t)t * it.ldW] = v;
  }
}

void launch_wprime(const WpItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(wprime_kernel, dim3(nitems), dim3(256), 0, s, items);
}

// Strictly-lower part of a batch of matrices set to zero (triangular factors).
__global__ void zero_lower_kernel(const CopyItem* __restrict__ items) {
  const CopyItem it = items[blockIdx.x];
  for (int64_t e = threadIdx.x; e < (int64_t)it.rows * it.cols; e += blockDim.x) {
    int i = (int)(e % it.rows), j = (int)(e / it.rows);
    if (i > j) it.dst[i + (int64_t)j * it.ldd] = 0.0;
  }
}
void launch_zero_lower(const CopyItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(zero_lower_kernel, dim3(nitems), dim3(256), 0, s, items);
}

// log|det| of LU factors: sum of log|U_tt| per matrix (one workgroup each).
__global__ __launch_bounds__(256) void logdet_kernel(const MatDesc* __restrict__ ds, double* out) {
  __shared__ double sh[8];
  const MatDesc d = ds[blockIdx.x];
  double p = 0.0;
  for (int t = threadIdx.x; t < d.m; t += 256) p += log(fabs(d.A[t + (int64_t)t * d.lda]));
  double s = block_sum256(p, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}
void launch_logdet(const MatDesc* d, int nmat, double* out, hipStream_t s) {
  if (nmat <= 0) return;
  hipLaunchKernelGGL(logdet_kernel, dim3(nmat), dim3(256), 0, s, d, out);
}

}  // namespace h2ulv
