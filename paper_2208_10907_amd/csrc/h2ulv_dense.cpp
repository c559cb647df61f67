// Batched dense building blocks of the sweep, each a short sequence of batched
// launches whose O(m^3) part runs in the grouped MFMA GEMM:
//   * blocked LU with partial pivoting and the inverse from it (Sec. II-B,
//     Eq. lu; the paper's GETRF/TRSM pair of Sec. III-D);
//   * triangular solves by diagonal blocks (inverted nb x nb blocks + GEMM);
//   * blocked Householder QR of the row-ID matrix W and the explicit
//     orthogonal factor U = [U^S U^R] (Sec. II-A: the skeleton and redundant
//     parts of the shared basis; LAPACK dgeqrf/dlarft/dorgqr conventions).
#include "h2ulv_dense.h"

#include <exception>
#include <map>
#include <mutex>

#include <algorithm>

namespace h2ulv {

namespace {

struct DevCache {
  std::mutex mu;
  std::multimap<size_t, void*> blocks;  // free blocks by size
  size_t cached = 0;
  int depth = 0;          // nesting of library calls holding the cache
  int64_t oom_releases = 0;      // times the cache was emptied after a failed hipMalloc
  int64_t reserve_releases = 0;  // times it was emptied to keep the free reserve
};

DevCache& dev_cache() {
  static DevCache c;
  return c;
}

size_t round_block(size_t b) {
  const size_t g = b >= ((size_t)1 << 20) ? ((size_t)2 << 20) : 256;
  return (b + g - 1) / g * g;
}

void release_locked(DevCache& c) {
  for (auto& kv : c.blocks) (void)hipFree(kv.second);
  c.blocks.clear();
  c.cached = 0;
}

}  // namespace

namespace {

// Tile-shape autotuning of the grouped GEMM.  The synthetic batch has the shape
// of the fill-in products: 96 items of 256 x 256, each a sum of 4 products with
// K = 256, the left operands shared by all items (like the D_kj blocks that many
// boxes read) and the right ones per item.
struct TileTune {
  std::mutex mu;
  bool have[2] = {false, false};
  double rate[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // [0] f64, [1] f32
};
TileTune& tile_tune(int dev) {
  static TileTune t[64];
  return t[dev & 63];
}

template <typename T>
void measure_tile_rates(hipStream_t s, double* out) {
  constexpr int NI = 96, NT = 4, D = 256;
  const int64_t blk = (int64_t)D * D;
  DBuf A(NT * blk * sizeof(T)), B(NI * blk * sizeof(T)), Cb(NI * blk * sizeof(T));
  H2ULV_HIP(hipMemsetAsync(A.p, 0, A.bytes, s));
  H2ULV_HIP(hipMemsetAsync(B.p, 0, B.bytes, s));
  std::vector<GemmItem<T>> items(NI);
  std::vector<GemmTerm<T>> terms(NI * NT);
  for (int i = 0; i < NI; ++i) {
    items[i] = GemmItem<T>{Cb.as<T>() + i * blk, D, D, D, i * NT, NT, 1.0, 0.0};
    for (int t = 0; t < NT; ++t)
      terms[i * NT + t] = GemmTerm<T>{A.as<T>() + t * blk, B.as<T>() + i * blk, D, D, D, 0};
  }
  const int shapes64[4][2] = {{64, 64}, {64, 128}, {128, 64}, {128, 128}};
  const int shapes32[2][2] = {{64, 64}, {128, 128}};
  const bool f64 = sizeof(T) == 8;
  const int ns = f64 ? 4 : 2;
  DBuf di(items.size() * sizeof(GemmItem<T>)), dt(terms.size() * sizeof(GemmTerm<T>)),
      dp((NI + 1) * sizeof(int64_t));
  H2ULV_HIP(hipMemcpyAsync(di.p, items.data(), di.bytes, hipMemcpyHostToDevice, s));
  H2ULV_HIP(hipMemcpyAsync(dt.p, terms.data(), dt.bytes, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  H2ULV_HIP(hipEventCreate(&e0));
  H2ULV_HIP(hipEventCreate(&e1));
  const double flops = 2.0 * NI * NT * (double)D * D * D;
  for (int c = 0; c < ns; ++c) {
    const int tm = f64 ? shapes64[c][0] : shapes32[c][0];
    const int tn = f64 ? shapes64[c][1] : shapes32[c][1];
    const int64_t per = (int64_t)(D / tm) * (D / tn);
    std::vector<int64_t> tp(NI + 1);
    for (int i = 0; i <= NI; ++i) tp[i] = i * per;
    H2ULV_HIP(hipMemcpyAsync(dp.p, tp.data(), dp.bytes, hipMemcpyHostToDevice, s));
    launch_gemm<T, T>(di.as<GemmItem<T>>(), dt.as<GemmTerm<T>>(), dp.as<int64_t>(), NI * per,
                      NI, tm, tn, s);  // warm-up
    H2ULV_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r)
      launch_gemm<T, T>(di.as<GemmItem<T>>(), dt.as<GemmTerm<T>>(), dp.as<int64_t>(), NI * per,
                        NI, tm, tn, s);
    H2ULV_HIP(hipEventRecord(e1, s));
    H2ULV_HIP(hipEventSynchronize(e1));
    float ms = 0;
    H2ULV_HIP(hipEventElapsedTime(&ms, e0, e1));
    out[c] = ms > 0 ? 3.0 * flops / (ms * 1e-3) / 1e12 : 1.0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  H2ULV_HIP(hipGetLastError());
}

}  // namespace

const double* gemm_tile_rates(bool f64, hipStream_t s) {
  int dev = 0;
  H2ULV_HIP(hipGetDevice(&dev));
  TileTune& t = tile_tune(dev);
  std::lock_guard<std::mutex> lk(t.mu);
  const int q = f64 ? 0 : 1;
  if (!t.have[q]) {
    if (f64)
      measure_tile_rates<double>(s, t.rate[0]);
    else
      measure_tile_rates<float>(s, t.rate[1]);
    t.have[q] = true;
  }
  return t.rate[q];
}

bool gemm_tile_rates_known(double* out6) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  TileTune& t = tile_tune(dev);
  std::lock_guard<std::mutex> lk(t.mu);
  for (int c = 0; c < 4; ++c) out6[c] = t.have[0] ? t.rate[0][c] : 0.0;
  for (int c = 0; c < 2; ++c) out6[4 + c] = t.have[1] ? t.rate[1][c] : 0.0;
  return t.have[0] || t.have[1];
}

AllocHook& current_alloc_hook() {
  thread_local AllocHook h;
  return h;
}

void* cache_alloc(size_t bytes, size_t* got) {
  DevCache& c = dev_cache();
  const size_t want = round_block(bytes);
  {
    std::lock_guard<std::mutex> lk(c.mu);
    // smallest cached block that fits without wasting more than half of it
    auto it = c.blocks.lower_bound(want);
    if (it != c.blocks.end() && it->first <= want + want / 2 + ((size_t)4 << 20)) {
      void* p = it->second;
      *got = it->first;
      c.cached -= it->first;
      c.blocks.erase(it);
      return p;
    }
  }
  // keep a reserve of free device memory for the runtime (kernel scratch,
  // queues) and other users: before growing into it, hand the cached blocks
  // back, after waiting for the device since queued work may still read them
  {
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) == hipSuccess) {
      const size_t reserve = std::max<size_t>((size_t)16 << 30, totb / 16);
      std::unique_lock<std::mutex> lk(c.mu);
      if (c.cached > 0 && freeb < want + reserve) {
        lk.unlock();
        (void)hipDeviceSynchronize();
        lk.lock();
        c.reserve_releases += 1;
        release_locked(c);
      }
    } else {
      (void)hipGetLastError();
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // cached blocks are free on the host side but queued work may still read
    // them: wait for the device before handing them back to the runtime
    (void)hipDeviceSynchronize();
    {
      std::lock_guard<std::mutex> lk(c.mu);
      c.oom_releases += 1;
      release_locked(c);
    }
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(H2ULV_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  *got = want;
  return p;
}

namespace {
struct PinnedPool {
  std::mutex mu;
  std::multimap<size_t, char*> blocks;
  size_t held = 0;
};
PinnedPool& pinned_pool() {
  static PinnedPool pp;
  return pp;
}
constexpr size_t PINNED_KEEP = (size_t)4 << 30;  // most pinned bytes kept for reuse
}  // namespace

char* pinned_get(size_t bytes, size_t* got) {
  PinnedPool& pp = pinned_pool();
  const size_t want = round_block(bytes);
  {
    std::lock_guard<std::mutex> lk(pp.mu);
    auto it = pp.blocks.lower_bound(want);
    if (it != pp.blocks.end() && it->first <= 2 * want) {
      char* p = it->second;
      *got = it->first;
      pp.held -= it->first;
      pp.blocks.erase(it);
      return p;
    }
  }
  char* p = nullptr;
  if (hipHostMalloc((void**)&p, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    fail(H2ULV_ERR_OOM, "pinned host allocation of " + std::to_string(bytes) + " bytes failed");
  }
  *got = want;
  return p;
}

void pinned_put(char* p, size_t bytes) {
  PinnedPool& pp = pinned_pool();
  std::lock_guard<std::mutex> lk(pp.mu);
  if (pp.held + bytes > PINNED_KEEP) {
    (void)hipHostFree(p);
    return;
  }
  pp.blocks.emplace(bytes, p);
  pp.held += bytes;
}

void cache_free(void* p, size_t bytes) {
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.blocks.emplace(bytes, p);
  c.cached += bytes;
}

void cache_release() {
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  release_locked(c);
}

int64_t cache_oom_releases() {
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  return c.oom_releases + c.reserve_releases;
}

size_t cache_bytes() {
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  return c.cached;
}

size_t free_device_bytes() {
  size_t freeb = 0, totb = 0;
  H2ULV_HIP(hipMemGetInfo(&freeb, &totb));
  return freeb + cache_bytes();
}

CacheScope::CacheScope() {
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.depth += 1;
}

CacheScope::~CacheScope() {
  // leaving by an exception: queued work may still use cached blocks, so the
  // cache is handed back once the device is idle
  const bool unwinding = std::uncaught_exceptions() > 0;
  if (unwinding) (void)hipDeviceSynchronize();
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.depth -= 1;
  if (c.depth == 0 && unwinding) release_locked(c);
}

const char* profile_name(const char* kernel, const char* site) {
  static std::mutex mu;
  static std::map<std::string, std::string> names;
  std::lock_guard<std::mutex> lk(mu);
  std::string key = std::string(kernel) + ":" + site;
  return names.emplace(key, key).first->second.c_str();
}

MemStats& mem_stats() {
  static MemStats ms;
  return ms;
}

Profiler& profiler() {
  static Profiler p;
  return p;
}

static constexpr int LU_NB = 64;   // triangular block width
static constexpr int LU_PANEL = 64;  // LU panel width
static constexpr int QR_NB = 32;   // Householder panel width

// X = L^-1 B (L unit lower) by blocks of LU_NB rows; B is overwritten.
void trsm_lower_unit(Stage& st, const std::vector<TriRhs>& sys) {
  if (sys.empty()) return;
  const int nb = LU_NB;
  int maxm = 0;
  std::vector<MatDesc> ds;
  std::vector<int64_t> bp(1, 0), off;
  int64_t tot = 0;
  for (auto& t : sys) {
    MatDesc d{};
    d.A = const_cast<double*>(t.T);
    d.lda = t.ldt;
    d.m = t.m;
    d.n = t.m;
    ds.push_back(d);
    int nbk = (t.m + nb - 1) / nb;
    bp.push_back(bp.back() + nbk);
    off.push_back(tot);
    tot += (int64_t)nbk * nb * nb;
    maxm = std::max(maxm, t.m);
  }
  double* inv = st.scratch<double>(tot);
  int nmat = (int)sys.size();
  int64_t nblk = bp.back();
  MatDesc* dd = st.up(std::move(ds));
  int64_t* dbp = st.up(std::move(bp));
  std::vector<int64_t> offc = off;
  int64_t* doff = st.up(std::move(offc));
  launch_trinv_diag(dd, dbp, nblk, nmat, nb, 0, inv, doff, st.s);
  H2ULV_HIP(hipGetLastError());
  for (int o = 0; o < maxm; o += nb) {
    GemmBatch<double> g1, g2;
    for (size_t b = 0; b < sys.size(); ++b) {
      const TriRhs& t = sys[b];
      if (t.m <= o || t.ncols <= 0) continue;
      int w = std::min(nb, t.m - o);
      const double* blk = inv + off[b] + (int64_t)(o / nb) * nb * nb;
      g1.one(t.X + o, t.ldx, w, t.ncols, w, blk, nb, false, t.B + o, t.ldb, false);
      int rest = t.m - o - w;
      if (rest > 0)
        g2.one(t.B + o + w, t.ldb, rest, t.ncols, w, t.T + (o + w) + (int64_t)o * t.ldt, t.ldt,
               false, t.X + o, t.ldx, false, -1.0, 1.0);
    }
    g1.run(st, "trsm");
    g2.run(st, "trsm");
  }
}

// X = U^-1 B (U upper with diagonal) by blocks from the bottom; B is overwritten.
void trsm_upper(Stage& st, const std::vector<TriRhs>& sys) {
  if (sys.empty()) return;
  const int nb = LU_NB;
  int maxblk = 0;
  std::vector<MatDesc> ds;
  std::vector<int64_t> bp(1, 0), off;
  int64_t tot = 0;
  for (auto& t : sys) {
    MatDesc d{};
    d.A = const_cast<double*>(t.T);
    d.lda = t.ldt;
    d.m = t.m;
    d.n = t.m;
    ds.push_back(d);
    int nbk = (t.m + nb - 1) / nb;
    bp.push_back(bp.back() + nbk);
    off.push_back(tot);
    tot += (int64_t)nbk * nb * nb;
    maxblk = std::max(maxblk, nbk);
  }
  double* inv = st.scratch<double>(tot);
  int nmat = (int)sys.size();
  int64_t nblk = bp.back();
  MatDesc* dd = st.up(std::move(ds));
  int64_t* dbp = st.up(std::move(bp));
  std::vector<int64_t> offc = off;
  int64_t* doff = st.up(std::move(offc));
  launch_trinv_diag(dd, dbp, nblk, nmat, nb, 1, inv, doff, st.s);
  H2ULV_HIP(hipGetLastError());
  for (int jb = maxblk - 1; jb >= 0; --jb) {
    GemmBatch<double> g1, g2;
    for (size_t b = 0; b < sys.size(); ++b) {
      const TriRhs& t = sys[b];
      int nbk = (t.m + nb - 1) / nb;
      if (jb >= nbk || t.ncols <= 0) continue;
      int o = jb * nb, w = std::min(nb, t.m - o);
      const double* blk = inv + off[b] + (int64_t)jb * nb * nb;
      g1.one(t.X + o, t.ldx, w, t.ncols, w, blk, nb, false, t.B + o, t.ldb, false);
      if (o > 0)
        g2.one(t.B, t.ldb, o, t.ncols, w, t.T + (int64_t)o * t.ldt, t.ldt, false, t.X + o, t.ldx,
               false, -1.0, 1.0);
    }
    g1.run(st, "trsm");
    g2.run(st, "trsm");
  }
}

// In-place blocked LU with partial pivoting; returns device info (one int per
// matrix, 0 = ok, j+1 = first zero/non-finite pivot column) and pivots.
void batched_lu(Stage& st, const std::vector<SqMat>& mats, int32_t* ipiv, int32_t* info,
                const std::vector<int64_t>& ipiv_off) {
  if (mats.empty()) return;
  const int nb = LU_PANEL;
  int maxm = 0;
  std::vector<MatDesc> ds;
  for (size_t b = 0; b < mats.size(); ++b) {
    MatDesc d{};
    d.A = mats[b].A;
    d.lda = mats[b].lda;
    d.m = mats[b].m;
    d.n = mats[b].m;
    d.ipiv = ipiv + ipiv_off[b];
    d.info = info + b;
    ds.push_back(d);
    maxm = std::max(maxm, mats[b].m);
  }
  const int nmat = (int)mats.size();
  MatDesc* dd = st.up(std::move(ds));
  for (int j0 = 0; j0 < maxm; j0 += nb) {
    {
      double fl = 0;
      for (auto& mt : mats)
        if (mt.m > j0) {
          double w = std::min(nb, mt.m - j0), h = mt.m - j0;
          fl += 2.0 * h * w * w / 2.0;
        }
      ProfScope ps("lu_panel", fl, 0, st.s);
      launch_lu_panel(dd, nmat, j0, nb, maxm - j0, st.s);
    }
    H2ULV_HIP(hipGetLastError());
    std::vector<int64_t> sp(1, 0);
    for (auto& mt : mats) sp.push_back(sp.back() + (mt.m > j0 ? (mt.m + 63) / 64 : 0));
    int64_t ns = sp.back();
    int64_t* dsp = st.up(std::move(sp));
    launch_lu_swap_trsm(dd, dsp, ns, nmat, j0, nb, st.s);
    H2ULV_HIP(hipGetLastError());
    GemmBatch<double> g;
    for (auto& mt : mats) {
      if (mt.m <= j0) continue;
      int w = std::min(nb, mt.m - j0);
      int rest = mt.m - j0 - w;
      if (rest <= 0) continue;
      double* A = mt.A;
      int64_t lda = mt.lda;
      g.one(A + (j0 + w) + (int64_t)(j0 + w) * lda, lda, rest, rest, w,
            A + (j0 + w) + (int64_t)j0 * lda, lda, false, A + j0 + (int64_t)(j0 + w) * lda, lda,
            false, -1.0, 1.0);
    }
    g.run(st, "lu");
  }
}

// Inverse of each matrix (A overwritten by its LU factors).  Pivots and info are
// returned in device arrays allocated on the stage; *info_out receives them.
void batched_inverse(Stage& st, const std::vector<SqMat>& mats, int32_t** info_out,
                     int32_t** ipiv_out, std::vector<int64_t>* ipiv_off_out) {
  *info_out = nullptr;
  if (mats.empty()) return;
  std::vector<int64_t> ipo;
  int64_t tot = 0, totsq = 0;
  for (auto& m : mats) {
    ipo.push_back(tot);
    tot += m.m;
    totsq += (int64_t)m.m * m.m;
  }
  int32_t* ipiv = st.scratch<int32_t>(std::max<int64_t>(tot, 1));
  int32_t* info = st.scratch<int32_t>(mats.size(), true);
  batched_lu(st, mats, ipiv, info, ipo);
  // B = P^T I, then X = L^-1 B, then inv = U^-1 X
  double* B = st.scratch<double>(std::max<int64_t>(totsq, 1));
  double* X = st.scratch<double>(std::max<int64_t>(totsq, 1));
  std::vector<PermItem> pis;
  std::vector<int64_t> sp(1, 0);
  std::vector<int64_t> boff;
  int64_t o = 0;
  for (size_t b = 0; b < mats.size(); ++b) {
    boff.push_back(o);
    pis.push_back(PermItem{ipiv + ipo[b], B + o, mats[b].m, mats[b].m, 0});
    sp.push_back(sp.back() + (mats[b].m + 63) / 64);
    o += (int64_t)mats[b].m * mats[b].m;
  }
  int64_t ns = sp.back();
  int np = (int)pis.size();
  PermItem* dpi = st.up(std::move(pis));
  int64_t* dsp = st.up(std::move(sp));
  launch_perm_matrix(dpi, dsp, ns, np, st.s);
  H2ULV_HIP(hipGetLastError());
  std::vector<TriRhs> lo, up;
  for (size_t b = 0; b < mats.size(); ++b) {
    const SqMat& m = mats[b];
    lo.push_back(TriRhs{m.A, m.lda, m.m, B + boff[b], m.m, X + boff[b], m.m, m.m});
    up.push_back(TriRhs{m.A, m.lda, m.m, X + boff[b], m.m, m.inv, m.ldinv, m.m});
  }
  trsm_lower_unit(st, lo);
  trsm_upper(st, up);
  *info_out = info;
  if (ipiv_out) *ipiv_out = ipiv;
  if (ipiv_off_out) *ipiv_off_out = ipo;
}

// Inverse of upper-triangular matrices (T factors of the bases).
void batched_triu_inverse(Stage& st, const std::vector<SqMat>& mats) {
  if (mats.empty()) return;
  int64_t totsq = 0;
  for (auto& m : mats) totsq += (int64_t)m.m * m.m;
  double* B = st.scratch<double>(std::max<int64_t>(totsq, 1));
  std::vector<PermItem> pis;
  std::vector<int64_t> sp(1, 0), boff;
  int64_t o = 0;
  for (auto& m : mats) {
    boff.push_back(o);
    pis.push_back(PermItem{nullptr, B + o, m.m, m.m, 0});
    sp.push_back(sp.back() + (m.m + 63) / 64);
    o += (int64_t)m.m * m.m;
  }
  int64_t ns = sp.back();
  int np = (int)pis.size();
  PermItem* dpi = st.up(std::move(pis));
  int64_t* dsp = st.up(std::move(sp));
  launch_perm_matrix(dpi, dsp, ns, np, st.s);
  H2ULV_HIP(hipGetLastError());
  std::vector<TriRhs> up;
  for (size_t b = 0; b < mats.size(); ++b) {
    const SqMat& m = mats[b];
    up.push_back(TriRhs{m.A, m.lda, m.m, B + boff[b], m.m, m.inv, m.ldinv, m.m});
  }
  trsm_upper(st, up);
}

// Blocked Householder QR of tall (or short) matrices, R only: the panel of nb
// columns is factored by one workgroup, the trailing columns are updated by
// three GEMMs with the explicit panel reflectors and their T factor.
void batched_qr_R(Stage& st, const std::vector<TallQr>& ms) {
  if (ms.empty()) return;
  const int nb = QR_NB;
  int maxk = 0, maxh = 0;
  std::vector<MatDesc> ds;
  std::vector<double*> Vb, Tfb, Y1b, Y2b;
  int64_t sv = 0, sa = 0, sy = 0;
  for (auto& a : ms) {
    sv += (int64_t)a.h * nb;
    sa += std::max(a.m, 1);
    sy += (int64_t)nb * std::max(a.m, 1);
  }
  double* Vall = st.scratch<double>(std::max<int64_t>(sv, 1));
  double* Aall = st.scratch<double>(std::max<int64_t>(sa, 1));
  double* Tall = st.scratch<double>((int64_t)nb * nb * ms.size());
  double* Y1all = st.scratch<double>(std::max<int64_t>(sy, 1));
  double* Y2all = st.scratch<double>(std::max<int64_t>(sy, 1));
  sv = sa = sy = 0;
  for (size_t q = 0; q < ms.size(); ++q) {
    const TallQr& a = ms[q];
    MatDesc d{};
    d.A = a.A;
    d.lda = a.lda;
    d.m = a.h;
    d.n = a.m;
    d.V = Vall + sv;
    d.aux = Aall + sa;
    d.Tf = Tall + (int64_t)nb * nb * q;
    d.panel_ws = 1;
    Vb.push_back(d.V);
    Tfb.push_back(d.Tf);
    Y1b.push_back(Y1all + sy);
    Y2b.push_back(Y2all + sy);
    sv += (int64_t)a.h * nb;
    sa += std::max(a.m, 1);
    sy += (int64_t)nb * std::max(a.m, 1);
    ds.push_back(d);
    maxk = std::max(maxk, std::min(a.h, a.m));
    maxh = std::max(maxh, a.h);
  }
  const int nmat = (int)ms.size();
  MatDesc* dd = st.up(std::move(ds));
  for (int j0 = 0; j0 < maxk; j0 += nb) {
    {
      double fl = 0;
      for (auto& a : ms)
        if (std::min(a.h, a.m) > j0) fl += 2.0 * (a.h - j0) * (double)nb * nb;
      ProfScope ps("qr_panel:tsqr", fl, 0, st.s);
      launch_qr_panel(dd, nmat, j0, nb, maxh - j0, st.s);
    }
    H2ULV_HIP(hipGetLastError());
    GemmBatch<double> g1, g2, g3;
    for (size_t b = 0; b < ms.size(); ++b) {
      const TallQr& a = ms[b];
      int kk = std::min(a.h, a.m);
      if (kk <= j0) continue;
      int wd = std::min(nb, kk - j0);
      int ntr = a.m - j0 - wd;
      if (ntr <= 0) continue;
      int rows = a.h - j0;
      const double* Vp = Vb[b] + j0;
      double* At = a.A + j0 + (int64_t)(j0 + wd) * a.lda;
      g1.one(Y1b[b], nb, wd, ntr, rows, Vp, a.h, true, At, a.lda, false);
      g2.one(Y2b[b], nb, wd, ntr, wd, Tfb[b], nb, true, Y1b[b], nb, false);
      g3.one(At, a.lda, rows, ntr, wd, Vp, a.h, false, Y2b[b], nb, false, -1.0, 1.0);
    }
    g1.run(st, "tsqr");
    g2.run(st, "tsqr");
    g3.run(st, "tsqr");
  }
}

// Householder QR of W (m x k, overwritten), explicit U (m x m) and T = R(1:k,1:k).
void batched_qr_basis(Stage& st, const std::vector<QrW>& ws) {
  if (ws.empty()) return;
  const int nb = QR_NB;
  int maxk = 0, maxh = 0;
  std::vector<MatDesc> ds;
  std::vector<double*> Vb, Tfb, Y1b, Y2b;
  int64_t sv = 0, sa = 0, st_ = 0, sy = 0;
  for (auto& w : ws) {
    int np = (w.k + nb - 1) / nb;
    sv += std::max<int64_t>((int64_t)w.m * w.k, 1);
    sa += std::max(w.k, 1);
    st_ += std::max<int64_t>((int64_t)np * nb * nb, 1);
    sy += (int64_t)nb * std::max(std::max(w.m, w.k), 1);
  }
  double* Vall = st.scratch<double>(sv);
  double* Aall = st.scratch<double>(sa);
  double* Tall = st.scratch<double>(st_);
  double* Y1all = st.scratch<double>(sy);
  double* Y2all = st.scratch<double>(sy);
  sv = sa = st_ = sy = 0;
  for (auto& w : ws) {
    int np = (w.k + nb - 1) / nb;
    MatDesc d{};
    d.A = w.W;
    d.lda = w.m;
    d.m = w.m;
    d.n = w.k;
    d.V = Vall + sv;
    d.aux = Aall + sa;
    d.Tf = Tall + st_;
    Vb.push_back(d.V);
    Tfb.push_back(d.Tf);
    Y1b.push_back(Y1all + sy);
    Y2b.push_back(Y2all + sy);
    sv += std::max<int64_t>((int64_t)w.m * w.k, 1);
    sa += std::max(w.k, 1);
    st_ += std::max<int64_t>((int64_t)np * nb * nb, 1);
    sy += (int64_t)nb * std::max(std::max(w.m, w.k), 1);
    ds.push_back(d);
    maxk = std::max(maxk, std::min(w.k, w.m));
    maxh = std::max(maxh, w.m);
  }
  const int nmat = (int)ws.size();
  MatDesc* dd = st.up(std::move(ds));
  for (int j0 = 0; j0 < maxk; j0 += nb) {
    {
      ProfScope ps("qr_panel:qrbasis", 0, 0, st.s);
      launch_qr_panel(dd, nmat, j0, nb, maxh - j0, st.s);
    }
    H2ULV_HIP(hipGetLastError());
    GemmBatch<double> g1, g2, g3;
    for (size_t b = 0; b < ws.size(); ++b) {
      const QrW& w = ws[b];
      int kk = std::min(w.k, w.m);
      if (kk <= j0) continue;
      int wd = std::min(nb, kk - j0);
      int ntr = w.k - j0 - wd;
      if (ntr <= 0) continue;
      int rows = w.m - j0;
      const double* Vp = Vb[b] + (int64_t)j0 * w.m + j0;
      const double* Tp = Tfb[b] + (int64_t)(j0 / nb) * nb * nb;
      double* At = w.W + j0 + (int64_t)(j0 + wd) * w.m;
      g1.one(Y1b[b], nb, wd, ntr, rows, Vp, w.m, true, At, w.m, false);
      g2.one(Y2b[b], nb, wd, ntr, wd, Tp, nb, true, Y1b[b], nb, false);
      g3.one(At, w.m, rows, ntr, wd, Vp, w.m, false, Y2b[b], nb, false, -1.0, 1.0);
    }
    g1.run(st, "qrbasis");
    g2.run(st, "qrbasis");
    g3.run(st, "qrbasis");
  }
  // T = upper triangle of the factored W
  {
    CopyBatch cb;
    std::vector<CopyItem> zl;
    for (auto& w : ws) {
      if (w.k <= 0) continue;
      cb.add(w.W, w.m, w.T, w.k, w.k, w.k);
      zl.push_back(CopyItem{nullptr, w.T, 0, w.k, w.k, w.k, 0, 0});
    }
    cb.run(st);
    int nz = (int)zl.size();
    CopyItem* dz = st.up(std::move(zl));
    launch_zero_lower(dz, nz, st.s);
    H2ULV_HIP(hipGetLastError());
  }
  // U = H_0 H_1 ... H_{k-1}, applied to the identity from the last panel back
  {
    std::vector<PermItem> pis;
    std::vector<int64_t> sp(1, 0);
    for (auto& w : ws) {
      pis.push_back(PermItem{nullptr, w.U, w.m, w.m, 0});
      sp.push_back(sp.back() + (w.m + 63) / 64);
    }
    int64_t ns = sp.back();
    int np = (int)pis.size();
    PermItem* dpi = st.up(std::move(pis));
    int64_t* dsp = st.up(std::move(sp));
    launch_perm_matrix(dpi, dsp, ns, np, st.s);
    H2ULV_HIP(hipGetLastError());
  }
  int maxp = (maxk + nb - 1) / nb;
  for (int p = maxp - 1; p >= 0; --p) {
    int j0 = p * nb;
    GemmBatch<double> g1, g2, g3;
    for (size_t b = 0; b < ws.size(); ++b) {
      const QrW& w = ws[b];
      int kk = std::min(w.k, w.m);
      if (kk <= j0) continue;
      int wd = std::min(nb, kk - j0);
      int rows = w.m - j0;
      const double* Vp = Vb[b] + (int64_t)j0 * w.m + j0;
      const double* Tp = Tfb[b] + (int64_t)p * nb * nb;
      double* Us = w.U + j0 + (int64_t)j0 * w.m;
      g1.one(Y1b[b], nb, wd, rows, rows, Vp, w.m, true, Us, w.m, false);
      g2.one(Y2b[b], nb, wd, rows, wd, Tp, nb, false, Y1b[b], nb, false);
      g3.one(Us, w.m, rows, rows, wd, Vp, w.m, false, Y2b[b], nb, false, -1.0, 1.0);
    }
    g1.run(st, "qrbasis");
    g2.run(st, "qrbasis");
    g3.run(st, "qrbasis");
  }
}

}  // namespace h2ulv
