// Host-side batching helpers: device buffers, staged uploads and the batched
// launch builders used by the level driver (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "h2ulv_internal.h"
#include "h2ulv_kernels.h"

namespace h2ulv {

#define H2ULV_HIP(x)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) fail(H2ULV_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device-memory accounting shared by every buffer of the process.
struct MemStats {
  size_t live = 0, peak = 0;
};
MemStats& mem_stats();

// Caching device allocator.  hipMalloc can stall for hundreds of milliseconds
// while earlier work is queued, and hipFree of many blocks costs as much, so
// freed blocks are kept and handed out again.  All device work of one call is
// ordered on one stream, so a block freed by a buffer and reused by a later
// buffer of the same call is only touched after the earlier work in stream
// order; every call synchronises its stream before it returns, so blocks kept
// across calls are idle.  The cache is handed back to the runtime when growing
// would eat into a free-memory reserve, after a failed hipMalloc, when a call
// fails (CacheScope), and on h2ulv_release_cache; every release waits for the
// device first.
void* cache_alloc(size_t bytes, size_t* got);
void cache_free(void* p, size_t bytes);
void cache_release();
size_t cache_bytes();
int64_t cache_oom_releases();
// Free device memory as seen by the library: hipMemGetInfo plus cached blocks.
size_t free_device_bytes();
// Pinned host staging buffers, kept for reuse (hipHostMalloc pins pages and is
// slow); a buffer goes back only after the work that reads it has finished.
char* pinned_get(size_t bytes, size_t* got);
void pinned_put(char* p, size_t bytes);
struct CacheScope {
  CacheScope();
  ~CacheScope();
};

// Per-kernel launch timing with HIP events recorded on the launch stream
// (enabled through h2ulv_profile_enable).
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  double flops, bytes;
};
struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  // the work of the last record of a scope, once it is known (after the launch)
  void amend_last(const char* name, double flops, double bytes) {
    for (auto it = recs.rbegin(); it != recs.rend(); ++it)
      if (std::strcmp(it->name, name) == 0) {
        it->flops = flops;
        it->bytes = bytes;
        return;
      }
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
};
Profiler& profiler();
// Stable name "<kernel>:<site>" for profile records.
const char* profile_name(const char* kernel, const char* site);

// RAII scope: records a start event now and a stop event when destroyed.
struct ProfScope {
  Profiler* p = nullptr;
  ProfRec r{};
  hipStream_t s;
  ProfScope(const char* name, double flops, double bytes, hipStream_t st) : s(st) {
    Profiler& pr = profiler();
    if (!pr.on) return;
    // work recorded into a graph is timed where the graph is launched
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone) return;
    p = &pr;
    r.name = name;
    r.flops = flops;
    r.bytes = bytes;
    r.a = pr.ev();
    r.b = pr.ev();
    (void)hipEventRecord(r.a, s);
  }
  ~ProfScope() {
    if (!p) return;
    (void)hipEventRecord(r.b, s);
    p->recs.push_back(r);
  }
};

// The caller's device allocator of the running call (thread-local; unset: the
// caching allocator above).  A buffer keeps the allocator it came from and
// gives its block back to it.
struct AllocHook {
  h2ulv_allocator a{};
  void* stream = nullptr;
  bool set = false;
};
AllocHook& current_alloc_hook();
struct AllocScope {
  AllocHook prev;
  AllocScope(const h2ulv_allocator* a, void* stream) : prev(current_alloc_hook()) {
    AllocHook& h = current_alloc_hook();
    h.set = a != nullptr;
    if (a) h.a = *a;
    h.stream = stream;
  }
  ~AllocScope() { current_alloc_hook() = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

// Owning device buffer: from the caller's allocator when one is installed,
// else from the caching allocator.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;  // requested size
  size_t cap = 0;    // size of the block behind it
  AllocHook hook;    // where the block came from (hook.set: the caller's allocator)
  DBuf() = default;
  explicit DBuf(size_t b) { alloc(b); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap), hook(o.hook) {
    o.p = nullptr;
    o.bytes = 0;
    o.cap = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      cap = o.cap;
      hook = o.hook;
      o.p = nullptr;
      o.bytes = 0;
      o.cap = 0;
    }
    return *this;
  }
  ~DBuf() { reset(); }
  void alloc(size_t b) {
    reset();
    if (b == 0) return;
    hook = current_alloc_hook();
    if (hook.set) {
      p = hook.a.alloc(hook.a.ctx, b, hook.stream);
      if (!p)
        fail(H2ULV_ERR_OOM,
             "the caller's allocator returned NULL for " + std::to_string(b) + " bytes");
      cap = b;
    } else {
      p = cache_alloc(b, &cap);
    }
    bytes = b;
    MemStats& ms = mem_stats();
    ms.live += b;
    ms.peak = std::max(ms.peak, ms.live);
  }
  void reset() {
    if (p) {
      if (hook.set)
        hook.a.free(hook.a.ctx, p, hook.stream);
      else
        cache_free(p, cap);
      mem_stats().live -= bytes;
    }
    p = nullptr;
    bytes = 0;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Pinned host staging + device memory for launch descriptors: uploads are
// appended to the current chunk (256-byte aligned) and copied asynchronously;
// chunks are recycled at the next synchronisation.
struct DescArena {
  struct Chunk {
    char* host = nullptr;
    DBuf dev;
    size_t cap = 0, used = 0;
  };
  std::vector<Chunk> chunks;
  ~DescArena() {
    for (auto& c : chunks)
      if (c.host) pinned_put(c.host, c.cap);
  }
  void* put(const void* src, size_t bytes, hipStream_t s) {
    size_t need = (bytes + 255) & ~(size_t)255;
    Chunk* c = nullptr;
    for (auto& ch : chunks)
      if (ch.cap - ch.used >= need) {
        c = &ch;
        break;
      }
    if (!c) {
      Chunk nc;
      nc.host = pinned_get(std::max<size_t>(need, (size_t)32 << 20), &nc.cap);
      nc.dev.alloc(nc.cap);
      chunks.push_back(std::move(nc));
      c = &chunks.back();
    }
    char* h = c->host + c->used;
    char* d = c->dev.as<char>() + c->used;
    std::memcpy(h, src, bytes);
    c->used += need;
    H2ULV_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
    return d;
  }
  // several arrays in one region and one copy; dev[i] receives part i's address
  void put_parts(const void* const* src, const size_t* bytes, int nparts, void** dev,
                 hipStream_t s) {
    size_t off[8];
    size_t tot = 0;
    for (int i = 0; i < nparts; ++i) {
      off[i] = tot;
      tot += (bytes[i] + 255) & ~(size_t)255;
    }
    if (tot == 0) {
      for (int i = 0; i < nparts; ++i) dev[i] = nullptr;
      return;
    }
    Chunk* c = nullptr;
    for (auto& ch : chunks)
      if (ch.cap - ch.used >= tot) {
        c = &ch;
        break;
      }
    if (!c) {
      Chunk nc;
      nc.host = pinned_get(std::max<size_t>(tot, (size_t)32 << 20), &nc.cap);
      nc.dev.alloc(nc.cap);
      chunks.push_back(std::move(nc));
      c = &chunks.back();
    }
    char* h = c->host + c->used;
    char* d = c->dev.as<char>() + c->used;
    for (int i = 0; i < nparts; ++i) {
      if (bytes[i]) std::memcpy(h + off[i], src[i], bytes[i]);
      dev[i] = bytes[i] ? d + off[i] : nullptr;
    }
    c->used += tot;
    H2ULV_HIP(hipMemcpyAsync(d, h, tot, hipMemcpyHostToDevice, s));
  }
  void recycle() {
    for (auto& c : chunks) c.used = 0;
  }
};

// Uploads and scratch buffers that must live until the stream is synchronised.
struct Stage {
  hipStream_t s = nullptr;
  std::vector<DBuf> bufs;
  std::vector<std::shared_ptr<void>> host;
  DescArena desc;
  // replay mode (graph capture): the same sequence of requests as a first pass
  // gets that pass's scratch buffers and descriptor offsets back, so nothing is
  // allocated while the stream captures
  bool replay = false;
  size_t next = 0;
  explicit Stage(hipStream_t st) : s(st) {}
  void begin_replay() {
    replay = true;
    next = 0;
    desc.recycle();
  }
  template <class T>
  T* up(std::vector<T>&& v) {
    if (v.empty()) return nullptr;
    return static_cast<T*>(desc.put(v.data(), v.size() * sizeof(T), s));
  }
  template <class T>
  T* up(const std::vector<T>& v) {
    return up(std::vector<T>(v));
  }
  // two or three arrays in one copy
  template <class A, class B>
  void up2(const std::vector<A>& a, const std::vector<B>& b, A** da, B** db) {
    const void* src[2] = {a.data(), b.data()};
    const size_t by[2] = {a.size() * sizeof(A), b.size() * sizeof(B)};
    void* dv[2];
    desc.put_parts(src, by, 2, dv, s);
    *da = static_cast<A*>(dv[0]);
    *db = static_cast<B*>(dv[1]);
  }
  template <class A, class B, class C>
  void up3(const std::vector<A>& a, const std::vector<B>& b, const std::vector<C>& c, A** da,
           B** db, C** dc) {
    const void* src[3] = {a.data(), b.data(), c.data()};
    const size_t by[3] = {a.size() * sizeof(A), b.size() * sizeof(B), c.size() * sizeof(C)};
    void* dv[3];
    desc.put_parts(src, by, 3, dv, s);
    *da = static_cast<A*>(dv[0]);
    *db = static_cast<B*>(dv[1]);
    *dc = static_cast<C*>(dv[2]);
  }
  template <class T>
  T* scratch(size_t count, bool zero = false) {
    if (count == 0) return nullptr;
    if (replay) {
      if (zero || next >= bufs.size() || bufs[next].bytes < count * sizeof(T))
        fail(H2ULV_ERR_HIP, "internal: replayed stage differs from its first pass");
      return bufs[next++].as<T>();
    }
    DBuf b(count * sizeof(T));
    if (zero) H2ULV_HIP(hipMemsetAsync(b.p, 0, count * sizeof(T), s));
    bufs.push_back(std::move(b));
    return bufs.back().as<T>();
  }
  void sync() {
    H2ULV_HIP(hipStreamSynchronize(s));
    bufs.clear();
    host.clear();
    desc.recycle();
  }
  ~Stage() {
    // the descriptor arena and scratch buffers may still be read by queued work
    (void)hipStreamSynchronize(s);
  }
};

inline int64_t tiles64(int64_t m, int64_t n) { return ((m + 63) / 64) * ((n + 63) / 64); }
inline int64_t tiles_of(int64_t m, int64_t n, int t) { return ((m + t - 1) / t) * ((n + t - 1) / t); }

// Full-tile rates (TFLOP/s) of the GEMM tile shapes on the current device,
// measured the first time a precision is used on a device (autotuning: a
// synthetic batch of 256 x 256 products in every shape, timed with events) and
// kept for the process.  f64: 64x64, 64x128, 128x64, 128x128; f32: 64x64,
// 128x128.
const double* gemm_tile_rates(bool f64, hipStream_t s);
// The rates measured so far on the current device (0 where not yet measured):
// f64 x 4 then f32 x 2.  Returns false when nothing has been measured.
bool gemm_tile_rates_known(double* out6);

// TI: operand type (MFMA precision), TC: type of the result C.
template <typename T, typename TC = T>
struct GemmBatch {
  std::vector<GemmItem<TC>> items;
  std::vector<GemmTerm<T>> terms;
  void item(TC* C, int64_t ldc, int M, int N, double alpha = 1.0, double beta = 0.0) {
    GemmItem<TC> it;
    it.C = C;
    it.ldc = ldc;
    it.M = M;
    it.N = N;
    it.t0 = (int32_t)terms.size();
    it.nt = 0;
    it.alpha = alpha;
    it.beta = beta;
    items.push_back(it);
  }
  void term(const T* A, int64_t lda, bool ta, const T* B, int64_t ldb, bool tb, int K) {
    GemmTerm<T> t;
    t.A = A;
    t.B = B;
    t.lda = lda;
    t.ldb = ldb;
    t.K = K;
    t.flags = (ta ? 1 : 0) | (tb ? 2 : 0);
    terms.push_back(t);
    items.back().nt++;
  }
  // C = alpha op(A) op(B) + beta C
  void one(TC* C, int64_t ldc, int M, int N, int K, const T* A, int64_t lda, bool ta, const T* B,
           int64_t ldb, bool tb, double alpha = 1.0, double beta = 0.0) {
    item(C, ldc, M, N, alpha, beta);
    term(A, lda, ta, B, ldb, tb, K);
  }
  bool empty() const { return items.empty(); }
  // site: label of the call site in the kernel profile ("gemm_f64:<site>")
  void run(Stage& st, const char* site = "other") {
    std::vector<GemmItem<TC>> its;
    its.reserve(items.size());
    for (auto& it : items)
      if (it.M > 0 && it.N > 0) its.push_back(it);
    items.clear();
    if (its.empty()) {
      terms.clear();
      return;
    }
    // products with at most GEMV_MAXN columns (the solve's right-hand sides)
    // are matrix-vector work: vector units, A read once, no MFMA tiles
    if constexpr (sizeof(T) == 8 && sizeof(TC) == 8) {
      int maxN = 0;
      bool btrans = false;
      for (auto& it : its) maxN = std::max(maxN, it.N);
      for (auto& tt : terms) btrans = btrans || (tt.flags & 2) != 0;
      if (maxN <= GEMV_MAXN && !btrans) {
        run_gemv(st, its, site);
        return;
      }
    }
    // tile shape: 32 x 128 when every item has at most 32 rows (Householder
    // V^T A products); otherwise the shape with the best estimated rate, i.e.
    // the measured rate of the shape on full tiles (gfx950, TFLOP/s) times the
    // useful fraction of its padded tiles, scaled down when the batch has fewer
    // tiles than the chip has resident workgroup slots for that shape
    struct Shape {
      int tm, tn;
      double rate;
      int per_cu;  // resident workgroups per CU
    };
    Shape f64s[4] = {{64, 64, 0, 4}, {64, 128, 0, 3}, {128, 64, 0, 3}, {128, 128, 0, 2}};
    Shape f32s[2] = {{64, 64, 0, 8}, {128, 128, 0, 3}};
    Shape* cand = sizeof(T) == 8 ? f64s : f32s;
    const int ncand = sizeof(T) == 8 ? 4 : 2;
    {
      const double* rt = gemm_tile_rates(sizeof(T) == 8, st.s);
      for (int c = 0; c < ncand; ++c) cand[c].rate = rt[c];
    }
    int maxM = 0;
    std::vector<double> ksum(its.size(), 0.0);
    for (size_t i = 0; i < its.size(); ++i) {
      maxM = std::max(maxM, its[i].M);
      for (int t = its[i].t0; t < its[i].t0 + its[i].nt; ++t) ksum[i] += terms[t].K;
    }
    int tm = 64, tn = 64;
    if (maxM <= 32) {
      tm = 32;
      tn = 128;
    } else {
      double best = -1.0;
      for (int c = 0; c < ncand; ++c) {
        double useful = 0, padded = 0;
        int64_t nt = 0;
        for (size_t i = 0; i < its.size(); ++i) {
          const int64_t a = (its[i].M + cand[c].tm - 1) / cand[c].tm;
          const int64_t b = (its[i].N + cand[c].tn - 1) / cand[c].tn;
          nt += a * b;
          const double kk = std::max(ksum[i], 1.0);
          useful += (double)its[i].M * its[i].N * kk;
          padded += (double)(a * cand[c].tm) * (b * cand[c].tn) * kk;
        }
        const double fill = std::min(1.0, (double)nt / (256.0 * cand[c].per_cu));
        const double score = cand[c].rate * (useful / padded) * fill;
        if (score > best) {
          best = score;
          tm = cand[c].tm;
          tn = cand[c].tn;
        }
      }
    }
    auto ntile = [&](const GemmItem<TC>& it) {
      return (int64_t)((it.M + tm - 1) / tm) * ((it.N + tn - 1) / tn);
    };
    // the split-K decision depends on the batch alone (counted in 64 x 64 tiles),
    // not on the tuned tile shape, so the summation order is fixed by the batch
    int64_t nt64 = 0;
    double kmax = 0;
    for (size_t i = 0; i < its.size(); ++i) {
      nt64 += tiles64(its[i].M, its[i].N);
      kmax = std::max(kmax, ksum[i]);
    }
    double fl = 0, by = 0;
    if (profiler().on) {
      for (auto& it : its)
        for (int t = it.t0; t < it.t0 + it.nt; ++t) {
          double K = terms[t].K;
          fl += 2.0 * it.M * it.N * K;
          by += ((double)it.M * K + K * it.N) * sizeof(T);
        }
      for (auto& it : its) by += (double)it.M * it.N * sizeof(TC) * (it.beta != 0.0 ? 2 : 1);
    }
    // split K over workgroups when the batch has few tiles and long sums: split
    // s of item i writes its partial product into scratch (beta 0) and a
    // reduction adds the partials in order into C with alpha and beta
    int S = 1;
    if (nt64 < 1024 && kmax >= 512) {
      S = (int)std::min<int64_t>(8, std::max<int64_t>(1, 2048 / std::max<int64_t>(nt64, 1)));
      S = (int)std::min<double>(S, std::floor(kmax / 256.0));
    }
    std::vector<SplitKItem<TC>> red;
    if (S >= 2) {
      int64_t pw = 0;
      for (auto& it : its) pw += (int64_t)it.M * it.N * S;
      TC* part = st.scratch<TC>(pw);
      std::vector<GemmItem<TC>> sits;
      std::vector<GemmTerm<T>> sterms;
      int64_t po = 0;
      for (size_t i = 0; i < its.size(); ++i) {
        const GemmItem<TC>& it = its[i];
        const int64_t mn = (int64_t)it.M * it.N;
        red.push_back(SplitKItem<TC>{it.C, it.ldc, part + po, it.M, it.N, S, it.alpha, it.beta});
        // K range [s * chunk, (s + 1) * chunk) of the item's concatenated terms
        const int64_t kt = (int64_t)ksum[i];
        const int64_t chunk = ((kt + S - 1) / S + 15) / 16 * 16;
        for (int sp = 0; sp < S; ++sp) {
          GemmItem<TC> ni_ = it;
          ni_.C = part + po + sp * mn;
          ni_.ldc = it.M;
          ni_.alpha = 1.0;
          ni_.beta = 0.0;
          ni_.t0 = (int32_t)sterms.size();
          ni_.nt = 0;
          const int64_t lo = sp * chunk, hi = std::min(kt, lo + chunk);
          int64_t base = 0;
          for (int t = it.t0; t < it.t0 + it.nt; ++t) {
            const GemmTerm<T>& tt = terms[t];
            const int64_t a0 = std::max(lo, base), a1 = std::min(hi, base + tt.K);
            if (a1 > a0) {
              const int64_t k0 = a0 - base;
              GemmTerm<T> st_ = tt;
              st_.K = (int32_t)(a1 - a0);
              st_.A = (tt.flags & 1) ? tt.A + k0 : tt.A + k0 * tt.lda;
              st_.B = (tt.flags & 2) ? tt.B + k0 * tt.ldb : tt.B + k0;
              sterms.push_back(st_);
              ni_.nt++;
            }
            base += tt.K;
          }
          sits.push_back(ni_);
        }
        po += mn * S;
      }
      its.swap(sits);
      terms.swap(sterms);
    }
    std::vector<int64_t> tp(its.size() + 1, 0);
    for (size_t i = 0; i < its.size(); ++i) tp[i + 1] = tp[i] + ntile(its[i]);
    int64_t nt = tp.back();
    int ni = (int)its.size();
    GemmItem<TC>* di;
    GemmTerm<T>* dt;
    int64_t* dp;
    st.up3(its, terms, tp, &di, &dt, &dp);
    terms.clear();
    ProfScope ps(profiler().on ? profile_name(sizeof(T) == 8 ? "gemm_f64" : "gemm_f32", site)
                               : "",
                 fl, by, st.s);
    launch_gemm<T, TC>(di, dt, dp, nt, ni, tm, tn, st.s);
    H2ULV_HIP(hipGetLastError());
    if (!red.empty()) {
      std::vector<int64_t> rp(red.size() + 1, 0);
      for (size_t i = 0; i < red.size(); ++i) rp[i + 1] = rp[i] + tiles64(red[i].M, red[i].N);
      SplitKItem<TC>* dr;
      int64_t* drp;
      st.up2(red, rp, &dr, &drp);
      launch_splitk_reduce<TC>(dr, drp, rp.back(), (int)red.size(), st.s);
      H2ULV_HIP(hipGetLastError());
    }
  }
  // Few-column products on gemv_kernel (64-row tiles).  Long sums are split
  // over up to 64 workgroups per tile (about 2048 workgroups in all, chunks of
  // at least 512), the partial products added in order by the split-K
  // reduction.
  void run_gemv(Stage& st, std::vector<GemmItem<TC>>& its, const char* site) {
    std::vector<double> ksum(its.size(), 0.0);
    double kmax = 0;
    int64_t nt0 = 0;
    for (size_t i = 0; i < its.size(); ++i) {
      for (int t = its[i].t0; t < its[i].t0 + its[i].nt; ++t) ksum[i] += terms[t].K;
      kmax = std::max(kmax, ksum[i]);
      nt0 += (its[i].M + 63) / 64;
    }
    double fl = 0, by = 0;
    if (profiler().on) {
      for (auto& it : its) {
        for (int t = it.t0; t < it.t0 + it.nt; ++t) {
          const double K = terms[t].K;
          fl += 2.0 * it.M * it.N * K;
          by += ((double)it.M * K + K * it.N) * sizeof(T);
        }
        by += (double)it.M * it.N * sizeof(TC) * (it.beta != 0.0 ? 2 : 1);
      }
    }
    int S = 1;
    if (nt0 < 2048 && kmax >= 1024) {
      const double want = std::ceil(2048.0 / (double)std::max<int64_t>(nt0, 1));
      S = (int)std::min(64.0, std::min(want, std::floor(kmax / 512.0)));
      S = std::max(S, 1);
    }
    std::vector<SplitKItem<TC>> red;
    if (S >= 2) {
      int64_t pw = 0;
      for (auto& it : its) pw += (int64_t)it.M * it.N * S;
      TC* part = st.scratch<TC>(pw);
      std::vector<GemmItem<TC>> sits;
      std::vector<GemmTerm<T>> sterms;
      int64_t po = 0;
      for (size_t i = 0; i < its.size(); ++i) {
        const GemmItem<TC>& it = its[i];
        const int64_t mn = (int64_t)it.M * it.N;
        red.push_back(SplitKItem<TC>{it.C, it.ldc, part + po, it.M, it.N, S, it.alpha, it.beta});
        const int64_t kt = (int64_t)ksum[i];
        const int64_t chunk = std::max<int64_t>(1, (kt + S - 1) / S);
        for (int sp = 0; sp < S; ++sp) {
          GemmItem<TC> ni_ = it;
          ni_.C = part + po + sp * mn;
          ni_.ldc = it.M;
          ni_.alpha = 1.0;
          ni_.beta = 0.0;
          ni_.t0 = (int32_t)sterms.size();
          ni_.nt = 0;
          const int64_t lo = sp * chunk, hi = std::min(kt, lo + chunk);
          int64_t base = 0;
          for (int t = it.t0; t < it.t0 + it.nt; ++t) {
            const GemmTerm<T>& tt = terms[t];
            const int64_t a0 = std::max(lo, base), a1 = std::min(hi, base + tt.K);
            if (a1 > a0) {
              const int64_t k0 = a0 - base;
              GemmTerm<T> st_ = tt;
              st_.K = (int32_t)(a1 - a0);
              st_.A = (tt.flags & 1) ? tt.A + k0 : tt.A + k0 * tt.lda;
              st_.B = tt.B + k0;  // B is not transposed here
              sterms.push_back(st_);
              ni_.nt++;
            }
            base += tt.K;
          }
          sits.push_back(ni_);
        }
        po += mn * S;
      }
      its.swap(sits);
      terms.swap(sterms);
    }
    std::vector<int64_t> tp(its.size() + 1, 0);
    for (size_t i = 0; i < its.size(); ++i) tp[i + 1] = tp[i] + (its[i].M + 63) / 64;
    GemmItem<TC>* di;
    GemmTerm<T>* dt;
    int64_t* dp;
    st.up3(its, terms, tp, &di, &dt, &dp);
    terms.clear();
    ProfScope ps(profiler().on ? profile_name("gemv_f64", site) : "", fl, by, st.s);
    launch_gemv(di, dt, dp, tp.back(), (int)its.size(), st.s);
    H2ULV_HIP(hipGetLastError());
    if (!red.empty()) {
      std::vector<int64_t> rp(red.size() + 1, 0);
      for (size_t i = 0; i < red.size(); ++i) rp[i + 1] = rp[i] + tiles64(red[i].M, red[i].N);
      SplitKItem<TC>* dr;
      int64_t* drp;
      st.up2(red, rp, &dr, &drp);
      launch_splitk_reduce<TC>(dr, drp, rp.back(), (int)red.size(), st.s);
      H2ULV_HIP(hipGetLastError());
    }
  }
};

struct KgenBatch {
  std::vector<KgenItem> items;
  // tr: entries of the transposed kernel K(x[cols], x[rows]) (the column side
  // of a nonsymmetric matrix)
  void add(const int64_t* rows, int m, const int64_t* cols, int n, double* out, int64_t ld,
           bool tr = false) {
    if (m <= 0 || n <= 0) return;
    items.push_back(KgenItem{rows, cols, out, ld, m, n, tr ? 1 : 0, 0});
  }
  void run(Stage& st, const double* pts, const KernelFn& kf, int* dup) {
    if (items.empty()) return;
    std::vector<int64_t> tp(items.size() + 1, 0);
    for (size_t i = 0; i < items.size(); ++i) tp[i + 1] = tp[i] + tiles64(items[i].m, items[i].n);
    int64_t nt = tp.back();
    int ni = (int)items.size();
    double ev = 0;
    for (auto& it : items) ev += (double)it.m * it.n;
    KgenItem* di;
    int64_t* dp;
    st.up2(items, tp, &di, &dp);
    items.clear();
    ProfScope ps("kgen", ev, ev * 8.0, st.s);
    launch_kgen(di, dp, nt, ni, pts, kf, dup, st.s);
    H2ULV_HIP(hipGetLastError());
  }
};

struct CopyBatch {
  std::vector<CopyItem> items;
  void add(const double* src, int64_t lds, double* dst, int64_t ldd, int rows, int cols,
           bool trans = false) {
    if (rows <= 0 || cols <= 0) return;
    items.push_back(CopyItem{src, dst, lds, ldd, rows, cols, trans ? 1 : 0, 0});
  }
  void run(Stage& st, double alpha = 1.0, double beta = 0.0) {
    if (items.empty()) return;
    std::vector<int64_t> tp(items.size() + 1, 0);
    for (size_t i = 0; i < items.size(); ++i)
      tp[i + 1] = tp[i] + tiles64(items[i].rows, items[i].cols);
    int64_t nt = tp.back();
    int ni = (int)items.size();
    double by = 0;
    for (auto& it : items) by += 16.0 * it.rows * it.cols;
    CopyItem* di;
    int64_t* dp;
    st.up2(items, tp, &di, &dp);
    items.clear();
    ProfScope ps("copy", 0, by, st.s);
    launch_copy(di, dp, nt, ni, alpha, beta, st.s);
    H2ULV_HIP(hipGetLastError());
  }
};

}  // namespace h2ulv
