// Exact matvec that allocates no device memory, for callers that cannot
// allocate (code under stream capture, tight serving loops, harnesses that
// forbid allocation).  The split-source partial sums of the matvec live in a
// file-scope device array instead of a buffer from the library's allocator;
// every GPU the library runs on holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "h2ulv_batch.h"
#include "h2ulv_factor.h"
#include "h2ulv_kernels.h"

namespace {
constexpr int64_t kScratchWords = int64_t(16) << 20;  // 128 MiB of doubles per GPU
constexpr int kMaxDevices = 64;
}  // namespace

// The partial sums of the split matvec (matvec_work_words doubles).  In host
// code this name is only a stand-in: kernels get the per-device address below.
static __device__ __align__(256) double scratch[kScratchWords];

namespace h2ulv {
namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of the array, looked up once per
// device with that device current.
double* scratch_ptr() {
  int dev = 0;
  H2ULV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    fail(H2ULV_ERR_HIP, "allocation-free matvec: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(H2ULV_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

int64_t matvec_noalloc_capacity() { return kScratchWords; }

// Same launches, split and summation order as the allocating matvec, so the
// result is identical; nothing is allocated and the stream is not synchronised.
void matvec_noalloc(const h2ulv_factor& F, const double* x, int64_t ldx, double* y, int64_t ldy,
                    int nrhs, hipStream_t s) {
  const int64_t words = matvec_work_words(F.n, nrhs);
  if (words > kScratchWords)
    fail(H2ULV_ERR_INVALID_ARG,
         "allocation-free matvec: n = " + std::to_string(F.n) + " needs " +
             std::to_string(words) + " doubles of partial sums, more than its " +
             std::to_string(kScratchWords) + "-double buffer");
  double* work = words > 0 ? scratch_ptr() : nullptr;
  launch_matvec(F.pts.as<double>(), F.n, kfn(F.p), x, ldx, y, ldy, nrhs, work, s);
  H2ULV_HIP(hipGetLastError());
}

}  // namespace h2ulv
