// lp_orth_noalloc: the batched orth of lp_orth without a problem and without
// any allocation, for callers that cannot allocate (code being captured into a
// HIP graph, tight serving loops).  Its scratch -- the Gram partials of both
// CholeskyQR passes, the first pass's Q and the triangular factors -- lives in
// one file-scope device array, `scratch`, of kScratchBytes; each GPU holds its
// own copy of it from the first call on that device until the process ends,
// and every call on a GPU shares that copy (calls that overlap on one GPU race).
// Nothing in the scratch needs to start at zero: every kernel writes the
// partials and factors it later reads.
#include <mutex>
#include <string>

#include "lp_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // 16 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};   // device address of `scratch` on each device (set once)

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of scratch a batch needs: two Gram-partial buffers, the intermediate Q
// and the factors (the layout cholqr2_passes reads and writes).
size_t need_bytes(int batch, int64_t d, int k) {
  const size_t nch = (size_t)((d + lp::kGramRows - 1) / lp::kGramRows);
  const size_t kk = (size_t)k * k;
  return 2 * up256((size_t)batch * nch * kk * 8) + up256((size_t)batch * d * k * 8) +
         up256((size_t)batch * 2 * kk * 8);
}

// The device address of `scratch` on the current device (hipGetSymbolAddress on
// the first call per device; the array's name is not a device address in host code).
hipError_t scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = (char*)p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" lp_status lp_orth_noalloc(int32_t k, int32_t batch, int64_t d, const double* Y,
                                     double* Q, int32_t* flags, void* stream) {
  if (Y == nullptr || Q == nullptr) return lp::report(LP_EINVAL, "Y and Q are required");
  if (k < 1 || k > lp::kMaxK || d < k || batch < 1)
    return lp::report(LP_EINVAL, "need 1 <= k <= min(d, 64) and batch >= 1");
  const size_t need = need_bytes(batch, d, k);
  if (need > kScratchBytes)
    return lp::report(LP_EINVAL, "batch x d x k too large for the 16 MiB static scratch (needs " +
                                     std::to_string(need) + " bytes)");
  char* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return lp::report(LP_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  const size_t nch = (size_t)((d + lp::kGramRows - 1) / lp::kGramRows);
  const size_t kk = (size_t)k * k;
  const int64_t dk = d * k;
  double* gram = (double*)base;
  double* gram2 = (double*)(base + up256((size_t)batch * nch * kk * 8));
  double* tmp = (double*)((char*)gram2 + up256((size_t)batch * nch * kk * 8));
  double* rfac = (double*)((char*)tmp + up256((size_t)batch * d * k * 8));
  hipStream_t s = (hipStream_t)stream;
  e = lp::launch_cross_gram(batch, d, k, Y, dk, Y, dk, gram, s);
  if (e == hipSuccess) e = lp::cholqr2_passes(batch, d, k, Y, gram, gram2, tmp, rfac, Q, nullptr, 0, flags, s);
  if (e != hipSuccess) return lp::report(LP_EDEVICE, std::string("orth: ") + hipGetErrorString(e));
  return LP_OK;
}
