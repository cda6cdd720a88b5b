// lbs_matvec_noalloc: the operator application of lbs_matvec for callers
// that cannot allocate device memory (code under graph capture, tight
// serving loops).  Its scratch buffers (FMM strengths and expansions,
// partial sums, completion counters, reduction space) live in one static
// device array per GPU instead of the handle's workspace.
#include <mutex>

#include "lbs_internal.h"

namespace lbs {
constexpr size_t kScratchBytes = (size_t)128 << 20;  // 128 MiB per GPU
}  // namespace lbs

static __device__ __align__(256) unsigned char scratch[lbs::kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up once per device
// with the device current; the array's host-side name is not a device
// address).
lbs_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    lbs::set_last_error("no current HIP device");
    return LBS_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      lbs::set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return LBS_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return LBS_OK;
}
}  // namespace

extern "C" lbs_status lbs_matvec_noalloc(lbs_handle h, int32_t op, int32_t prec,
                                         int32_t nrhs, const double *x, double *y,
                                         void *stream) {
  void *base = nullptr;
  const lbs_status st = scratch_address(&base);
  if (st != LBS_OK) return st;
  return lbs::matvec_in_scratch(h, op, prec, nrhs, x, y, stream, (char *)base,
                                lbs::kScratchBytes);
}
