// fit_energy_noalloc: fit_energy's five values with the partial sums in a
// fixed device array of the library instead of memory the handle allocates
// on demand.
#include <mutex>
#include <string>

#include "fit_host.hpp"

namespace fit {

// Partial rows of the fixed scratch (kPartTerms doubles each), then the 12
// doubles the combination reads: 8192 * 10 * 8 B + 128 B = 640 KiB per device.
constexpr int64_t kScratchRows = 8192;
constexpr int64_t kScratchWork = kScratchRows * kPartTerms;
constexpr size_t kScratchDoubles = (size_t)kScratchWork + 16;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on device dev, looked up once per device (each
// device holds its own copy of the array).  In host code the array's name is
// not a device address; only this pointer is passed to kernels.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static int scratch_of(int dev, double** p) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FIT_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* q = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !q) return hip_fail(e, "scratch symbol address");
    g_scratch_ptr[dev] = static_cast<double*>(q);
  }
  *p = g_scratch_ptr[dev];
  return FIT_OK;
}

}  // namespace fit

using namespace fit;

extern "C" {

int fit_energy_noalloc(fit_grid* g, double* out) {
  if (!g || !out) return fail(FIT_E_INVALID, "null argument");
  if (!g->e_alt || !g->h_alt)
    return fail(FIT_E_STATE, "the allocation-free energies need the second field buffer set "
                             "(bind it with fit_bind_fields, or run a step first)");
  const int64_t rows = energy_rows(g);
  if (rows > kScratchRows)
    return fail(FIT_E_INVALID, "the grid needs " + std::to_string(rows) +
                                   " partial-sum rows; the fixed scratch holds " +
                                   std::to_string(kScratchRows));
  double* p = nullptr;
  if (int rc = scratch_of(g->dev, &p)) return rc;
  return energy_enqueue(g, p, p + kScratchWork, out);
}

}  // extern "C"
