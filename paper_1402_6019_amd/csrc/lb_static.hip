// Device scratch for the entry point that allocates nothing (lb_profile_noalloc): a
// file-scope array of fixed size in every device's code object, whose device address is
// looked up once per device when a context is created on it.  Host code never passes the
// array's name to a kernel or a copy (on the host it only names the symbol): it uses the
// address hipGetSymbolAddress returned for the current device.

#include <hip/hip_runtime.h>

#include <mutex>

#include "lb_internal.hpp"

namespace lb355 {

// 4 MiB of doubles per device: the profile pass's block sums and row sums,
// (64-column blocks per row + 1) * ly * PROF_N doubles.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_addr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  double *p = nullptr;
  e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_addr[device] = p;
  return hipSuccess;
}

double *static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_addr[device];
}

}  // namespace lb355
