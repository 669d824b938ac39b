// The device scratch of the allocation-free entry point: a file-scope
// static array, one copy per GPU the library runs on, held until the
// process ends.  Host code never passes the array's name to a kernel (in
// host code the name is a host-side stand-in); it resolves each device's
// address once, with that device current, and uses that address.
#include <mutex>

#include "kernels.hpp"

static __device__ __align__(256) uint8_t scratch[ilp::kStaticScratchBytes];

namespace ilp {

namespace {
constexpr int kMaxDevices = 64;
uint8_t* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

hipError_t static_scratch(int ordinal, uint8_t** ptr) {
  if (ordinal < 0 || ordinal >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[ordinal]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != ordinal) return hipErrorInvalidDevice;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[ordinal] = static_cast<uint8_t*>(p);
  }
  *ptr = g_scratch[ordinal];
  return hipSuccess;
}

}  // namespace ilp
