// Entry points that allocate no device memory, for callers that cannot allocate: code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation.  Their work memory is one
// fixed file-scope device array per GPU (`scratch`), resolved once per device to its address.
#include <mutex>

#include "device_common.h"
#include "internal.h"
#include "../../include/regmg.h"

namespace rmg {

// Size of the per-device work array (every GPU the library runs on holds it until the process
// ends): 32 MiB, the four work vectors of rmg_convergence_factor_noalloc for up to 1,048,576
// regional dofs.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, taken with that device current (each GPU holds its
// own copy of the array at its own address); the array's name is only a host-side stand-in.
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices] = {};

static void* device_scratch(int device) {
  RMG_REQUIRE(device >= 0 && device < kMaxDevices, RMG_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    RMG_HIP(hipGetDevice(&cur));
    RMG_REQUIRE(cur == device, RMG_ERR_DEVICE, "internal: scratch resolved with another device current");
    void* p = nullptr;
    RMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    RMG_REQUIRE(p != nullptr, RMG_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace rmg

using namespace rmg;

extern "C" {

rmg_status rmg_convergence_factor_noalloc(rmg_handle* h, int cycles, double* rho) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && rho != nullptr, RMG_ERR_ARG, "null handle or output");
  bind_handle(h);
  RMG_REQUIRE(h->have_hierarchy, RMG_ERR_NOT_SETUP, "hierarchy not set up");
  RMG_REQUIRE(cycles >= 1 && cycles <= 10000, RMG_ERR_ARG, "cycles must be in [1, 10000]");
  const int64_t n = h->levels[0]->ndofs();
  RMG_REQUIRE((size_t)n * 4 * sizeof(double) <= kScratchBytes, RMG_ERR_ARG,
              "rmg_convergence_factor_noalloc: " + std::to_string(n) + " regional dofs need " +
                  std::to_string((size_t)n * 4 * sizeof(double)) + " bytes of work memory, more than the " +
                  std::to_string(kScratchBytes) + "-byte scratch array (at most " +
                  std::to_string(kScratchBytes / (4 * sizeof(double))) + " dofs)");
  double* work = static_cast<double*>(device_scratch(h->device));
  *rho = convergence_factor(h, cycles, work);
  API_END
}

}  // extern "C"
