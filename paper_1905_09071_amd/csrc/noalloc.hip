// agg_rhs_noalloc: the right-hand side of agg_rhs with its per-state workspace
// (forward spectra, combined spectrum, partial dot products, loss weights) taken
// from a fixed device array of this library instead of plan-owned buffers, for
// callers that cannot allocate device memory at call time.
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the variable's name to a kernel or a copy (on the host that name
// is only a stand-in): its device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "../../include/agg.h"
#include "internal.h"

namespace agg {

constexpr size_t kScratchBytes = size_t(64) << 20;   // AGG_NOALLOC_SCRATCH_BYTES

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on device `dev`, looked up once with that device
// current (the caller's current device is restored).
static agg_status scratch_address(int dev, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) {
    *out = it->second;
    return AGG_OK;
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  void* ptr = nullptr;
  e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!ptr) return set_error(AGG_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
  addr.emplace(dev, ptr);
  *out = ptr;
  return AGG_OK;
}

}  // namespace agg

using namespace agg;

extern "C" agg_status agg_rhs_noalloc(agg_plan* plan, const double* n, double* dndt, int32_t batch) {
  if (!plan || !n || !dndt) return set_error(AGG_EINVAL, "NULL argument");
  if (plan_is_plain(plan)) return set_error(AGG_EINVAL, "agg_rhs_noalloc takes shared-column plans only");
  if (batch < 1 || batch > plan_batch(plan))
    return set_error(AGG_EINVAL, "batch must be in [1, the plan's batch]");
  const size_t per = rhs_workspace_bytes(plan);
  if (per > kScratchBytes / (size_t)batch)
    return set_error(AGG_EUNSUPPORTED, "workspace of " + std::to_string(per) + " bytes per state x " +
                                           std::to_string(batch) + " states exceeds the " +
                                           std::to_string(kScratchBytes) + "-byte static scratch array");
  void* ws = nullptr;
  agg_status rc = scratch_address(plan_device(plan), &ws);
  if (rc != AGG_OK) return rc;
  return rhs_in_workspace(plan, n, dndt, (int)batch, ws);
}
