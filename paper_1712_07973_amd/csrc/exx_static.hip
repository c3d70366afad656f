// exx_static.hip -- exx_compute without any allocation: the workspace is a
// fixed-size array in device memory that the library owns (one per GPU, held
// until the process ends), for callers that cannot allocate (code under HIP
// graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "exx_internal.hpp"

namespace {

// The workspace of every exx_compute_noalloc call on a device.  In host code
// `scratch` only names the symbol: its device address is taken once per device
// with hipGetSymbolAddress and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[EXX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the device's
// first call, with that device current).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return exx::record_error(EXX_ERR_INVALID_ARG, "device index out of range for the static workspace");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return exx::record_hip_error(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return EXX_OK;
}

}  // namespace

extern "C" int exx_compute_noalloc(exx_plan* plan, const double* psi, const double* occ,
                                   int n_orb, int mode, unsigned flags, double* ex_out,
                                   double* kpsi, double* pair_e, void* stream) {
  if (!plan) return exx::record_error(EXX_ERR_INVALID_ARG, "plan is NULL");
  if (n_orb <= 0) return exx::record_error(EXX_ERR_INVALID_ARG, "n_orb must be positive");
  size_t need = 0;
  if (int rc = exx_workspace_bytes(plan, n_orb, &need)) return rc;
  if (need > (size_t)EXX_NOALLOC_SCRATCH_BYTES)
    return exx::record_error(EXX_ERR_WORKSPACE,
                             "exx_compute_noalloc needs " + std::to_string(need) +
                                 " bytes of workspace, above its static maximum of " +
                                 std::to_string((size_t)EXX_NOALLOC_SCRATCH_BYTES) +
                                 " (lower the plan's batch_slots or the orbital count)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return exx::record_hip_error(e, "hipGetDevice");
  if (dev != plan->device)
    return exx::record_error(EXX_ERR_INVALID_ARG,
                             "exx_compute_noalloc: the current device is not the plan's device");
  void* ws = nullptr;
  if (int rc = scratch_address(dev, &ws)) return rc;
  return exx::compute_impl(plan, psi, occ, n_orb, mode, flags, ex_out, kpsi, pair_e, ws,
                           (size_t)EXX_NOALLOC_SCRATCH_BYTES, stream, false);
}
