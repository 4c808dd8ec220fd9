// polydet_solve_noalloc: polydet_solve with the workspace taken from a file-scope device
// array instead of a caller's buffer, for callers that cannot allocate device memory.
//
// Each device the library runs on holds its own copy of `scratch` (it is allocated when the
// code object is loaded there and held until the process ends). In host code the array's
// name is only a stand-in for the symbol: its device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and only that address is ever passed
// to kernels. Every call on one device shares the array; calls that overlap on one device
// (other streams, other threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "abi_internal.h"
#include "polydet.h"

static __device__ __align__(256) uint8_t scratch[POLYDET_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// The device address of `scratch` on the current device (looked up on first use).
polydet_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return pd::abi_fail(POLYDET_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return pd::abi_fail(POLYDET_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return pd::abi_fail(POLYDET_EDEVICE,
                          std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return POLYDET_OK;
}

}  // namespace

extern "C" polydet_status polydet_solve_noalloc(polydet_plan_t plan, const int64_t* d_coeffs,
                                                uint32_t* d_out, void* stream) {
  if (!plan) return pd::abi_fail(POLYDET_EINVAL, "NULL plan");
  polydet_plan_info info;
  polydet_status st = polydet_plan_query(plan, 0, &info);
  if (st != POLYDET_OK) return st;
  if (info.workspace_bytes > (size_t)POLYDET_NOALLOC_SCRATCH_BYTES)
    return pd::abi_fail(POLYDET_EINVAL,
                        "the plan's workspace (" + std::to_string(info.workspace_bytes) +
                            " bytes) exceeds the no-allocation scratch (" +
                            std::to_string((size_t)POLYDET_NOALLOC_SCRATCH_BYTES) + " bytes)");
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != POLYDET_OK) return st;
  // polydet_solve checks the rest (batch plans, NULL buffers, the plan's device) and only
  // enqueues kernels: it allocates nothing and clears nothing that a later stage reads
  // before writing it
  return polydet_solve(plan, d_coeffs, d_out, ws, (size_t)POLYDET_NOALLOC_SCRATCH_BYTES, stream);
}
