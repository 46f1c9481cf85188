// Allocation-free prior step: glr_prior_step with a library-owned workspace.
//
// The workspace is a file-scope device array (one copy per GPU, resident from
// the code object's load until the process ends).  In host code the array's
// name is only a stand-in for the symbol, not a device address, so its
// address on the current device is looked up once per device with
// hipGetSymbolAddress and only that pointer is ever handed to kernels or
// copies.  The call itself then runs the same launch sequence as
// glr_prior_step on that pointer: no hipMalloc, hipFree or other allocating
// routine is reached (plans with per-stage timing, which create HIP events,
// are refused).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[GLR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
glr_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof buf, "glr_prior_step_static: hipGetDevice: %s", hipGetErrorString(e));
    return glr_set_error(GLR_ERR_HIP, buf);
  }
  if (dev < 0 || dev >= kMaxDevices)
    return glr_set_error(GLR_ERR_UNSUPPORTED, "glr_prior_step_static: device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char buf[256];
      snprintf(buf, sizeof buf, "glr_prior_step_static: hipGetSymbolAddress: %s",
               hipGetErrorString(e));
      return glr_set_error(GLR_ERR_HIP, buf);
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GLR_OK;
}

}  // namespace

extern "C" GLR_API glr_status glr_prior_step_static(glr_plan* pl, const void* x_in, float sigma,
                                                    void* x_out, void* stream) {
  if (!pl) return glr_set_error(GLR_ERR_INVALID_ARG, "glr_prior_step_static: plan is NULL");
  if (!x_in || !x_out)
    return glr_set_error(GLR_ERR_INVALID_ARG, "glr_prior_step_static: x_in or x_out is NULL");
  if (pl->timing)
    return glr_set_error(GLR_ERR_UNSUPPORTED,
                         "glr_prior_step_static: plans with per-stage timing create HIP events");
  if (pl->ws.total > (size_t)GLR_STATIC_SCRATCH_BYTES) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "glr_prior_step_static: the plan needs a %zu-byte workspace, above the %zu-byte "
             "static scratch",
             pl->ws.total, (size_t)GLR_STATIC_SCRATCH_BYTES);
    return glr_set_error(GLR_ERR_WORKSPACE_TOO_SMALL, buf);
  }
  void* ws = nullptr;
  glr_status e = scratch_on_current_device(&ws);
  if (e) return e;
  // every call on this GPU shares the array: the statistics region is
  // cleared by each call (the prior step's other buffers start from values
  // the call itself writes)
  pl->stats_ws = nullptr;
  return glr_prior_step(pl, x_in, sigma, x_out, ws, stream);
}
