// sos_filt_static: sos_filt for callers that cannot allocate device memory.
//
// sos_filt needs a caller workspace for its exact inter-tile carry (the
// tiles' end states, the scan's second buffer and the powers of the
// transition) and for the lane runs of wide groups.  This entry point takes
// that workspace from a fixed buffer in the library's own device image
// instead, so the caller passes only x and y.  Everything else (argument
// checks, the choice between run-in and scan, the kernels) is sos_filt's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.hpp"

namespace {

constexpr int kMaxDevices = 64;

// The workspace of sos_filt_static, one copy per device (it lives in the
// code object's data, so each GPU that loads the library holds its own
// until the process ends).  On the host this name is only a stand-in for
// the device symbol: host code uses the address that hipGetSymbolAddress
// returns for the current device, never the name itself.
static __device__ __align__(256) unsigned char scratch[SOS_STATIC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once
// per device with that device current; nullptr on failure.
void *scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_ptr[dev] = ptr;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" sos_status sos_filt_static(sos_plan_t p, const void *x, void *y, int64_t n,
                                      sos_stream_t stream) {
  if (!p || n < 0) return SOS_E_ARG;
  if (n == 0) return SOS_OK;
  const sos_status chk = sosf::check_filt_args(*p, x, y, n);
  if (chk != SOS_OK) return chk;
  const size_t need = sos_workspace_size(p, n);
  if (need > (size_t)SOS_STATIC_SCRATCH_BYTES) return SOS_E_SCRATCH;
  void *ws = nullptr;
  if (need > 0) {
    ws = scratch_on_current_device();
    if (!ws) return SOS_E_DEVICE;
  }
  return sos_filt(p, x, y, n, ws, stream);
}
