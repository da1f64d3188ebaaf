// filter2d_backward_noalloc: the backward with a library-owned workspace, for
// callers that may not allocate device memory.
//
// The workspace is a file-scope device array.  In host code its name is only
// a host-side stand-in for the symbol, so its device address is looked up once
// per device with hipGetSymbolAddress (with that device current) and only
// that address is handed to the kernels.  Each device holds its own copy of
// the array for the life of the process; calls on one device share it, so
// they must not overlap in time (they race otherwise).
#include <hip/hip_runtime.h>

#include <mutex>

#include "f2d_host.hpp"

namespace f2d {
namespace {

constexpr size_t kScratchBytes = F2D_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
f2d_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(F2D_EUNSUPPORTED, "noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return fail(F2D_EHIP, "noalloc: hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return F2D_OK;
}

}  // namespace

f2d_status run_backward_noalloc(const Problem& pr, const f2d_tensor* grad_outs, int32_t n_grad_outs,
                                const f2d_tensor* grad_input, float* grad_filter, hipStream_t s) {
  if (f2d_status e = check_backward(pr, grad_outs, n_grad_outs, grad_input)) return e;
  const size_t need = backward_workspace(pr);
  if (need > kScratchBytes)
    return fail(F2D_EWORKSPACE, "noalloc: these arguments need %zu bytes of scratch; the static scratch holds %zu",
                need, kScratchBytes);
  if (!grad_input && !grad_filter) return ok();
  void* ws = nullptr;
  if (f2d_status st = scratch_address(&ws)) return st;
  // every scratch value the kernels read is written earlier in the same call
  // (frame values by the adjoint, one partial set per work unit), so nothing
  // needs clearing between calls
  return run_backward(pr, grad_outs, n_grad_outs, grad_input, grad_filter, ws, kScratchBytes, s);
}

}  // namespace f2d
