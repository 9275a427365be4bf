// mgme_matrix_element_noalloc: the matrix-element call for callers that
// cannot allocate device memory.  Its staging buffers live in a fixed
// file-scope device array instead of the stream-ordered allocator; see
// include/mgme.h for the contract.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mgme.h"
#include "internal.h"

namespace {

// One copy per GPU, held by the process until it ends.  Host code must never
// pass this name to a kernel or a copy: it is a host-side stand-in.  Use the
// per-device address from scratch_on() instead.
static __device__ __align__(256) char scratch[MGME_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up
// once per device.
int scratch_on(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return mgme::set_error(MGME_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return mgme::set_error(MGME_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
    }
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return MGME_OK;
}

}  // namespace

extern "C" int mgme_matrix_element_noalloc(const mgme_process* proc, const double* d_mom, long long nevt,
                                           long long ld, int precision, double* d_me, void* hip_stream) {
  if (!proc) return mgme::set_error(MGME_EINVAL, "process is NULL");
  if (precision < MGME_FP64 || precision > MGME_FP64_FP32COLOUR)
    return mgme::set_error(MGME_EINVAL, "unknown precision");
  if (mgme::workspace_min_bytes(proc, precision) > (long long)MGME_NOALLOC_SCRATCH_BYTES)
    return mgme::set_error(MGME_EINVAL, "one 64-event sub-batch of this process and precision needs more than "
                                        "MGME_NOALLOC_SCRATCH_BYTES of staging");
  if (nevt <= 0) return mgme::matrix_element_ws(proc, d_mom, nevt, ld, precision, d_me, nullptr,
                                                (hipStream_t)hip_stream);
  const int device = mgme::process_device(proc);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return mgme::set_error(MGME_EDEVICE, "hipGetDevice");
  if (cur != device && hipSetDevice(device) != hipSuccess) return mgme::set_error(MGME_EDEVICE, "hipSetDevice");
  mgme::Workspace ws{nullptr, (long long)MGME_NOALLOC_SCRATCH_BYTES};
  const int rc = scratch_on(device, &ws.ptr);
  if (rc != MGME_OK) return rc;
  return mgme::matrix_element_ws(proc, d_mom, nevt, ld, precision, d_me, &ws, (hipStream_t)hip_stream);
}
