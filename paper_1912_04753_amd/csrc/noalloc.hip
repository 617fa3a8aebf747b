// The allocation-free entry point: ripk_compute_K for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops),
// with every workspace buffer cut from one file-scope device array.
//
// Each device the library runs on holds its own copy of `scratch` from the
// time the code object is loaded until the process ends.  Host code never
// passes the array's name to a kernel or a copy: it takes the device address
// once per device with hipGetSymbolAddress (with that device current) and
// uses that address from then on.
#include <mutex>

#include "ripk_internal.h"

namespace {

constexpr size_t kScratchBytes = RIPK_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch`, per device

// The scratch address on `device` (current); looked up on the first call.
hipError_t scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = ptr;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" ripk_status ripk_compute_K_noalloc(const ripk_plan_desc *desc, const ripk_points *pts,
                                              void *stream, ripk_K_out *out) {
  if (!desc) return ripk::set_error(RIPK_EINVAL, "null descriptor");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device < 0 || desc->device >= ndev ||
      desc->device >= kMaxDevices)
    return ripk::set_error(RIPK_EINVAL, "device out of range");
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(desc->device) != hipSuccess)
    return ripk::set_error(RIPK_EDEVICE, "cannot select the descriptor's device");
  void *ptr = nullptr;
  const hipError_t e = scratch_address(desc->device, &ptr);
  ripk_status s;
  if (e != hipSuccess || !ptr)
    s = ripk::set_error(RIPK_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
  else
    s = ripk::compute_K_in_scratch(desc, pts, (hipStream_t)stream, (unsigned char *)ptr,
                                   kScratchBytes, out);
  (void)hipSetDevice(prev);
  return s;
}
