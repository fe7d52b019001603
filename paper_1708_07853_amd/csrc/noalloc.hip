// dwt2_fwd_noalloc: the forward transform with a workspace the library holds
// in device memory it never allocates at run time -- a file-scope device
// array, one per GPU the library runs on, kept until the process ends -- for
// callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.h"

namespace dwt2 {
namespace {

// The largest workspace dwt2_fwd_noalloc serves: 96 MiB, enough for one
// 8192 x 8192 image at six levels (its LL_1 .. LL_5 buffers and sync words
// take about 86 MB).
constexpr size_t kScratchBytes = (size_t)96 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

// The array's device address on the current device.  In host code the
// array's name is only a stand-in, so every use below goes through this
// address, looked up once per device with that device current.
int scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(DWT2_ERR_HIP, "no current device (or device index above %d)", kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DWT2_ERR_HIP, "looking up the scratch array on device %d failed: %s", dev, hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return DWT2_OK;
}

}  // namespace
}  // namespace dwt2

using namespace dwt2;

extern "C" {

int dwt2_fwd_noalloc(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
                     int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels,
                     int32_t mode, int32_t boundary, void* stream) {
  clear_error();
  const size_t need = dwt2_workspace_size(width, height, batch, levels, mode);
  if (need > kScratchBytes)
    return fail(DWT2_ERR_WORKSPACE, "this call needs %zu bytes of workspace; the scratch array holds %zu", need,
                kScratchBytes);
  void* ws = nullptr;
  if (need > 0) {  // need == 0: invalid arguments, which the transform reports
    const int st = scratch_ptr(&ws);
    if (st) return st;
  }
  return fwd_levels_path(src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                         levels, mode, boundary, ws, need > 0 ? kScratchBytes : 0, stream);
}

}  // extern "C"
