// Fused hard-threshold denoising for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid
// hipMalloc): the workspace of sl_denoise_fused is a file-scope device array
// instead of a caller buffer.  The kernels are those of sl_denoise_fused.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/shearlet.h"
#include "system.hpp"

namespace {

constexpr size_t kScratchBytes = SL_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code this name is
// only a handle for hipGetSymbolAddress; kernels get the device address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of this device's copy of the array, looked up once per
// device with that device current.
int scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return sl::hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return sl::set_error(SL_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return SL_OK;
}

}  // namespace

extern "C" int sl_denoise_fused_noalloc(const sl_system *s, const float *x_dev, int batch,
                                        const float *sigma_dev, const float *K_host,
                                        float *out_dev, void *stream) {
  if (!s) return sl::set_error(SL_EINVAL, "system is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->device)
    return sl::set_error(SL_EINVAL, "the current HIP device is not the system's device");
  if (dev < 0 || dev >= kMaxDevices) return sl::set_error(SL_EUNSUPPORTED, "device index too large");
  size_t need = 0;
  int rc = sl_workspace_size(s, batch, &need);
  if (rc) return rc;
  if (need > kScratchBytes)
    return sl::set_error(SL_ENOMEM,
                         "sl_denoise_fused_noalloc needs " + std::to_string(need) +
                             " bytes of scratch but its static array holds " +
                             std::to_string(kScratchBytes) +
                             ": use a smaller batch or chunk (sl_system_set_chunk_bytes)");
  void *ws = nullptr;
  rc = scratch_address(dev, &ws);
  if (rc) return rc;
  return sl_denoise_fused(s, x_dev, batch, sigma_dev, K_host, out_dev, ws, kScratchBytes, stream);
}
