// Elementwise pass of the image-decomposition iteration (Algorithm 4,
// Section 5 image decomposition): the signals fed to the two forward
// transforms, each the image minus the other part's current estimate.  (The
// inpainting iteration forms its input inside the forward row pass.)
#include <hip/hip_runtime.h>

#include "inpaint.hpp"

namespace sl {

namespace {

constexpr int kMixThreads = 256;

template <bool FIRST>
__global__ __launch_bounds__(kMixThreads) void k_decompose_mix(
    const float4 *__restrict__ f, const float4 *f0, const float4 *f1, float4 *__restrict__ g0,
    float4 *__restrict__ g1, size_t n4, const float *__restrict__ delta_init, float fac,
    float *__restrict__ sigma, int B) {
  if (blockIdx.x == 0)
    for (int b = threadIdx.x; b < B; b += kMixThreads) sigma[b] = delta_init[b] * fac;
  const size_t stride = (size_t)gridDim.x * kMixThreads;
  for (size_t i = (size_t)blockIdx.x * kMixThreads + threadIdx.x; i < n4; i += stride) {
    const float4 a = f[i];
    if (FIRST) {
      g0[i] = a;
      g1[i] = a;
    } else {
      const float4 p = f0[i], q = f1[i];
      g0[i] = make_float4(a.x - q.x, a.y - q.y, a.z - q.z, a.w - q.w);
      g1[i] = make_float4(a.x - p.x, a.y - p.y, a.z - p.z, a.w - p.w);
    }
  }
}

unsigned mix_blocks(size_t n4) {
  // a few waves of blocks per CU; the grid-stride loop covers the rest
  const size_t want = (n4 + kMixThreads - 1) / kMixThreads;
  return (unsigned)(want < 8192 ? (want ? want : 1) : 8192);
}

}  // namespace

hipError_t launch_decompose_mix(const float *f, const float *f0, const float *f1, float *g0,
                                float *g1, size_t n, bool first, const float *delta_init,
                                float fac, float *sigma, int B, hipStream_t st) {
  const size_t n4 = n / 4;
  if (first)
    hipLaunchKernelGGL(k_decompose_mix<true>, dim3(mix_blocks(n4)), dim3(kMixThreads), 0, st,
                       (const float4 *)f, (const float4 *)f0, (const float4 *)f1, (float4 *)g0,
                       (float4 *)g1, n4, delta_init, fac, sigma, B);
  else
    hipLaunchKernelGGL(k_decompose_mix<false>, dim3(mix_blocks(n4)), dim3(kMixThreads), 0, st,
                       (const float4 *)f, (const float4 *)f0, (const float4 *)f1, (float4 *)g0,
                       (float4 *)g1, n4, delta_init, fac, sigma, B);
  return hipGetLastError();
}

}  // namespace sl
