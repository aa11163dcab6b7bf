// Elementwise pass of the inpainting iteration (Algorithm 3, Section 5 image
// and video inpainting): the signal fed to the forward transform combines
// the known samples with the current estimate in the missing ones.
#include <hip/hip_runtime.h>

#include "inpaint.hpp"

namespace sl {

namespace {

constexpr int kMixThreads = 256;

template <bool FIRST>
__global__ __launch_bounds__(kMixThreads) void k_inpaint_mix(
    const float4 *__restrict__ fm, const uchar4 *__restrict__ mask, const float4 *f,
    float4 *__restrict__ g, size_t n4, const float *__restrict__ delta_init, float fac,
    float *__restrict__ sigma, int B) {
  if (blockIdx.x == 0)
    for (int b = threadIdx.x; b < B; b += kMixThreads) sigma[b] = delta_init[b] * fac;
  const size_t stride = (size_t)gridDim.x * kMixThreads;
  for (size_t i = (size_t)blockIdx.x * kMixThreads + threadIdx.x; i < n4; i += stride) {
    const float4 a = fm[i];
    const uchar4 m = mask[i];
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!FIRST) p = f[i];
    float4 r;
    r.x = m.x ? a.x : p.x;
    r.y = m.y ? a.y : p.y;
    r.z = m.z ? a.z : p.z;
    r.w = m.w ? a.w : p.w;
    g[i] = r;
  }
}

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

hipError_t launch_inpaint_mix(const float *fm, const uint8_t *mask, const float *f, float *g,
                              size_t n, bool first, const float *delta_init, float fac,
                              float *sigma, int B, hipStream_t st) {
  const size_t n4 = n / 4;
  const unsigned blocks = mix_blocks(n4);
  if (first)
    hipLaunchKernelGGL(k_inpaint_mix<true>, dim3(blocks), dim3(kMixThreads), 0, st,
                       (const float4 *)fm, (const uchar4 *)mask, (const float4 *)f, (float4 *)g,
                       n4, delta_init, fac, sigma, B);
  else
    hipLaunchKernelGGL(k_inpaint_mix<false>, dim3(blocks), dim3(kMixThreads), 0, st,
                       (const float4 *)fm, (const uchar4 *)mask, (const float4 *)f, (float4 *)g,
                       n4, delta_init, fac, sigma, B);
  return hipGetLastError();
}

}  // namespace sl
