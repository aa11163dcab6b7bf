// Training-data synthesis on the GPU: piecewise-constant cartoon images
// (ellipses and polygons painted in order, membership at pixel centres) plus
// Gaussian noise from a counter-based generator.  Used by the learned
// shrinkage training loop; not part of the transform.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sl {

constexpr int kShapeRecord = 24;

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// standard normal from one 64-bit counter (Box-Muller on two 32-bit halves)
__device__ __forceinline__ float gauss(uint64_t key) {
  const uint64_t h = splitmix64(key);
  const float u1 = ((float)(uint32_t)(h >> 40) + 0.5f) * (1.0f / 16777216.0f);
  const float u2 = (float)(uint32_t)(h & 0xFFFFFFull) * (1.0f / 16777216.0f);
  return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

__global__ void k_render(const float *__restrict__ shapes, int H, int W, int max_shapes,
                         const float *__restrict__ sigma, uint64_t seed, float *__restrict__ clean,
                         float *__restrict__ noisy) {
  const int n = blockIdx.y;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= H * W) return;
  const float px = (float)(pix % W) + 0.5f, py = (float)(pix / W) + 0.5f;
  const float *rec0 = shapes + (size_t)n * (1 + max_shapes * kShapeRecord);
  float v = rec0[0];
  for (int k = 0; k < max_shapes; ++k) {
    const float *r = rec0 + 1 + k * kShapeRecord;
    const int type = (int)r[0];
    if (type == 1) {
      const float dx = px - r[2], dy = py - r[3];
      const float u = dx * r[6] + dy * r[7], w = -dx * r[7] + dy * r[6];
      const float qa = u / r[4], qb = w / r[5];
      if (qa * qa + qb * qb <= 1.0f) v = r[1];
    } else if (type == 2) {
      const int nv = (int)r[2];
      bool inside = false;
      for (int a = 0; a < nv; ++a) {
        const int b = (a + 1) % nv;
        const float x1 = r[3 + 2 * a], y1 = r[4 + 2 * a], x2 = r[3 + 2 * b], y2 = r[4 + 2 * b];
        if ((y1 > py) != (y2 > py)) {
          const float xi = x1 + (py - y1) * (x2 - x1) / (y2 - y1);
          if (px < xi) inside = !inside;
        }
      }
      if (inside) v = r[1];
    }
  }
  const size_t o = (size_t)n * H * W + pix;
  clean[o] = v;
  if (noisy) noisy[o] = v + sigma[n] * gauss(seed ^ ((uint64_t)n << 40) ^ (uint64_t)pix);
}

hipError_t render_cartoons(const float *shapes, int n, int H, int W, int max_shapes,
                           const float *sigma, uint64_t seed, float *clean, float *noisy,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_render, dim3((H * W + 255) / 256, n), dim3(256), 0, st, shapes, H, W,
                     max_shapes, sigma, seed, clean, noisy);
  return hipGetLastError();
}

}  // namespace sl
