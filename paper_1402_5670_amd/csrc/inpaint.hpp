// Device pass of the image-decomposition iteration (internal to libshearlet).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sl {

// Inputs of one image-decomposition iteration (Algorithm 4): with
// f_res = f - (f0 + f1),  g0 = f_res + f0 = f - f1  and  g1 = f_res + f1 =
// f - f0, both from the estimates of the iteration's start; first = true
// treats f0 and f1 as zero (not read).  Also writes the threshold scale of
// the iteration, sigma[b] = delta_init[b] * fac, for the fused denoise
// passes.  n = B * npix, a multiple of 4; all arrays 16-byte aligned.
hipError_t launch_decompose_mix(const float *f, const float *f0, const float *f1, float *g0,
                                float *g1, size_t n, bool first, const float *delta_init,
                                float fac, float *sigma, int B, hipStream_t st);

}  // namespace sl
