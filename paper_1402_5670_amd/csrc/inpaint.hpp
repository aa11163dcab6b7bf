// Device pass of the inpainting iteration (internal to libshearlet).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sl {

// Input of one inpainting iteration (Algorithm 3): with a binary mask M,
//   g = M .* (f_masked - f) + f  =  f_masked where M = 1, f where M = 0,
// written as the selection; first = true treats f as zero (the iteration
// starts from f_inpainted = 0 and f is not read).  Also writes the threshold
// scale of the iteration, sigma[b] = delta_init[b] * fac, for the fused
// denoise pass.  n = B * npix, a multiple of 4; fm, f, g 16-byte aligned,
// mask 4-byte aligned.
hipError_t launch_inpaint_mix(const float *fm, const uint8_t *mask, const float *f, float *g,
                              size_t n, bool first, const float *delta_init, float fac,
                              float *sigma, int B, hipStream_t st);

// Inputs of one image-decomposition iteration (Algorithm 4): with
// f_res = f - (f0 + f1),  g0 = f_res + f0 = f - f1  and  g1 = f_res + f1 =
// f - f0, both from the estimates of the iteration's start; first = true
// treats f0 and f1 as zero (not read).  sigma[b] = delta_init[b] * fac.
// Same size and alignment rules as launch_inpaint_mix.
hipError_t launch_decompose_mix(const float *f, const float *f0, const float *f1, float *g0,
                                float *g1, size_t n, bool first, const float *delta_init,
                                float fac, float *sigma, int B, hipStream_t st);

}  // namespace sl
