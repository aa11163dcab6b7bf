// Learned-shrinkage network: shared definitions (internal to libshearlet).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dispatch.hpp"

namespace sl {

// Parameter blob of one scale (float32): W1[32][2][9] b1[32] W2[32][32][9]
// b2[32] W3[1][32][9] b3[1]; weights indexed [co][ci][t], t = 3 dy + dx.
constexpr int kOffW1 = 0, kOffB1 = 576, kOffW2 = 608, kOffB2 = 9824, kOffW3 = 9856,
              kOffB3 = 10144, kCnnParams = 10145;

enum { CONV_RELU = 0, CONV_MASKED = 1, CONV_GAIN = 2 };

// Detail planes processed by a launch, grouped by scale: global plane g of
// scale j (start[j] <= g < start[j+1]) is image (g - start[j]) / nsub[j] and
// subband first[j] + (g - start[j]) % nsub[j].  A launch covers planes
// p0 .. p0 + P - 1 (local index p = g - p0).
struct CnnPlanes {
  int R, J, B, p0;
  int start[kMaxScales + 1];
  int nsub[kMaxScales], first[kMaxScales];
  const float *sigma;   // [B]
  const float *l2;      // [R]
};

__device__ __forceinline__ void plane_info(const CnnPlanes &pl, int p, int &b, int &i, int &j) {
  const int g = p + pl.p0;
  j = 0;
  while (j + 1 < pl.J && g >= pl.start[j + 1]) ++j;
  const int q = g - pl.start[j];
  b = q / pl.nsub[j];
  i = pl.first[j] + q % pl.nsub[j];
}

hipError_t cnn_x0(const float *coef, const CnnPlanes &pl, int P, int H, int W, uint16_t *x0,
                  hipStream_t st);
hipError_t cnn_conv(const uint16_t *in, const uint16_t *Wp, int NB, const float *bias,
                    int bias_stride, const CnnPlanes &pl, int P, int H, int W, int mode,
                    uint16_t *out, const uint16_t *mask, const float *coef, float *coef_out,
                    float *gain, hipStream_t st);
// fused inference over P planes; a persistent grid (one or two blocks per
// compute unit, by LDS size; nblocks = compute units) walks the output tiles
hipError_t cnn_fused(const float *coef, const CnnPlanes &pl, int P, int H, int W,
                     const uint16_t *W1k, const uint16_t *W2p, const uint16_t *W3m,
                     const float *params, float *coef_out, float *gain, int nblocks,
                     hipStream_t st);
hipError_t cnn_dz(const float *dcoef, const float *coef, const float *gain, const CnnPlanes &pl,
                  int P, int H, int W, uint16_t *dz, float *dzf, hipStream_t st);
// weight gradient over planes [plane0, plane0 + nplanes) (local indices)
// in_blocks / out_blocks: 16-channel blocks of x / dy that can be nonzero (1 or 2)
hipError_t cnn_wgrad(const uint16_t *x, const uint16_t *dy, int H, int W, int plane0,
                     int nplanes, int nblocks, float *partial, float *outv, int in_blocks,
                     int out_blocks, hipStream_t st);
hipError_t cnn_pack(const float *params, int J, int layer, int mode, uint16_t *Wp, int NB,
                    hipStream_t st);
hipError_t cnn_adam(float *p, const float *g, float *m, float *v, int n, float lr, double b1,
                    double b2, double eps, int t, hipStream_t st);
hipError_t cnn_copy_lowpass(const float *coef, float *coef_out, int B, int R, int HWn,
                            hipStream_t st);
hipError_t sq_error_grad(const float *a, const float *b, size_t n, float scale, float *out,
                         float *partial, int nblocks, float *loss, hipStream_t st);
hipError_t cnn_grad_assemble(const float *dW1, const float *dW2, const float *dW3, int j,
                             float *grads, hipStream_t st);

}  // namespace sl
