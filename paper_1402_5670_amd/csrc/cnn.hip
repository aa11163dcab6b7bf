// Learned shrinkage network on gfx950 matrix cores (an extension beyond the
// paper: a per-scale CNN predicting a gain in [0, 1] for every detail
// coefficient; hard thresholding, Section 5.3, is its fallback).
//
//   x0 = (|c| / (sigma ||psi_i||_2), sigma * 255 / 50)        2 channels
//   h1 = relu(conv3x3(x0; W1) + b1)     h2 = relu(conv3x3(h1; W2) + b2)
//   g  = sigmoid(conv3x3(h2; W3) + b3)  shrunk coefficient g * c
//
// Activations are channel-last bfloat16 tensors [P][H][W][32] (P planes, 64 B
// per pixel, unused channels zero).  A 3x3 convolution is an implicit GEMM:
// for every tap, 16 output pixels x 16 output channels accumulate one
// v_mfma_f32_16x16x32_bf16 over the 32 input channels (FP32 accumulation).
// Operand layout of that instruction (64 lanes, l = lane):
//   A[m][k]: m = l % 16, k = 8 (l / 16) + j, j = 0..7  (8 bf16 per lane)
//   B[k][n]: n = l % 16, k = 8 (l / 16) + j
//   D[m][n]: n = l % 16, m = 4 (l / 16) + i, i = 0..3  (4 floats per lane)
// The backward data pass is the same convolution with flipped, transposed
// weights; weight gradients put pixels on the reduction axis.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cnn.hpp"

namespace sl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int TH = 8, TW = 32;                 // output tile
constexpr int HH = TH + 2, HW2 = TW + 2;       // input halo tile
constexpr int CH = 32;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);             // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// x0 planes from the coefficients
// ---------------------------------------------------------------------------
__global__ void k_cnn_x0(const float *__restrict__ coef, CnnPlanes pl, uint16_t *__restrict__ x0,
                         int HWn) {
  const int p = blockIdx.y;
  const int px = blockIdx.x * blockDim.x + threadIdx.x;
  if (px >= HWn) return;
  int b, i, j;
  plane_info(pl, p, b, i, j);
  const float sg = pl.sigma[b];
  const float c = coef[((size_t)b * pl.R + i) * HWn + px];
  const float v0 = fabsf(c) / (sg * pl.l2[i]);
  const float v1 = sg * (255.0f / 50.0f);
  uint4 *dst = (uint4 *)(x0 + ((size_t)p * HWn + px) * CH);
  dst[0] = make_uint4((uint32_t)f2bf(v0) | ((uint32_t)f2bf(v1) << 16), 0u, 0u, 0u);
  dst[1] = make_uint4(0u, 0u, 0u, 0u);
  dst[2] = make_uint4(0u, 0u, 0u, 0u);
  dst[3] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// 3x3 convolution, implicit GEMM on MFMA
// ---------------------------------------------------------------------------
// Wp: packed weight operands [J][9][NB][64 lanes][8] bf16; bias [J][..] float.
// The weights are the A operand and the activation tile the B operand, so a
// lane receives 4 consecutive output channels (16 nb + 4 (lane / 16) + i) of
// one pixel (lane % 16) and stores them with one 8-byte write.  The halo tile
// keeps pixels at a 40-channel stride (80 bytes) in LDS.
constexpr int kConvCP = 40;
template <int NB, int MODE>
__global__ void __launch_bounds__(256)
k_conv3x3(const uint16_t *__restrict__ in, const uint16_t *__restrict__ Wp,
          const float *__restrict__ bias, int bias_stride, CnnPlanes pl, int H, int W,
          uint16_t *__restrict__ out, const uint16_t *__restrict__ mask,
          const float *__restrict__ coef, float *__restrict__ coef_out, float *__restrict__ gain) {
  __shared__ __attribute__((aligned(16))) uint16_t tile[HH * HW2 * kConvCP];
  const int p = blockIdx.z;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const size_t HWn = (size_t)H * W;
  const uint16_t *src = in + (size_t)p * HWn * CH;
  int b, i, j;
  plane_info(pl, p, b, i, j);
  // halo tile: 16-byte chunks, zero outside the image
  for (int q = threadIdx.x; q < HH * HW2 * 4; q += 256) {
    const int pix = q >> 2, part = q & 3;
    const int yy = ty0 + pix / HW2 - 1, xx = tx0 + pix % HW2 - 1;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (yy >= 0 && yy < H && xx >= 0 && xx < W)
      v = ((const uint4 *)(src + ((size_t)yy * W + xx) * CH))[part];
    *(uint4 *)(tile + pix * kConvCP + 8 * part) = v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  bf16x8 wb[9][NB];
  const uint16_t *wj = Wp + (size_t)j * 9 * NB * 64 * 8;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      wb[t][nb] = *(const bf16x8 *)(wj + (((size_t)t * NB + nb) * 64 + lane) * 8);
  // accumulator initial values: the bias of each lane's 4 channels (layer 3
  // has one output channel, channel 0)
  f32x4 binit[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ch = 16 * nb + 4 * g + e;
      float v = 0.f;
      if constexpr (MODE == CONV_RELU) v = bias[(size_t)j * bias_stride + ch];
      if constexpr (MODE == CONV_GAIN) v = ch == 0 ? bias[(size_t)j * bias_stride] : 0.f;
      binit[nb][e] = v;
    }
  __syncthreads();
  // 16 pixel blocks (row r, half h) per tile; wave w takes blocks w, w+4, w+8, w+12
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int blk = wave + 4 * s;
    const int r = blk >> 1, c0 = (blk & 1) * 16;
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = binit[nb];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t % 3;
      const int pix = (r + dy) * HW2 + c0 + (lane & 15) + dx;
      const bf16x8 xb = *(const bf16x8 *)(tile + pix * kConvCP + 8 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[t][nb], xb, acc[nb], 0, 0, 0);
    }
    const int yy = ty0 + r, xx = tx0 + c0 + (lane & 15);
    if (yy >= H || xx >= W) continue;
    const size_t opix = (size_t)p * HWn + (size_t)yy * W + xx;
    if constexpr (MODE == CONV_RELU) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = (__bf16)fmaxf(acc[nb][e], 0.f);
        *(bf16x4 *)(out + opix * CH + 16 * nb + 4 * g) = o;
      }
    } else if constexpr (MODE == CONV_MASKED) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const uint2 mk = *(const uint2 *)(mask + opix * CH + 16 * nb + 4 * g);
        const uint16_t *mh = (const uint16_t *)&mk;
        bf16x4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = (__bf16)(mh[e] != 0 ? acc[nb][e] : 0.f);
        *(bf16x4 *)(out + opix * CH + 16 * nb + 4 * g) = o;
      }
    } else {   // CONV_GAIN: channel 0 sits in lane group 0, element 0
      if (g == 0) {
        const float gv = 1.0f / (1.0f + __expf(-acc[0][0]));
        const size_t co = ((size_t)b * pl.R + i) * HWn + (size_t)yy * W + xx;
        if (gain) gain[co] = gv;
        if (coef_out) coef_out[co] = gv * coef[co];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// fused inference: the three layers of 16 x 32 output tiles in LDS
// ---------------------------------------------------------------------------
// Regions (rows x cols): x0 22 x 38, h1 20 x 36, h2 18 x 34, output 16 x 32.
// Activations outside the image are zero (the "same" zero padding of every
// layer).  The weights are the A operand and the activations the B operand,
// so each lane receives 4 consecutive output channels of one pixel
// (D[m = channel][n = pixel]) and stores them with one 8-byte LDS write.
// Layer 1 packs its 9 taps x 2 input channels into one K = 32 operand
// (k = 2 t + c, k >= 18 zero); layer 2 is the per-tap implicit GEMM.  Layer 3
// has one output channel: an MFMA with the 9 taps on the M axis yields
// D[t][p] = sum_ci W3[ci][t] h2[p][ci] for every h2 pixel p, and the output is
// b3 + sum_t D[t][p + offset(t)].  D needs h2 at p only, so it is computed
// from the layer-2 accumulators in registers and h2 never reaches LDS.
// h1 pixels are padded to 48 channels (96 bytes, 16-byte aligned).  Measured
// per 32 images: 40 channels 17.7 ms, 48 channels 17.3 ms, 56 channels
// 17.9 ms, 64 channels (128-byte stride) 24.0 ms.
// Output tile FTH x 32 (SL_CNN_FTH = 16 or 8), one thread per output pixel;
// pixel stride of h1 SL_CNN_CHP bfloat16 values (>= 32, a multiple of 8).
#ifndef SL_CNN_FTH
#define SL_CNN_FTH 16
#endif
#ifndef SL_CNN_CHP
#define SL_CNN_CHP 48
#endif
constexpr int FTH = SL_CNN_FTH, FTW = 32;
constexpr int X0H = FTH + 6, X0W = FTW + 6;
constexpr int H1H = FTH + 4, H1W = FTW + 4;
constexpr int H2H = FTH + 2, H2W = FTW + 2;
constexpr int NX0 = X0H * X0W, NH1 = H1H * H1W, NH2 = H2H * H2W;
constexpr int CHP = SL_CNN_CHP;
constexpr int kFusedThreads = FTH * FTW;
static_assert(NH1 % 16 == 0 && CHP % 8 == 0 && CHP >= 32, "tile geometry");
constexpr int kX0PerThread = (NX0 + kFusedThreads - 1) / kFusedThreads;
// LDS (bytes): h1 | layer-3 partial sums D[16][NH2] | x0 | 2 x raw centre
// coefficients.  h2 never reaches LDS: layer 3 consumes it from the layer-2
// accumulators.
constexpr int kLdsH1 = NH1 * CHP * 2, kLdsD3 = 16 * NH2 * 4, kLdsX0 = ((NX0 * 4 + 15) / 16) * 16,
              kLdsC = FTH * FTW * 4;
constexpr int kLdsFused = kLdsH1 + kLdsD3 + kLdsX0 + 2 * kLdsC;
// blocks of the persistent grid per compute unit (160 KiB of LDS each)
constexpr int kFusedBlocksPerCU = (2 * kLdsFused <= 160 * 1024) ? 2 : 1;

// relu(d) on 4 channels (the bias is the accumulator's initial value), zero
// outside the image, rounded to bfloat16 (round to nearest even, as f2bf) by
// the native conversion
// (relu as a signed integer maximum of the float bits: negative floats have
// the sign bit set, so max(bits, 0) maps them to +0 and keeps the others)
template <bool INTERIOR>
__device__ __forceinline__ bf16x4 relu_bf16x4(f32x4 d, bool in) {
  bf16x4 o;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float v = __int_as_float(max(__float_as_int(d[e]), 0));
    o[e] = (__bf16)((INTERIOR || in) ? v : 0.f);
  }
  return o;
}

struct FusedTile {
  int p, ty0, tx0, b, i, j;
};

__device__ __forceinline__ FusedTile fused_tile(const CnnPlanes &pl, int tile, int tiles_x,
                                                int tiles_per_plane) {
  FusedTile f;
  f.p = tile / tiles_per_plane;
  const int r = tile % tiles_per_plane;
  f.ty0 = (r / tiles_x) * FTH;
  f.tx0 = (r % tiles_x) * FTW;
  plane_info(pl, f.p, f.b, f.i, f.j);
  return f;
}

template <int V>
struct IntC {
  static constexpr int value = V;
};

__global__ void __launch_bounds__(kFusedThreads)
k_cnn_fused(const float *__restrict__ coef, CnnPlanes pl, int H, int W, int ntiles,
            const uint16_t *__restrict__ W1k, const uint16_t *__restrict__ W2p,
            const uint16_t *__restrict__ W3m, const float *__restrict__ params,
            float *__restrict__ coef_out, float *__restrict__ gain) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kLdsFused];
  uint16_t *h1s = (uint16_t *)smem;
  float *d3 = (float *)(smem + kLdsH1);
  uint32_t *x0s = (uint32_t *)(smem + kLdsH1 + kLdsD3);
  float *cs = (float *)(smem + kLdsH1 + kLdsD3 + kLdsX0);   // [2][FTH * FTW]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  constexpr int NW = kFusedThreads / 64;
  const int tiles_x = (W + FTW - 1) / FTW;
  const int tiles_per_plane = tiles_x * ((H + FTH - 1) / FTH);
  const size_t HWn = (size_t)H * W;

  // x0 staging: thread positions in the x0 region do not depend on the tile
  int xq_r[kX0PerThread], xq_c[kX0PerThread], xq_cs[kX0PerThread];
#pragma unroll
  for (int u = 0; u < kX0PerThread; ++u) {
    const int q = threadIdx.x + u * kFusedThreads;
    xq_r[u] = q < NX0 ? q / X0W : -1000;
    xq_c[u] = q % X0W;
    const int r = xq_r[u], c = xq_c[u];
    xq_cs[u] = (r >= 3 && r < 3 + FTH && c >= 3 && c < 3 + FTW) ? (r - 3) * FTW + c - 3 : -1;
  }
  float xr[kX0PerThread];
  auto fetch = [&](const FusedTile &f) {
    const float *cpl = coef + ((size_t)f.b * pl.R + f.i) * HWn;
#pragma unroll
    for (int u = 0; u < kX0PerThread; ++u) {
      const int yy = f.ty0 - 3 + xq_r[u], xx = f.tx0 - 3 + xq_c[u];
      xr[u] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? cpl[(size_t)yy * W + xx] : 0.f;
    }
  };
  auto stage = [&](const FusedTile &f, int buf) {
    const float sg = pl.sigma[f.b];
    const float inv = 1.0f / (sg * pl.l2[f.i]);
    const uint32_t ch1 = (uint32_t)f2bf(sg * (255.0f / 50.0f)) << 16;
#pragma unroll
    for (int u = 0; u < kX0PerThread; ++u) {
      if (xq_r[u] < 0) continue;
      const int q = threadIdx.x + u * kFusedThreads;
      // out-of-image positions were fetched as 0; their x0 must be 0 in both channels
      const int yy = f.ty0 - 3 + xq_r[u], xx = f.tx0 - 3 + xq_c[u];
      const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
      x0s[q] = in ? ((uint32_t)f2bf(fabsf(xr[u]) * inv) | ch1) : 0u;
      if (xq_cs[u] >= 0) cs[buf * FTH * FTW + xq_cs[u]] = xr[u];
    }
  };

  // layer-1 operand: dword h of a lane's K slice is the (channel 0, channel 1)
  // pair of tap t = 4 g + h (k = 8 g + 2 h + channel).  Slots of taps >= 9
  // have zero weights; they read tap 0 (a staged, finite value) instead.
  int toff[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int t = 4 * g + h;
    toff[h] = t < 9 ? (t / 3) * X0W + t % 3 : 0;
  }

  // weights of the current scale (reloaded when the scale changes); the
  // biases become the accumulators' initial values
  bf16x8 w1[2], w2[9][2], w3;
  f32x4 bias1[2], bias2[2];
  float b3 = 0.f;
  int cur_j = -1;
  auto load_weights = [&](int j) {
    const float *P = params + (size_t)j * kCnnParams;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      w1[nb] = *(const bf16x8 *)(W1k + (((size_t)j * 2 + nb) * 64 + lane) * 8);
#pragma unroll
      for (int t = 0; t < 9; ++t)
        w2[t][nb] = *(const bf16x8 *)(W2p + ((((size_t)j * 9 + t) * 2 + nb) * 64 + lane) * 8);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ch = 16 * nb + 4 * g + q;
        bias1[nb][q] = P[kOffB1 + ch];
        bias2[nb][q] = P[kOffB2 + ch];
      }
    }
    w3 = *(const bf16x8 *)(W3m + ((size_t)j * 64 + lane) * 8);
    b3 = P[kOffB3];
  };

  // the three layers and the output of tile f; INTERIOR: the x0 region lies
  // inside the image, so no activation needs the zero padding mask
  auto layers = [&](const FusedTile &f, int buf, auto interior) {
    constexpr bool INTERIOR = decltype(interior)::value != 0;
    // ---- layer 1: NH1 pixels in blocks of 16; wave w takes blocks w, w + NW,
    // ..., three at a time (independent products and operand reads; 16.6 ->
    // 16.4 ms per 32 images against two at a time)
    auto l1 = [&](int bA, auto count) {
      constexpr int S = decltype(count)::value;
      bf16x8 xb[S];
      int qq[S];
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) {
        const int q = (bA + NW * s2) * 16 + (lane & 15);
        qq[s2] = q;
        const int base = (q / H1W) * X0W + q % H1W;
        uint32_t u[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) u[h] = x0s[base + toff[h]];
        xb[s2] = *(const bf16x8 *)u;
      }
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) {
        const int q = qq[s2];
        bool in = true;
        if constexpr (!INTERIOR) {
          const int r = q / H1W, c = q % H1W;
          const int yy = f.ty0 - 2 + r, xx = f.tx0 - 2 + c;
          in = yy >= 0 && yy < H && xx >= 0 && xx < W;
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[nb], xb[s2], bias1[nb], 0, 0, 0);
          *(bf16x4 *)(h1s + q * CHP + 16 * nb + 4 * g) = relu_bf16x4<INTERIOR>(d, in);
        }
      }
      __builtin_amdgcn_s_setprio(0);
    };
    constexpr int NB1 = NH1 / 16;
    for (int bA = wave; bA < NB1; bA += 3 * NW) {
      if (bA + 2 * NW < NB1) l1(bA, IntC<3>{});
      else if (bA + NW < NB1) l1(bA, IntC<2>{});
      else l1(bA, IntC<1>{});
    }
    __syncthreads();
    // ---- layer 2: NH2 pixels in NB2 blocks of 16 (the last may be partial).
    // Wave w of NW takes blocks w, w + NW, w + 2 NW, ..., three at a time (six
    // independent accumulators, the next tap's operands in flight; 240 VGPRs,
    // still two waves per SIMD; 16.7 -> 16.5 ms per 32 images against two at
    // a time)
    constexpr int NB2 = (NH2 + 15) / 16;
    auto l2 = [&](int bA, auto count) {
      constexpr int S = decltype(count)::value;
      int qq[S], base[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int q = (bA + NW * s) * 16 + (lane & 15);
        qq[s] = q;
        const int qc = q < NH2 ? q : NH2 - 1;   // duplicate a valid pixel; not stored
        base[s] = (qc / H2W) * H1W + qc % H2W;
      }
      f32x4 acc[S][2];
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[s][nb] = bias2[nb];
      const uint16_t *hp = h1s + 8 * g;
      bf16x8 xa[S];
#pragma unroll
      for (int s = 0; s < S; ++s) xa[s] = *(const bf16x8 *)(hp + base[s] * CHP);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        bf16x8 xn[S];
        if (t < 8) {
          const int off = ((t + 1) / 3) * H1W + (t + 1) % 3;
#pragma unroll
          for (int s = 0; s < S; ++s) xn[s] = *(const bf16x8 *)(hp + (base[s] + off) * CHP);
        }
        // a wave raises its issue priority while it issues its products, which
        // keeps the matrix pipe fed while the other wave of the SIMD issues its
        // LDS reads in the gaps (layers 1 and 2: 17.2 -> 16.8 ms per 32
        // images, bitwise-equal outputs)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[t][nb], xa[s], acc[s][nb], 0, 0, 0);
        __builtin_amdgcn_s_setprio(0);
        if (t < 8) {
#pragma unroll
          for (int s = 0; s < S; ++s) xa[s] = xn[s];
        }
      }
      // layer 3 on the h2 values of these pixels: lane group g holds channels
      // 4 g .. 4 g + 3 and 16 + 4 g .. 16 + 4 g + 3 of its pixel, the K order
      // of the packed layer-3 weights; D[t][q] for the 16 taps (9 used)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int q = qq[s];
        bool in = true;
        if constexpr (!INTERIOR) {
          const int qc = q < NH2 ? q : NH2 - 1;
          const int r = qc / H2W, c = qc % H2W;
          const int yy = f.ty0 - 1 + r, xx = f.tx0 - 1 + c;
          in = yy >= 0 && yy < H && xx >= 0 && xx < W;
        }
        const bf16x4 lo = relu_bf16x4<INTERIOR>(acc[s][0], in);
        const bf16x4 hi = relu_bf16x4<INTERIOR>(acc[s][1], in);
        const bf16x8 hb = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, hb, f32x4{0.f, 0.f, 0.f, 0.f},
                                                                0, 0, 0);
        if (q < NH2) {
#pragma unroll
          for (int e = 0; e < 4; ++e) d3[(4 * g + e) * NH2 + q] = d[e];
        }
      }
    };
    for (int bA = wave; bA < NB2; bA += 3 * NW) {
      if (bA + 2 * NW < NB2) l2(bA, IntC<3>{});
      else if (bA + NW < NB2) l2(bA, IntC<2>{});
      else l2(bA, IntC<1>{});
    }
    __syncthreads();
    // ---- output: one pixel per thread
    const int r = threadIdx.x / FTW, c = threadIdx.x % FTW;
    float z = b3;
#pragma unroll
    for (int t = 0; t < 9; ++t) z += d3[t * NH2 + (r + t / 3) * H2W + c + t % 3];
    const int yy = f.ty0 + r, xx = f.tx0 + c;
    if (INTERIOR || (yy < H && xx < W)) {
      const float gv = 1.0f / (1.0f + __expf(-z));
      const size_t co = ((size_t)f.b * pl.R + f.i) * HWn + (size_t)yy * W + xx;
      if (gain) gain[co] = gv;
      coef_out[co] = gv * cs[buf * FTH * FTW + threadIdx.x];
    }
  };

  int tile = blockIdx.x;
  if (tile >= ntiles) return;
  FusedTile f = fused_tile(pl, tile, tiles_x, tiles_per_plane);
  fetch(f);
  stage(f, 0);
  int buf = 0;
  __syncthreads();
  for (;;) {
    if (f.j != cur_j) {
      load_weights(f.j);
      cur_j = f.j;
    }
    // prefetch the next tile's coefficients; they land during the layers
    const int next = tile + gridDim.x;
    FusedTile fn = f;
    if (next < ntiles) {
      fn = fused_tile(pl, next, tiles_x, tiles_per_plane);
      fetch(fn);
    }
    const bool interior = f.ty0 >= 3 && f.ty0 + FTH + 3 <= H && f.tx0 >= 3 && f.tx0 + FTW + 3 <= W;
    if (interior) layers(f, buf, IntC<1>{});
    else layers(f, buf, IntC<0>{});
    if (next >= ntiles) break;
    // x0 was last read by layer 1 and the other centre buffer by the previous
    // tile's output: stage the next tile
    buf ^= 1;
    stage(fn, buf);
    tile = next;
    f = fn;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// backward helpers
// ---------------------------------------------------------------------------
// dz = dL/dc' * c * g (1 - g) on channel 0 of a zero-padded bf16 tensor;
// dbias3 partial sums are reduced later from dzf (float copy).
__global__ void k_cnn_dz(const float *__restrict__ dcoef, const float *__restrict__ coef,
                         const float *__restrict__ gain, CnnPlanes pl, int HWn,
                         uint16_t *__restrict__ dz, float *__restrict__ dzf) {
  const int p = blockIdx.y;
  const int px = blockIdx.x * blockDim.x + threadIdx.x;
  if (px >= HWn) return;
  int b, i, j;
  plane_info(pl, p, b, i, j);
  const size_t co = ((size_t)b * pl.R + i) * HWn + px;
  const size_t o = (size_t)p * HWn + px;
  const float g = gain[co];
  const float v = dcoef[co] * coef[co] * g * (1.f - g);
  if (dzf) dzf[o] = v;
  uint4 *dst = (uint4 *)(dz + o * CH);
  dst[0] = make_uint4((uint32_t)f2bf(v), 0u, 0u, 0u);
  dst[1] = make_uint4(0u, 0u, 0u, 0u);
  dst[2] = make_uint4(0u, 0u, 0u, 0u);
  dst[3] = make_uint4(0u, 0u, 0u, 0u);
}

// Weight gradients dW[t][ci][co] = sum_p x[p + t - 1][ci] dy[p][co] and
// db[co] = sum_p dy[p][co] over the tiles of planes of one scale.  Each block
// walks tiles with a grid stride and writes one partial [9*32*32 + 32].
// Pixels are the reduction axis: A[m = ci][k = pixel], B[k = pixel][n = co].
// Weight gradients of one layer over a range of planes: for every tap t,
// dW[t][ci][co] = sum_p x[p + offset(t)][ci] dy[p][co] (implicit GEMM with the
// pixels on the reduction axis; operands transposed to channel-major tiles in
// LDS) and dbias[co] = sum_p dy[p][co].  MB x NB selects the 16 x 16 blocks of
// (ci, co) that can be nonzero: layer 1 has 2 input channels (MB = 1), layer 3
// one output channel (NB = 1).  Only the channel quarters that those blocks
// read are loaded (XQ, DQ quarters of 8 channels).  A wave takes one tap row
// dy and one (mb, nb) block and computes its three taps dx = 0, 1, 2 together:
// the x rows are padded to 16-byte alignment, each lane reads 16 pixels with
// two aligned 16-byte loads and forms the three shifted operands in registers,
// and the dy operand is shared.  Each block writes its partial sums;
// k_reduce_partials adds them in a fixed order.
constexpr int kWgRow = 48;   // padded halo row (>= TW + 2 + 14, multiple of 8)
template <int MB, int NB>
__global__ void __launch_bounds__(256)
k_conv_wgrad(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dy, int H, int W,
             int plane0, int nplanes, float *__restrict__ partial) {
  constexpr int XQ = 2 * MB, DQ = 2 * NB;            // channel quarters of x and dy
  constexpr int NTRIP = 3 * MB * NB;                  // (tap row, mb, nb) units
  constexpr int TPW = (NTRIP + 3) / 4;                // per wave (4 waves)
  __shared__ __attribute__((aligned(16))) uint16_t xs[8 * XQ][HH * kWgRow];
  __shared__ __attribute__((aligned(16))) uint16_t ds[8 * DQ][TH * TW];
  __shared__ float bsum[256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  const size_t HWn = (size_t)H * W;
  f32x4 acc[TPW][3];
#pragma unroll
  for (int s = 0; s < TPW; ++s)
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[s][d] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbias = 0.f;     // channel threadIdx.x % 32, pixels threadIdx.x / 32 + 8 i
  const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
  const int ntiles = nplanes * tiles_x * tiles_y;
  for (int q = blockIdx.x; q < ntiles; q += gridDim.x) {
    const int p = plane0 + q / (tiles_x * tiles_y);
    const int rem = q % (tiles_x * tiles_y);
    const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
    __syncthreads();
    // halo tile of x and output tile of dy, 8 channels (16 bytes) per load,
    // transposed to [channel][pixel]
    for (int k = threadIdx.x; k < HH * HW2 * XQ; k += 256) {
      const int pix = k / XQ, qu = k % XQ;
      const int r = pix / HW2, c = pix % HW2;
      const int yy = ty0 + r - 1, xx = tx0 + c - 1;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = ((const uint4 *)(x + ((size_t)p * HWn + (size_t)yy * W + xx) * CH))[qu];
      const uint16_t *h = (const uint16_t *)&v;
#pragma unroll
      for (int e = 0; e < 8; ++e) xs[8 * qu + e][r * kWgRow + c] = h[e];
    }
    for (int k = threadIdx.x; k < TH * TW * DQ; k += 256) {
      const int pix = k / DQ, qu = k % DQ;
      const int yy = ty0 + pix / TW, xx = tx0 + pix % TW;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (yy < H && xx < W)
        v = ((const uint4 *)(dy + ((size_t)p * HWn + (size_t)yy * W + xx) * CH))[qu];
      const uint16_t *h = (const uint16_t *)&v;
#pragma unroll
      for (int e = 0; e < 8; ++e) ds[8 * qu + e][pix] = h[e];
    }
    __syncthreads();
    if ((threadIdx.x & 31) < 8 * DQ) {
      const int c = threadIdx.x & 31;
#pragma unroll
      for (int k = threadIdx.x >> 5; k < TH * TW; k += 8) dbias += bf2f(ds[c][k]);
    }
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      const int trip = wave + 4 * s;
      if (trip < NTRIP) {
        const int dyy = trip / (MB * NB), mb = (trip / NB) % MB, nb = trip % NB;
        const int ci = 16 * mb + (lane & 15), co = 16 * nb + (lane & 15);
        for (int r = 0; r < TH; ++r) {
          const uint4 u0 = *(const uint4 *)&xs[ci][(r + dyy) * kWgRow + 8 * g];
          const uint4 u1 = *(const uint4 *)&xs[ci][(r + dyy) * kWgRow + 8 * g + 8];
          const bf16x8 bb = *(const bf16x8 *)&ds[co][r * TW + 8 * g];
          // pixels 8 g + dx .. 8 g + dx + 7 of the halo row for dx = 0, 1, 2
          const uint4 a1 = make_uint4(__builtin_amdgcn_alignbit(u0.y, u0.x, 16),
                                      __builtin_amdgcn_alignbit(u0.z, u0.y, 16),
                                      __builtin_amdgcn_alignbit(u0.w, u0.z, 16),
                                      __builtin_amdgcn_alignbit(u1.x, u0.w, 16));
          const uint4 a2 = make_uint4(u0.y, u0.z, u0.w, u1.x);
          acc[s][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8 *)&u0, bb, acc[s][0], 0, 0, 0);
          acc[s][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8 *)&a1, bb, acc[s][1], 0, 0, 0);
          acc[s][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8 *)&a2, bb, acc[s][2], 0, 0, 0);
        }
      }
    }
  }
  // D[m = ci][n = co]: lane holds ci = 16 mb + 4 (lane / 16) + e, co = 16 nb + lane % 16;
  // blocks outside MB x NB are zero
  float *dst = partial + (size_t)blockIdx.x * (9 * CH * CH + CH);
  for (int k = threadIdx.x; k < 9 * CH * CH; k += 256) {
    const int ci = (k / CH) % CH, co = k % CH;
    if (ci >= 16 * MB || co >= 16 * NB) dst[k] = 0.f;
  }
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int trip = wave + 4 * s;
    if (trip < NTRIP) {
      const int dyy = trip / (MB * NB), mb = (trip / NB) % MB, nb = trip % NB;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int t = 3 * dyy + d;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ci = 16 * mb + 4 * g + e, co = 16 * nb + (lane & 15);
          dst[(t * CH + ci) * CH + co] = acc[s][d][e];
        }
      }
    }
  }
  bsum[threadIdx.x] = dbias;
  __syncthreads();
  if (threadIdx.x < CH) {
    float sum = 0.f;
#pragma unroll
    for (int g2 = 0; g2 < 8; ++g2) sum += bsum[g2 * 32 + threadIdx.x];
    dst[9 * CH * CH + threadIdx.x] = sum;
  }
}

// Sum block partials in a fixed order (deterministic).
__global__ void k_reduce_partials(const float *__restrict__ partial, int nparts, int len,
                                  float *__restrict__ outv) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  float s = 0.f;
  for (int q = 0; q < nparts; ++q) s += partial[(size_t)q * len + k];
  outv[k] = s;
}

// Pack the conv B operands of every scale from the FP32 parameter blobs,
// layout [J][taps][NB][64 lanes][8]:
// mode 0: forward layer (W[co][ci][t]); mode 1: transposed layer with flipped
// taps (W'[ci][co][8 - t]) for the backward data pass; mode 2: layer 1 with
// its 9 taps x 2 channels packed into one K = 32 operand (taps = 1).
__global__ void k_pack(const float *__restrict__ params, int J, int layer, int mode,
                       uint16_t *__restrict__ Wp, int NB) {
  const int taps = mode >= 2 ? 1 : 9;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // over J*taps*NB*64*8
  const int total = J * taps * NB * 64 * 8;
  if (idx >= total) return;
  const int jj = idx % 8, lane = (idx / 8) % 64, nb = (idx / 512) % NB;
  const int t = (idx / (512 * NB)) % taps;
  const int js = idx / (512 * NB * taps);
  const int n = 16 * nb + (lane & 15);          // output channel of this conv
  const int k = 8 * (lane >> 4) + jj;           // input channel of this conv
  const float *P = params + (size_t)js * kCnnParams;
  float v = 0.f;
  // forward weight of the requested layer: Wl[co][ci][t] with sizes (cout, cin)
  const int off[3] = {kOffW1, kOffW2, kOffW3};
  const int cin[3] = {2, 32, 32}, cout[3] = {32, 32, 1};
  const int l = layer - 1;
  if (mode == 2) {
    const int tt = k >> 1, cc = k & 1;
    if (n < 32 && tt < 9) v = P[off[0] + (n * 2 + cc) * 9 + tt];
  } else if (mode == 3) {
    // layer 3 with the taps as output rows: row n = tap.  Column k of lane
    // group kg = k / 8 is the channel that the layer-2 accumulators of that
    // group hold: 4 kg + k % 8 for k % 8 < 4, else 16 + 4 kg + k % 8 - 4.
    const int kg = k >> 3, kj = k & 7;
    const int ch = kj < 4 ? 4 * kg + kj : 16 + 4 * kg + (kj - 4);
    if (n < 9) v = P[off[2] + ch * 9 + n];
  } else if (mode == 0) {
    if (n < cout[l] && k < cin[l]) v = P[off[l] + (n * cin[l] + k) * 9 + t];
  } else {
    // transposed: this conv maps the layer's output channels (k) to its input channels (n)
    if (n < cin[l] && k < cout[l]) v = P[off[l] + (k * cin[l] + n) * 9 + (8 - t)];
  }
  Wp[idx] = f2bf(v);
}

// Adam (Kingma and Ba) on the FP32 master parameters.  The constants b1,
// 1 - b1, b2, 1 - b2 and the bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
// are formed in double on the host and rounded once (1 - 0.999f in float32
// would be 1.3e-5 off 0.001).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float omb1, float b2,
                       float omb2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gg = g[k];
  const float mm = b1 * m[k] + omb1 * gg;
  const float vv = b2 * v[k] + omb2 * gg * gg;
  m[k] = mm;
  v[k] = vv;
  p[k] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t cnn_x0(const float *coef, const CnnPlanes &pl, int P, int H, int W, uint16_t *x0,
                  hipStream_t st) {
  const int HWn = H * W;
  hipLaunchKernelGGL(k_cnn_x0, dim3((HWn + 255) / 256, P), dim3(256), 0, st, coef, pl, x0, HWn);
  return hipGetLastError();
}

hipError_t cnn_conv(const uint16_t *in, const uint16_t *Wp, int NB, const float *bias,
                    int bias_stride, const CnnPlanes &pl, int P, int H, int W, int mode,
                    uint16_t *out, const uint16_t *mask, const float *coef, float *coef_out,
                    float *gain, hipStream_t st) {
  dim3 grid((W + TW - 1) / TW, (H + TH - 1) / TH, P);
  if (mode == CONV_RELU && NB == 2)
    hipLaunchKernelGGL((k_conv3x3<2, CONV_RELU>), grid, dim3(256), 0, st, in, Wp, bias,
                       bias_stride, pl, H, W, out, mask, coef, coef_out, gain);
  else if (mode == CONV_MASKED && NB == 2)
    hipLaunchKernelGGL((k_conv3x3<2, CONV_MASKED>), grid, dim3(256), 0, st, in, Wp, bias,
                       bias_stride, pl, H, W, out, mask, coef, coef_out, gain);
  else if (mode == CONV_GAIN && NB == 1)
    hipLaunchKernelGGL((k_conv3x3<1, CONV_GAIN>), grid, dim3(256), 0, st, in, Wp, bias,
                       bias_stride, pl, H, W, out, mask, coef, coef_out, gain);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t cnn_fused(const float *coef, const CnnPlanes &pl, int P, int H, int W,
                     const uint16_t *W1k, const uint16_t *W2p, const uint16_t *W3m,
                     const float *params, float *coef_out, float *gain, int nblocks,
                     hipStream_t st) {
  const int ntiles = P * ((W + FTW - 1) / FTW) * ((H + FTH - 1) / FTH);
  nblocks *= kFusedBlocksPerCU;
  const int grid = nblocks < ntiles ? nblocks : ntiles;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(k_cnn_fused, dim3(grid), dim3(kFusedThreads), 0, st, coef, pl, H, W, ntiles,
                     W1k, W2p, W3m, params, coef_out, gain);
  return hipGetLastError();
}

hipError_t cnn_dz(const float *dcoef, const float *coef, const float *gain, const CnnPlanes &pl,
                  int P, int H, int W, uint16_t *dz, float *dzf, hipStream_t st) {
  const int HWn = H * W;
  hipLaunchKernelGGL(k_cnn_dz, dim3((HWn + 255) / 256, P), dim3(256), 0, st, dcoef, coef, gain,
                     pl, HWn, dz, dzf);
  return hipGetLastError();
}

hipError_t cnn_wgrad(const uint16_t *x, const uint16_t *dy, int H, int W, int plane0,
                     int nplanes, int nblocks, float *partial, float *outv, int in_blocks,
                     int out_blocks, hipStream_t st) {
  if (in_blocks == 2 && out_blocks == 2)
    hipLaunchKernelGGL((k_conv_wgrad<2, 2>), dim3(nblocks), dim3(256), 0, st, x, dy, H, W, plane0,
                       nplanes, partial);
  else if (in_blocks == 1 && out_blocks == 2)
    hipLaunchKernelGGL((k_conv_wgrad<1, 2>), dim3(nblocks), dim3(256), 0, st, x, dy, H, W, plane0,
                       nplanes, partial);
  else if (in_blocks == 2 && out_blocks == 1)
    hipLaunchKernelGGL((k_conv_wgrad<2, 1>), dim3(nblocks), dim3(256), 0, st, x, dy, H, W, plane0,
                       nplanes, partial);
  else
    return hipErrorInvalidValue;
  const int len = 9 * CH * CH + CH;
  hipLaunchKernelGGL(k_reduce_partials, dim3((len + 255) / 256), dim3(256), 0, st, partial,
                     nblocks, len, outv);
  return hipGetLastError();
}

__global__ void k_copy_lowpass(const float *__restrict__ coef, float *__restrict__ out, int R,
                               int HWn) {
  const int b = blockIdx.y;
  const int px = blockIdx.x * blockDim.x + threadIdx.x;
  if (px < HWn) out[(size_t)b * R * HWn + px] = coef[(size_t)b * R * HWn + px];
}

// out = scale (a - b); partial[block] = sum of (a - b)^2 over the block's stride
__global__ void k_sqerr(const float *__restrict__ a, const float *__restrict__ b, size_t n,
                        float scale, float *__restrict__ out, float *__restrict__ partial) {
  __shared__ float red[256];
  float s = 0.f;
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
    const float d = a[k] - b[k];
    out[k] = scale * d;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t sq_error_grad(const float *a, const float *b, size_t n, float scale, float *out,
                         float *partial, int nblocks, float *loss, hipStream_t st) {
  hipLaunchKernelGGL(k_sqerr, dim3(nblocks), dim3(256), 0, st, a, b, n, scale, out, partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, st, partial, nblocks, 1, loss);
  return hipGetLastError();
}

hipError_t cnn_copy_lowpass(const float *coef, float *coef_out, int B, int R, int HWn,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_copy_lowpass, dim3((HWn + 255) / 256, B), dim3(256), 0, st, coef, coef_out,
                     R, HWn);
  return hipGetLastError();
}

// Scatter the full [9][32][32] + [32] weight gradients of the three layers
// into the parameter-blob layout of scale j (grads [J][kCnnParams]).
// dW1 comes from x = x0 (ci < 2), dW3 from dy = dz (co = 0).
__global__ void k_grad_assemble(const float *__restrict__ g1, const float *__restrict__ g2,
                                const float *__restrict__ g3, int j, float *__restrict__ grads) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kCnnParams) return;
  constexpr int L = 9 * CH * CH;   // bias sums follow the weights
  float v;
  if (k < kOffB1) {            // W1[co][ci][t], ci < 2: full[t][ci][co] of layer 1
    const int co = k / 18, ci = (k / 9) % 2, t = k % 9;
    v = g1[(t * CH + ci) * CH + co];
  } else if (k < kOffW2) {
    v = g1[L + (k - kOffB1)];
  } else if (k < kOffB2) {
    const int q = k - kOffW2, co = q / 288, ci = (q / 9) % 32, t = q % 9;
    v = g2[(t * CH + ci) * CH + co];
  } else if (k < kOffW3) {
    v = g2[L + (k - kOffB2)];
  } else if (k < kOffB3) {     // W3[0][ci][t]
    const int q = k - kOffW3, ci = q / 9, t = q % 9;
    v = g3[(t * CH + ci) * CH + 0];
  } else {
    v = g3[L + 0];
  }
  grads[(size_t)j * kCnnParams + k] = v;
}

hipError_t cnn_grad_assemble(const float *dW1, const float *dW2, const float *dW3, int j,
                             float *grads, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_assemble, dim3((kCnnParams + 255) / 256), dim3(256), 0, st, dW1, dW2,
                     dW3, j, grads);
  return hipGetLastError();
}

hipError_t cnn_pack(const float *params, int J, int layer, int mode, uint16_t *Wp, int NB,
                    hipStream_t st) {
  // mode 2 (packed layer 1) has one operand per (scale, nb): index as taps = 1
  const int total = J * (mode == 2 ? 1 : 9) * NB * 64 * 8;
  hipLaunchKernelGGL(k_pack, dim3((total + 255) / 256), dim3(256), 0, st, params, J, layer, mode,
                     Wp, NB);
  return hipGetLastError();
}

hipError_t cnn_adam(float *p, const float *g, float *m, float *v, int n, float lr, double b1,
                    double b2, double eps, int t, hipStream_t st) {
  const float c1 = (float)(1.0 - std::pow(b1, (double)t));
  const float c2 = (float)(1.0 - std::pow(b2, (double)t));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, (float)b1,
                     (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, c1, c2);
  return hipGetLastError();
}

}  // namespace sl
