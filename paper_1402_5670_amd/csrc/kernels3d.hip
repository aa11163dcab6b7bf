// 3D transform passes on gfx950 (Section 3.3 filters, Algorithms 1 and 2).
//
// A volume [D][H][W] is transformed axis by axis with the line kernels of the
// 2D path applied to reshaped views: x lines are rows of a (D*H) x W image,
// y lines are columns of D images of H x W, z lines are columns of one
// D x (H*W) image.  Only the z pass is specific to 3D: it generates the
// filters on the fly from their factors
//     psi_hat(xi) = g_hat_{J-j}(xi_a) Phi_hat_{j,k1}(xi_a, xi_s1) Phi_hat_{j,k2}(xi_a, xi_s2)
// (main axis a and secondary axes s1, s2 of the pyramid), so the R full
// filter volumes never exist in memory.
#include <hip/hip_runtime.h>

#include "dispatch.hpp"
#include "fft_core.hpp"

namespace sl {

template <int N>
struct Tile3 {
  static constexpr int NT = Plan<N>::NT;
  static constexpr int E = Plan<N>::E;
  static constexpr int M = NT >= 128 ? 8 : 16;
  static constexpr int THREADS = M * NT;
};

// psi_hat_i along the z line of voxel column (y, x).  Unless z is the
// pyramid's main axis, only one factor varies along the line:
//   psi_hat(z) = c * tab[base + z * stride],
// with c the product of the two factors that are constant on the line (the
// lowpass: g_hat(x) h_hat(y) times h_hat(z)).  With z as the main axis all
// three factors vary: psi_hat(z) = tab[g + z] * tab[p1 + z] * tab[p2 + z].
struct ZLine {
  float c;
  int base, stride;   // one varying factor (main axis x or y, or lowpass)
  int g, p1, p2;      // main axis z (stride < 0 marks this case)
};

__device__ __forceinline__ ZLine zline(const Sub3D &d, const float *__restrict__ tab, int y,
                                       int x) {
  ZLine L;
  L.g = L.p1 = L.p2 = 0;
  if (d.cone == 0) {
    L.c = tab[d.g_off + x] * tab[d.p1_off + y];
    L.base = d.p2_off;
    L.stride = 1;
    return L;
  }
  const int idx[4] = {0, x, y, 0};
  if (d.am == 3) {
    L.c = 1.f;
    L.base = 0;
    L.stride = -1;
    L.g = d.g_off;
    L.p1 = d.p1_off + idx[d.s1] * d.n_main;
    L.p2 = d.p2_off + idx[d.s2] * d.n_main;
    return L;
  }
  const int im = idx[d.am];
  if (d.s1 == 3) {
    L.c = tab[d.g_off + im] * tab[d.p2_off + idx[d.s2] * d.n_main + im];
    L.base = d.p1_off + im;
  } else {
    L.c = tab[d.g_off + im] * tab[d.p1_off + idx[d.s1] * d.n_main + im];
    L.base = d.p2_off + im;
  }
  L.stride = d.n_main;
  return L;
}

__device__ __forceinline__ float zline_at(const ZLine &L, const float *__restrict__ tab, int z) {
  if (L.stride >= 0) return L.c * tab[L.base + z * L.stride];
  return tab[L.g + z] * tab[L.p1 + z] * tab[L.p2 + z];
}

// z pass of the forward transform: F * (psi_a + i psi_b), inverse DFT along z.
// Columns are the H*W voxels of a z-slice; grid (ceil(HW/M), nb).
template <int N>
__global__ void __launch_bounds__(Tile3<N>::THREADS)
k_z_filter_ifft(const float2 *__restrict__ F, const Sub3D *__restrict__ subs,
                const float *__restrict__ tab, float2 *__restrict__ T, int H, int W, int R,
                int b0, int p0, int np, const float2 *__restrict__ tw) {
  constexpr int NT = Tile3<N>::NT, M = Tile3<N>::M, E = Tile3<N>::E;
  __shared__ float2 lds[M * N];
  __shared__ float2 twl[N];   // twiddles staged once (ordered by the FFT's leading barrier)
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = tw[i];
  const int HW = H * W;
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < HW;
  const int cc = ok ? col : 0;
  const int y = cc / W, x = cc % W;
  const int b = b0 + blockIdx.y;
  const size_t vol = (size_t)N * HW;
  float2 f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) f[e] = F[(size_t)b * vol + (size_t)(t + e * NT) * HW + cc];
  for (int pp = 0; pp < np; ++pp) {
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const ZLine la = zline(subs[ia], tab, y, x);
    const ZLine lb = zline(subs[ib < R ? ib : ia], tab, y, x);
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int z = t + e * NT;
      const float a = zline_at(la, tab, z);
      const float bb = ib < R ? zline_at(lb, tab, z) : 0.f;
      v[e] = make_float2(f[e].x * a - f[e].y * bb, f[e].y * a + f[e].x * bb);
    }
    fft_line_p<Plan<N>, true>(v, t, LdsLine{lds + m, M}, TwLds{twl});
    if (ok) {
      float2 *To = T + ((size_t)blockIdx.y * np + pp) * vol + col;
#pragma unroll
      for (int e = 0; e < E; ++e) stream_store(&To[(size_t)(t + e * NT) * HW], v[e]);
    }
  }
}

// z pass of the inverse transform: DFT along z of each pair's U, multiply by
// (psi_a - i psi_b), sum over the pairs of the chunk; the last chunk divides
// by Psi_hat and applies the inverse DFT along z.
template <int N>
__global__ void __launch_bounds__(Tile3<N>::THREADS)
k_z_fft_acc(const float2 *__restrict__ U, const Sub3D *__restrict__ subs,
            const float *__restrict__ tab, const float *__restrict__ psi, float2 *__restrict__ ACC,
            int H, int W, int R, int b0, int p0, int np, int first, int last,
            const float2 *__restrict__ tw) {
  constexpr int NT = Tile3<N>::NT, M = Tile3<N>::M, E = Tile3<N>::E;
  __shared__ float2 lds[M * N];
  __shared__ float2 twl[N];   // twiddles staged once (ordered by the FFT's leading barrier)
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = tw[i];
  const int HW = H * W;
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < HW;
  const int cc = ok ? col : 0;
  const int y = cc / W, x = cc % W;
  const int b = b0 + blockIdx.y;
  const size_t vol = (size_t)N * HW;
  float2 *accp = ACC + (size_t)b * vol + cc;
  float2 acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e)
    acc[e] = first ? make_float2(0.f, 0.f) : accp[(size_t)(t + e * NT) * HW];
  for (int pp = 0; pp < np; ++pp) {
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const float2 *Ui = U + ((size_t)blockIdx.y * np + pp) * vol + cc;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = stream_load(&Ui[(size_t)(t + e * NT) * HW]);
    fft_line_p<Plan<N>, false>(v, t, LdsLine{lds + m, M}, TwLds{twl});
    const ZLine la = zline(subs[ia], tab, y, x);
    const ZLine lb = zline(subs[ib < R ? ib : ia], tab, y, x);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int z = t + e * NT;
      const float a = zline_at(la, tab, z);
      const float bb = ib < R ? zline_at(lb, tab, z) : 0.f;
      acc[e].x += a * v[e].x + bb * v[e].y;
      acc[e].y += a * v[e].y - bb * v[e].x;
    }
  }
  if (last) {
    const float *ps = psi + cc;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float d = ps[(size_t)(t + e * NT) * HW];
      acc[e] = make_float2(acc[e].x / d, acc[e].y / d);
    }
    fft_line_p<Plan<N>, true>(acc, t, LdsLine{lds + m, M}, TwLds{twl});
  }
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) accp[(size_t)(t + e * NT) * HW] = acc[e];
  }
}

#define SL_FOR_EACH_N(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

hipError_t launch_z_filter_ifft(const Sys3D &s, const float2 *F, float2 *T, Chunk c,
                                hipStream_t st) {
  const int HW = s.H * s.W;
  switch (s.D) {
#define X(N)                                                                                  \
  case N:                                                                                     \
    hipLaunchKernelGGL(k_z_filter_ifft<N>, dim3((HW + Tile3<N>::M - 1) / Tile3<N>::M, c.nb),   \
                       dim3(Tile3<N>::THREADS), 0, st, F, s.subs, s.tab, T, s.H, s.W, s.R, c.b0, \
                       c.p0, c.np, s.twD);                                                    \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_z_fft_acc(const Sys3D &s, const float2 *U, float2 *ACC, Chunk c, bool first,
                            bool last, hipStream_t st) {
  const int HW = s.H * s.W;
  switch (s.D) {
#define X(N)                                                                                  \
  case N:                                                                                     \
    hipLaunchKernelGGL(k_z_fft_acc<N>, dim3((HW + Tile3<N>::M - 1) / Tile3<N>::M, c.nb),       \
                       dim3(Tile3<N>::THREADS), 0, st, U, s.subs, s.tab, s.psi, ACC, s.H, s.W, \
                       s.R, c.b0, c.p0, c.np, (int)first, (int)last, s.twD);                  \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sl
