// 3D transform passes on gfx950 (Section 3.3 filters, Algorithms 1 and 2).
//
// A volume [D][H][W] is transformed axis by axis with the line kernels of the
// 2D path applied to reshaped views: x lines are rows of a (D*H) x W image,
// y lines are columns of D images of H x W, z lines are columns of one
// D x (H*W) image.  Only the z pass is specific to 3D: it forms the filters
// on the fly from their factors
//     psi_hat(xi) = g_hat_{J-j}(xi_a) Phi_hat_{j,k1}(xi_a, xi_s1) Phi_hat_{j,k2}(xi_a, xi_s2)
// (main axis a and secondary axes s1, s2 of the pyramid), regrouped per pair
// of subbands into one (y, x) block and (z, x), (z, y) blocks (ZPair), so the
// R full filter volumes never exist in memory.
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

// Filters of one pair along one z line, from the pair's blocks of the factor
// table (ZPair): psi(z) = C * X[z W + x] * Y[z H + y], one float2 load per
// present factor and voxel (the lanes of a column tile, at consecutive x,
// read consecutive elements of X and one element of Y).  Value e of thread t
// sits at z = t + e NT: the lane's part of the address is one 32-bit byte
// offset (row t), the step e NT rows is wave-uniform, so no per-value
// addresses stay live across the pair loop.
template <bool HX, bool HY>
struct ZFilt {
  const char *X, *Y;    // pair blocks (uniform)
  size_t sx, sy;        // bytes per value step (uniform)
  unsigned ox, oy;      // lane offsets of rows t
  float2 c;
  __device__ __forceinline__ float2 operator()(int e) const {
    float2 f = c;
    if constexpr (HX) {
      const float2 q = *(const float2 *)(X + e * sx + ox);
      f.x *= q.x;
      f.y *= q.y;
    }
    if constexpr (HY) {
      const float2 q = *(const float2 *)(Y + e * sy + oy);
      f.x *= q.x;
      f.y *= q.y;
    }
    return f;
  }
};

// Runs body(filter) with the pair's filter functor.  Which factors a pair has
// is uniform over the block, hence one instance of the body per combination.
// c is the pair's C at this column, which the caller loads one pair ahead.
template <int NT, class Body>
__device__ __forceinline__ void with_zfilters(const float2 *__restrict__ tab, const ZPair &zp,
                                              float2 c, int t, int y, int x, int H, int W,
                                              Body &&body) {
  const char *X = (const char *)(tab + zp.x), *Y = (const char *)(tab + zp.y);
  const size_t sx = (size_t)NT * W * sizeof(float2), sy = (size_t)NT * H * sizeof(float2);
  const unsigned ox = (unsigned)(t * W + x) * (unsigned)sizeof(float2);
  const unsigned oy = (unsigned)(t * H + y) * (unsigned)sizeof(float2);
  if (zp.x >= 0 && zp.y >= 0)
    body(ZFilt<true, true>{X, Y, sx, sy, ox, oy, c});
  else if (zp.x >= 0)
    body(ZFilt<true, false>{X, Y, sx, sy, ox, oy, c});
  else
    body(ZFilt<false, true>{X, Y, sx, sy, ox, oy, c});
}

// z pass of the forward transform: F * (psi_a + i psi_b), inverse DFT along z.
// Columns are the H*W voxels of a z-slice; grid (ceil(HW/M), nb * split):
// each image's pair loop is cut into split parts of consecutive pairs.
template <int N>
__global__ void __launch_bounds__(Tile3<N>::THREADS)
k_z_filter_ifft(const float2 *__restrict__ F, const ZPair *__restrict__ pairs,
                const float2 *__restrict__ tab, float2 *__restrict__ T, int H, int W, int R,
                int b0, int p0, int np, int split, int zdft, const float2 *__restrict__ tw) {
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
  // blockIdx.y = (image of the chunk, part of the pair loop)
  const int bl = blockIdx.y / split, part = blockIdx.y % split;
  const int per = (np + split - 1) / split;
  const int q0 = part * per, q1 = min(np, q0 + per);
  const int b = b0 + bl;
  const size_t vol = (size_t)N * HW;
  float2 f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) f[e] = F[(size_t)b * vol + (size_t)(t + e * NT) * HW + cc];
  // zdft: F holds the x and y transforms only; its DFT along z is taken here,
  // once per block, instead of in a pass of its own over the volume
  if (zdft) fft_line_p<Plan<N>, false>(f, t, LdsLine{lds + m, M}, TwLds{twl});
  float2 cn = q0 < q1 ? (tab + pairs[p0 + q0].c)[y * W + x] : make_float2(0.f, 0.f);
  for (int pp = q0; pp < q1; ++pp) {
    const float2 c = cn;
    if (pp + 1 < q1) cn = (tab + pairs[p0 + pp + 1].c)[y * W + x];
    float2 v[E];
    with_zfilters<NT>(tab, pairs[p0 + pp], c, t, y, x, H, W, [&](const auto &psi) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float2 q = psi(e);
        v[e] = make_float2(f[e].x * q.x - f[e].y * q.y, f[e].y * q.x + f[e].x * q.y);
      }
    });
    fft_line_p<Plan<N>, true>(v, t, LdsLine{lds + m, M}, TwLds{twl});
    if (ok) {
      float2 *To = T + ((size_t)bl * np + pp) * vol + col;
#pragma unroll
      for (int e = 0; e < E; ++e) stream_store(&To[(size_t)(t + e * NT) * HW], v[e]);
    }
  }
}

// z pass of the inverse transform: DFT along z of each pair's U, multiply by
// (psi_a - i psi_b), sum over the pairs of the chunk; the last chunk divides
// by Psi_hat and applies the inverse DFT along z.
// (128- and 192-point lines: at least 4 waves per SIMD, which those
// instances reach at 128 VGPRs (192: 2 spilled); the register allocator
// otherwise settles on 130 and 3 waves.  192^3: 2.53 -> 2.46 ms per inverse)
template <int N>
__global__ void __launch_bounds__(Tile3<N>::THREADS)
    __attribute__((amdgpu_waves_per_eu(N == 128 || N == 192 ? 4 : 1)))
k_z_fft_acc(const float2 *__restrict__ U, const ZPair *__restrict__ pairs,
            const float2 *__restrict__ tab, const float *__restrict__ psi, float2 *__restrict__ ACC,
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
  float2 cn = (tab + pairs[p0].c)[y * W + x];
  // U of pair pp: wave-uniform base per value, one 32-bit lane offset.  Up
  // to 128-point lines the next pair's U is loaded before this pair's
  // transform (128^3: 235 -> 225 us); longer lines lose an occupancy step.
  constexpr bool kAhead = N <= 128;
  const char *Ub = (const char *)(U + (size_t)blockIdx.y * np * vol);
  const unsigned lo = (unsigned)(t * HW + cc) * (unsigned)sizeof(float2);
  auto uload = [&](float2 (&d)[E], int pp) {
    const char *Up = Ub + (size_t)pp * vol * sizeof(float2);
#pragma unroll
    for (int e = 0; e < E; ++e)
      d[e] = stream_load((const float2 *)(Up + (size_t)e * NT * HW * sizeof(float2) + lo));
  };
  float2 nx[E];
  if constexpr (kAhead) uload(nx, 0);
  for (int pp = 0; pp < np; ++pp) {
    const float2 c = cn;
    if (pp + 1 < np) cn = (tab + pairs[p0 + pp + 1].c)[y * W + x];
    float2 v[E];
    if constexpr (kAhead) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = nx[e];
      if (pp + 1 < np) uload(nx, pp + 1);
    } else {
      uload(v, pp);
    }
    fft_line_p<Plan<N>, false>(v, t, LdsLine{lds + m, M}, TwLds{twl});
    with_zfilters<NT>(tab, pairs[p0 + pp], c, t, y, x, H, W, [&](const auto &psi) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float2 q = psi(e);
        acc[e].x += q.x * v[e].x + q.y * v[e].y;
        acc[e].y += q.x * v[e].y - q.y * v[e].x;
      }
    });
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

// Parts to split the forward z pass's pair loop into.  Its blocks run the
// whole pair loop of a chunk, so a grid a little larger than one round of
// resident blocks leaves a mostly idle last round (192^3: 2304 blocks, 1024
// resident, three rounds for 2.25 rounds of work).  Each part reloads its
// column tile of F (1/np of what it writes); the split that minimises the
// rounds per unit of work wins, ties going to fewer parts.  Each part also
// repeats the z DFT of its tile of F when the pass takes that DFT itself.
template <int N>
static int z_split(int nblocks, int np, int num_cu) {
  static int per_cu = -1;
  if (per_cu < 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_z_filter_ifft<N>, Tile3<N>::THREADS,
                                                     0) != hipSuccess || n < 1)
      n = 1;
    per_cu = n;
  }
  const long resident = (long)per_cu * num_cu;
  int best = 1;
  double best_cost = 1e30;
  for (int sp = 1; sp <= 4 && sp <= np; ++sp) {
    const long rounds = ((long)nblocks * sp + resident - 1) / resident;
    const double cost = (double)rounds / sp;
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = sp;
    }
  }
  return best;
}

hipError_t launch_z_filter_ifft(const Sys3D &s, const float2 *F, float2 *T, Chunk c, bool zdft,
                                hipStream_t st) {
  const int HW = s.H * s.W;
  switch (s.D) {
#define X(N)                                                                                  \
  case N: {                                                                                   \
    const int tiles = (HW + Tile3<N>::M - 1) / Tile3<N>::M;                                   \
    const int sp = z_split<N>(tiles * c.nb, c.np, s.num_cu);                                  \
    hipLaunchKernelGGL(k_z_filter_ifft<N>, dim3(tiles, c.nb * sp), dim3(Tile3<N>::THREADS), 0, \
                       st, F, s.pairs, s.tab, T, s.H, s.W, s.R, c.b0, c.p0, c.np, sp,         \
                       (int)zdft, s.twD);                                                     \
    break;                                                                                    \
  }
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
                       dim3(Tile3<N>::THREADS), 0, st, U, s.pairs, s.tab, s.psi, ACC, s.H, s.W, \
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
