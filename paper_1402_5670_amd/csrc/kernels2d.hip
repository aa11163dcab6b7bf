// 2D transform passes on gfx950 (Algorithms 1 and 2 of the paper, computed
// by the convolution theorem, Section 4).
//
// Data flow for a batch (filters psi_hat_i are real and even, so two real
// subbands share one complex transform):
//   forward   x --row DFT--> A --column DFT--> F            (once per image)
//             F * (psi_a + i psi_b) --column IDFT--> T        (per pair)
//             T --row IDFT--> c_a = Re, c_b = Im              (per pair)
//   inverse   c_a + i c_b --row DFT--> U                      (per pair)
//             ACC += (psi_a - i psi_b) * colDFT(U)            (sum over pairs)
//             ACC / Psi_hat --column IDFT--> --row IDFT--> Re  (once per image)
// Re of the last step equals the dual-frame reconstruction because the
// imaginary cross terms psi_a C_b - psi_b C_a have Hermitian spectra and
// therefore transform to purely imaginary signals.
//
// Each block owns M lines of one image; the FFT of a line runs in registers
// with LDS exchanges between radix stages (fft_core.hpp).  Row passes read
// and write whole rows; column passes move M adjacent columns per row.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "dispatch.hpp"
#include "fft_core.hpp"

namespace sl {

// Row tiles: M rows per block.  Column tiles: M adjacent columns per block;
// with SL_COL_EMUL > 1 each thread of a column pass owns SL_COL_EMUL times
// more values, halving the threads per column and doubling the columns per
// block (wider coalesced segments) for lengths 256..512.
#ifndef SL_COL_EMUL
#define SL_COL_EMUL 1
#endif
// EM (line plan): each thread holds EM times the plan's values, so a line
// takes EM times fewer threads (EM = 2 makes a 1024-point row one wavefront,
// whose radix exchanges need no block barrier); the coefficient row passes
// take it per system (sl_system_set_line_plan, autotuned for uneven
// batches), and so does the inverse accumulation of 1024-point columns
// (launch_cols_fft_acc); the other column passes keep EM = 1.
template <int N, int EM = 1>
struct Tile {
  using PL = Plan<N, EM>;
  static constexpr int NT = PL::NT;
  static constexpr int E = PL::E;
  static constexpr int M = NT >= 128 ? 8 : 16;     // lines per block
  static constexpr int THREADS = M * NT;
};
// row FFT of a Tile line: wavefront-local exchanges when the line fits a wave
template <int N, int EM, bool INV>
__device__ __forceinline__ void row_fft(float2 (&v)[(Tile<N, EM>::E)], int t, const LdsLine &lds,
                                        const float2 *__restrict__ tw) {
  fft_line_p<Plan<N, EM>, INV, wave_lines<Plan<N, EM>::NT>()>(v, t, lds, tw);
}
// line plans with EM = 2 exist for these lengths
template <int N>
constexpr bool em2_length() { return N == 1024; }
template <int N>
struct CTile {
  static constexpr int EM = (N >= 256 && N <= 512) ? SL_COL_EMUL : 1;
  using PL = Plan<N, EM>;
  static constexpr int NT = PL::NT;
  static constexpr int E = PL::E;
  static constexpr int M = (NT * 16 <= 1024 ? 16 : 8) * (EM > 1 ? 2 : 1);
  static constexpr int THREADS = M * NT;
};

// ---------------------------------------------------------------------------
// storage encode / decode
// ---------------------------------------------------------------------------
template <int DT>
struct Store;
// T is the element type of the coefficient tensor; Raw its bit pattern as a
// plain scalar (kernels load and store Raw values, so that all loads of a row
// can be issued before the first conversion).
template <>
struct Store<0> {
  using T = float;
  using Raw = float;
  __device__ static T enc(float v) { return v; }
  __device__ static float dec(T v) { return v; }
  __device__ static Raw enc_raw(float v) { return v; }
  __device__ static float dec_raw(Raw v) { return v; }
};
template <>
struct Store<1> {
  using T = __half;
  using Raw = unsigned short;
  __device__ static T enc(float v) { return __float2half_rn(v); }
  __device__ static float dec(T v) { return __half2float(v); }
  __device__ static Raw enc_raw(float v) { return __half_as_ushort(__float2half_rn(v)); }
  __device__ static float dec_raw(Raw v) { return __half2float(__ushort_as_half(v)); }
};
template <>
struct Store<2> {
  using T = __hip_bfloat16;
  using Raw = unsigned short;
  __device__ static T enc(float v) { return __float2bfloat16(v); }
  __device__ static float dec(T v) { return __bfloat162float(v); }
  __device__ static Raw enc_raw(float v) { return __bfloat16_as_ushort(__float2bfloat16(v)); }
  __device__ static float dec_raw(Raw v) { return __uint_as_float((unsigned)v << 16); }
};

// Coefficient planes are streamed once per call; with SL_NT_COEF the float32
// coefficient stores and loads carry the non-temporal hint so that they do
// not displace the pass intermediates from the caches.
#ifndef SL_NT_COEF
#define SL_NT_COEF 0
#endif
template <class T>
__device__ __forceinline__ void coef_store(T *p, T v) {
  if constexpr (SL_NT_COEF && sizeof(T) == 4) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <class T>
__device__ __forceinline__ T coef_load(const T *p) {
  if constexpr (SL_NT_COEF && sizeof(T) == 4) return __builtin_nontemporal_load(p);
  else return *p;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// MIX = 0: rows of x; MIX = 1 / 2: rows of the inpainting input (MixArgs),
// first iteration / later ones.
template <int N, int MIX>
__global__ void __launch_bounds__(Tile<N>::THREADS)
k_rows_real_fft(const float *__restrict__ x, float2 *__restrict__ A, unsigned *__restrict__ xmax,
                int H, const float2 *__restrict__ tw, MixArgs mix, int B) {
  constexpr int NT = Tile<N>::NT, M = Tile<N>::M, E = Tile<N>::E;
  __shared__ float2 lds[M * row_lds_len<N>()];
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int row = blockIdx.x * M + m, b = blockIdx.y;
  const bool ok = row < H;
  const size_t off = ((size_t)b * H + (ok ? row : 0)) * N;
  if (MIX && blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < B; i += blockDim.x) mix.sigma[i] = mix.delta_init[i] * mix.fac;
  float2 v[E];
  float amax = 0.f;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    float a = 0.f;
    if (ok) {
      const size_t i = off + t + e * NT;
      if constexpr (MIX == 0) {
        a = x[i];
      } else {
        // all three loads issued together, then the selection
        const unsigned char known = mix.mask[i];
        const float fm = mix.fm[i], fe = MIX == 2 ? mix.f[i] : 0.f;
        a = known ? fm : fe;
      }
    }
    v[e] = make_float2(a, 0.f);
    amax = fmaxf(amax, fabsf(a));
  }
  if (xmax) {
    if constexpr (Tile<N>::THREADS % 64 == 0) {
      // one atomic per block: wave maxima through LDS (the FFT's LDS is not
      // in use yet)
      constexpr int NWV = Tile<N>::THREADS / 64;
      float *wm = (float *)lds;
      amax = wave_max(amax);
      if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = amax;
      __syncthreads();
      if (threadIdx.x == 0) {
        float mm = wm[0];
#pragma unroll
        for (int w = 1; w < NWV; ++w) mm = fmaxf(mm, wm[w]);
        atomicMax(xmax + b, __float_as_uint(mm));
      }
      __syncthreads();
    } else {
      atomicMax(xmax + b, __float_as_uint(amax));   // partial wave: no cross-lane reduction
    }
  }
  fft_line<N, false>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) A[off + t + e * NT] = v[e];
  }
}

// NT: A and F are pair-plane streams (non-temporal accesses)
template <int N, bool INV, bool NT_>
__global__ void __launch_bounds__(CTile<N>::THREADS)
k_cols_fft(const float2 *__restrict__ A, float2 *__restrict__ F, int W,
           const float2 *__restrict__ tw) {
  constexpr int NT = CTile<N>::NT, M = CTile<N>::M, E = CTile<N>::E;
  using PL = typename CTile<N>::PL;
  __shared__ float2 lds[M * N];
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < W;
  const size_t base = (size_t)blockIdx.y * N * W + (ok ? col : 0);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = ok ? stream_load<NT_>(&A[base + (size_t)(t + e * NT) * W]) : make_float2(0.f, 0.f);
  fft_line_p<PL, INV>(v, t, LdsLine{lds + m, M}, tw);
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) stream_store<NT_>(&F[base + (size_t)(t + e * NT) * W], v[e]);
  }
}

// Images per column block: the filter pair tile is loaded once and applied
// to BT images (fewer filter re-reads, more registers).  Measured on MI355X
// for 32 x 512^2: BT = 1 is best for the forward column pass, BT = 2 for the
// inverse accumulation pass.
#ifndef SL_INV_BT
#define SL_INV_BT 2
#endif
constexpr int kFwdBT = 1, kInvBT = SL_INV_BT;

template <int N, int BT>
__global__ void __launch_bounds__(CTile<N>::THREADS)
k_cols_filter_ifft(const float2 *__restrict__ F, const float *__restrict__ filt,
                   float2 *__restrict__ T, int W, int R, int b0, int nb, int p0, int np,
                   const float2 *__restrict__ tw) {
  constexpr int NT = CTile<N>::NT, M = CTile<N>::M, E = CTile<N>::E;
  using PL = typename CTile<N>::PL;
  __shared__ float2 lds[M * N];
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < W;
  const int cc = ok ? col : 0;
  const size_t plane = (size_t)N * W;
  float2 f[BT][E];
#pragma unroll
  for (int bt = 0; bt < BT; ++bt) {
    const int bl = blockIdx.y * BT + bt;
    const int b = b0 + (bl < nb ? bl : 0);
#pragma unroll
    for (int e = 0; e < E; ++e) f[bt][e] = F[(size_t)b * plane + (size_t)(t + e * NT) * W + cc];
  }
  for (int pp = 0; pp < np; ++pp) {
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const float *fa = filt + (size_t)ia * plane + cc;
    const float *fb = filt + (size_t)(ib < R ? ib : ia) * plane + cc;
    float a[E], bb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t o = (size_t)(t + e * NT) * W;
      a[e] = fa[o];
      bb[e] = ib < R ? fb[o] : 0.f;
    }
#pragma unroll
    for (int bt = 0; bt < BT; ++bt) {
      const int bl = blockIdx.y * BT + bt;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e)
        v[e] = make_float2(f[bt][e].x * a[e] - f[bt][e].y * bb[e],
                           f[bt][e].y * a[e] + f[bt][e].x * bb[e]);
      fft_line_p<PL, true>(v, t, LdsLine{lds + m, M}, tw);
      if (ok && bl < nb) {
        float2 *To = T + ((size_t)bl * np + pp) * plane + col;
#pragma unroll
        for (int e = 0; e < E; ++e) stream_store(&To[(size_t)(t + e * NT) * W], v[e]);
      }
    }
  }
}

// Column passes, variant with the twiddles staged in LDS, 32-bit element
// offsets (thread (m, t) of a tile owns rows t + e NT of column col, at
// element offset o0 + e se from a uniform plane base, o0 = t W + col,
// se = NT W; planes hold at most 1024 x 1024 values) and the next subband
// pair's operands fetched before the current pair's FFT.
// Measured on the 32 x 512^2 batch: this variant is 13% faster for the
// forward pass (the prefetch hides the filter loads) and 20% slower for the
// inverse accumulation (two FFTs per filter load there favour twiddles held
// in registers), so only the forward uses it by default.
#ifndef SL_COL_V3_FWD
#define SL_COL_V3_FWD 1
#endif
#ifndef SL_COL_V3_INV
#define SL_COL_V3_INV 0
#endif
// Column tile of the forward filter pass: MW columns per block (at most the
// generic column tile's width).  On the 32 x 512^2 batch 8 columns (two
// blocks per CU) was 30% slower than 16 with tiles in linear order; with the
// XCD-grouped order of col_tile() the step is the same and the fused denoise
// 1.5% slower, while a single image gains (one 512^2 image, R = 49: 4% per
// inpainting iteration), so a chunk of one image takes 8 columns; its pair
// planes (50 MB at 512^2, R = 49) stay in the Infinity Cache between the
// passes, so that instance stores them without the non-temporal hint (3% per
// iteration).  Forcing more waves per SIMD (amdgpu_waves_per_eu) spills
// registers.
constexpr int kFwdWide = 16, kFwdNarrow = 8;
template <int N, int MW, int EM = 1>
struct FTile {
  using PL = Plan<N, EM>;
  static constexpr int NT = PL::NT;
  static constexpr int E = PL::E;
  static constexpr int MC = EM == 1 ? CTile<N>::M : (NT * 16 <= 1024 ? 16 : 8);
  static constexpr int M = MC < MW ? MC : MW;
  static constexpr int THREADS = M * NT;
};

template <int N>
__device__ __forceinline__ void stage_twiddles(float2 *twl, const float2 *__restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = tw[i];
}

template <int N, int BT, int MW, int EM = 1>
__global__ void __launch_bounds__((FTile<N, MW, EM>::THREADS))
k_cols_filter_ifft3(const float2 *__restrict__ F, const float *__restrict__ filt,
                    float2 *__restrict__ T, int W, int R, int b0, int nb, int p0, int np,
                    const float2 *__restrict__ tw) {
  constexpr int NT = FTile<N, MW, EM>::NT, M = FTile<N, MW, EM>::M, E = FTile<N, MW, EM>::E;
  using PL = typename FTile<N, MW, EM>::PL;
  __shared__ float2 lds[M * N];
  __shared__ float2 twl[N];
  stage_twiddles<N>(twl, tw);       // the FFT's leading barrier orders it
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < W;
  const size_t plane = (size_t)N * W;
  // Element (row t + e NT, column col) of a plane.  With two images per
  // block, a wave-uniform base (plane, row step e NT) plus one 32-bit lane
  // byte offset keeps the per-value addresses out of the registers the
  // second image needs; one image per block keeps 32-bit element offsets
  // (measured 10 us faster at 512^2).
  const unsigned o0 = (unsigned)t * W + (ok ? col : 0), se = (unsigned)NT * W;
  const unsigned lo = o0 * 8u, lo4 = lo / 2;
  const size_t sb8 = (size_t)NT * W * 8, sb4 = sb8 / 2;
  auto at8 = [&](const float2 *base, int e) -> const float2 * {
    if constexpr (BT > 1) return (const float2 *)((const char *)base + e * sb8 + lo);
    return base + (o0 + e * se);
  };
  auto at4 = [&](const float *base, int e) -> const float * {
    if constexpr (BT > 1) return (const float *)((const char *)base + e * sb4 + lo4);
    return base + (o0 + e * se);
  };
  // pairs [q0, q1) of the chunk: gridDim.z groups split the pair loop when
  // the column tiles alone would leave compute units idle (small batches)
  const int per = (np + (int)gridDim.z - 1) / (int)gridDim.z;
  const int q0 = (int)blockIdx.z * per, q1 = min(np, q0 + per);
  if (q0 >= q1) return;
  float2 f[BT][E];
#pragma unroll
  for (int bt = 0; bt < BT; ++bt) {
    const int bl = blockIdx.y * BT + bt;
    const float2 *Fb = F + (size_t)(b0 + (bl < nb ? bl : 0)) * plane;
#pragma unroll
    for (int e = 0; e < E; ++e) f[bt][e] = *at8(Fb, e);
  }
  auto load_pair = [&](int pp, float(&a)[E], float(&b)[E]) {
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const float *fa = filt + (size_t)ia * plane;
    const float *fb = filt + (size_t)(ib < R ? ib : ia) * plane;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = *at4(fa, e);
      b[e] = *at4(fb, e);
    }
    if (ib >= R) {
#pragma unroll
      for (int e = 0; e < E; ++e) b[e] = 0.f;
    }
  };
  float a[E], bb[E];
  load_pair(q0, a, bb);
  for (int pp = q0; pp < q1; ++pp) {
    float2 v[BT][E];
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
#pragma unroll
      for (int e = 0; e < E; ++e)
        v[bt][e] = make_float2(f[bt][e].x * a[e] - f[bt][e].y * bb[e],
                               f[bt][e].y * a[e] + f[bt][e].x * bb[e]);
    if (pp + 1 < q1) load_pair(pp + 1, a, bb);   // lands during the FFTs below
#pragma unroll
    for (int bt = 0; bt < BT; ++bt) {
      const int bl = blockIdx.y * BT + bt;
      fft_line_p<PL, true>(v[bt], t, LdsLine{lds + m, M}, TwLds{twl});
      if (ok && bl < nb) {
        float2 *To = T + ((size_t)bl * np + pp) * plane;
#pragma unroll
        for (int e = 0; e < E; ++e) stream_store<SL_NT_STREAM && MW != kFwdNarrow>((float2 *)at8(To, e), v[bt][e]);
      }
    }
  }
}

template <int N, int BT>
__global__ void __launch_bounds__(CTile<N>::THREADS)
k_cols_fft_acc3(const float2 *__restrict__ U, const float *__restrict__ filt,
                const float *__restrict__ psi, float2 *__restrict__ ACC, int W, int R, int b0,
                int nb, int p0, int np, int first, int last, const float2 *__restrict__ tw) {
  constexpr int NT = CTile<N>::NT, M = CTile<N>::M, E = CTile<N>::E;
  using PL = typename CTile<N>::PL;
  __shared__ float2 lds[M * N];
  __shared__ float2 twl[N];
  stage_twiddles<N>(twl, tw);
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < W;
  const unsigned o0 = (unsigned)t * W + (ok ? col : 0), se = (unsigned)NT * W;
  const size_t plane = (size_t)N * W;
  float2 acc[BT][E];
#pragma unroll
  for (int bt = 0; bt < BT; ++bt) {
    const int bl = blockIdx.y * BT + bt;
    const float2 *accp = ACC + (size_t)(b0 + (bl < nb ? bl : 0)) * plane;
#pragma unroll
    for (int e = 0; e < E; ++e)
      acc[bt][e] = first ? make_float2(0.f, 0.f) : accp[o0 + e * se];
  }
  for (int pp = 0; pp < np; ++pp) {
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const float *fa = filt + (size_t)ia * plane;
    const float *fb = filt + (size_t)(ib < R ? ib : ia) * plane;
    // filter pair first: only needed after the FFTs
    float a[E], bb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = fa[o0 + e * se];
      bb[e] = fb[o0 + e * se];
    }
    if (ib >= R) {
#pragma unroll
      for (int e = 0; e < E; ++e) bb[e] = 0.f;
    }
#pragma unroll
    for (int bt = 0; bt < BT; ++bt) {
      const int bl = blockIdx.y * BT + bt;
      const float2 *Ui = U + ((size_t)(bl < nb ? bl : 0) * np + pp) * plane;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = stream_load(&Ui[o0 + e * se]);
      fft_line_p<PL, false>(v, t, LdsLine{lds + m, M}, TwLds{twl});
#pragma unroll
      for (int e = 0; e < E; ++e) {
        // (psi_a - i psi_b) * v
        acc[bt][e].x += a[e] * v[e].x + bb[e] * v[e].y;
        acc[bt][e].y += a[e] * v[e].y - bb[e] * v[e].x;
      }
    }
  }
#pragma unroll
  for (int bt = 0; bt < BT; ++bt) {
    const int bl = blockIdx.y * BT + bt;
    if (last) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float d = psi[o0 + e * se];
        acc[bt][e] = make_float2(acc[bt][e].x / d, acc[bt][e].y / d);
      }
      fft_line_p<PL, true>(acc[bt], t, LdsLine{lds + m, M}, TwLds{twl});
    }
    if (ok && bl < nb) {
      float2 *accp = ACC + (size_t)(b0 + bl) * plane;
#pragma unroll
      for (int e = 0; e < E; ++e) accp[o0 + e * se] = acc[bt][e];
    }
  }
}

template <int N, int DT, int EM = 1>
__global__ void __launch_bounds__((Tile<N, EM>::THREADS))
k_rows_coef(const float2 *__restrict__ T, typename Store<DT>::T *__restrict__ coef,
            const float *__restrict__ scales, int H, int R, int b0, int p0, int np, float inv_hw,
            const float2 *__restrict__ tw) {
  constexpr int NT = Tile<N, EM>::NT, M = Tile<N, EM>::M, E = Tile<N, EM>::E;
  __shared__ float2 lds[M * row_lds_len<N>()];
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int row = blockIdx.x * M + m;
  const bool ok = row < H;
  const int rr = ok ? row : 0;
  const int pp = blockIdx.y, bl = blockIdx.z, b = b0 + bl;
  const int ia = 2 * (p0 + pp), ib = ia + 1;
  const size_t plane = (size_t)H * N;
  const float2 *Ti = T + ((size_t)bl * np + pp) * plane + (size_t)rr * N;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = Ti[t + e * NT];
  row_fft<N, EM, true>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
  if (!ok) return;
  float sa = inv_hw, sb = inv_hw;
  if (DT != 0) {
    sa = inv_hw / scales[(size_t)b * R + ia];
    if (ib < R) sb = inv_hw / scales[(size_t)b * R + ib];
  }
  using Raw = typename Store<DT>::Raw;
  Raw *ca = (Raw *)(coef + ((size_t)b * R + ia) * plane + (size_t)row * N);
#pragma unroll
  for (int e = 0; e < E; ++e) coef_store(ca + t + e * NT, Store<DT>::enc_raw(v[e].x * sa));
  if (ib < R) {
    Raw *cb = (Raw *)(coef + ((size_t)b * R + ib) * plane + (size_t)row * N);
#pragma unroll
    for (int e = 0; e < E; ++e) coef_store(cb + t + e * NT, Store<DT>::enc_raw(v[e].y * sb));
  }
}

// k_rows_coef with the row-group loop and next-row prefetch of k_rows_thr,
// used for 16-bit storage, whose stores are half as long (32 x 512^2 FP16:
// step 2.29 -> 2.21 ms; with FP32 coefficients it was 4% slower)
// Body of the prefetching coefficient row pass for one block: M lines of NT
// threads, row groups gx, gx + G, ... of pair pp of chunk image bl.  Shared
// by k_rows_coef_pf (grid = (G, np, nb)) and the multi-class row pass.
template <int N, int DT, int EM, int M>
__device__ __forceinline__ void rows_coef_pf_body(float2 *lds, const float2 *__restrict__ T,
                                                  typename Store<DT>::T *__restrict__ coef,
                                                  const float *__restrict__ scales, int H, int R,
                                                  int b0, int p0, int np, float inv_hw,
                                                  const float2 *__restrict__ tw, int gx, int G,
                                                  int pp, int bl) {
  constexpr int NT = Tile<N, EM>::NT, E = Tile<N, EM>::E;
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int b = b0 + bl;
  const int ia = 2 * (p0 + pp), ib = ia + 1;
  const size_t plane = (size_t)H * N;
  const float2 *Tp = T + ((size_t)bl * np + pp) * plane;
  float sa = inv_hw, sb = inv_hw;
  if (DT != 0) {
    sa = inv_hw / scales[(size_t)b * R + ia];
    if (ib < R) sb = inv_hw / scales[(size_t)b * R + ib];
  }
  using Raw = typename Store<DT>::Raw;
  Raw *ca0 = (Raw *)(coef + ((size_t)b * R + ia) * plane);
  Raw *cb0 = (Raw *)(coef + ((size_t)b * R + (ib < R ? ib : ia)) * plane);
  const int nrg = (H + M - 1) / M;
  float2 nx[E];
  auto load = [&](int rg) {
    const int row = rg * M + m;
    const float2 *src = Tp + (size_t)(row < H ? row : 0) * N;
#pragma unroll
    for (int e = 0; e < E; ++e) nx[e] = src[t + e * NT];
  };
  if (gx < nrg) load(gx);
  for (int rg = gx; rg < nrg; rg += G) {
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = nx[e];
    if (rg + G < nrg) load(rg + G);
    row_fft<N, EM, true>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
    const int row = rg * M + m;
    if (row < H) {
      Raw *ca = ca0 + (size_t)row * N;
#pragma unroll
      for (int e = 0; e < E; ++e) coef_store(ca + t + e * NT, Store<DT>::enc_raw(v[e].x * sa));
      if (ib < R) {
        Raw *cb = cb0 + (size_t)row * N;
#pragma unroll
        for (int e = 0; e < E; ++e) coef_store(cb + t + e * NT, Store<DT>::enc_raw(v[e].y * sb));
      }
    }
  }
}

template <int N, int DT, int EM = 1>
__global__ void __launch_bounds__((Tile<N, EM>::THREADS / 2 > 0 ? Tile<N, EM>::THREADS / 2 : 1))
k_rows_coef_pf(const float2 *__restrict__ T, typename Store<DT>::T *__restrict__ coef,
               const float *__restrict__ scales, int H, int R, int b0, int p0, int np,
               float inv_hw, const float2 *__restrict__ tw) {
  constexpr int M = Tile<N, EM>::M / 2 > 0 ? Tile<N, EM>::M / 2 : 1;
  __shared__ float2 lds[M * row_lds_len<N>()];
  rows_coef_pf_body<N, DT, EM, M>(lds, T, coef, scales, H, R, b0, p0, np, inv_hw, tw,
                                  (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y,
                                  (int)blockIdx.z);
}

// scale_{b,i} = 2^(ceil(log2(max|x_b| * ||psi_i||_1)) - 15): |c| <= max|x| ||psi||_1
// (Young), so the stored values stay below 2^15 in magnitude.
__global__ void k_scales(const unsigned *__restrict__ xmax, const float *__restrict__ l1,
                         float *__restrict__ scales, int B, int R) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * R) return;
  float bound = __uint_as_float(xmax[i / R]) * l1[i % R];
  scales[i] = bound > 0.f ? exp2f(ceilf(log2f(bound)) - 15.f) : 1.f;
}

// F[b][p] /= Psi_hat[p]: turns the forward transform into the adjoint of the
// inverse (dual filters psi_hat_i / Psi_hat, eq. dual_filter).
__global__ void k_div_psi(float2 *__restrict__ F, const float *__restrict__ psi, size_t npix) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npix) return;
  const float d = psi[k];
  float2 *f = F + (size_t)blockIdx.y * npix + k;
  *f = make_float2(f->x / d, f->y / d);
}

__global__ void k_zero_u32(unsigned *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// inverse
// ---------------------------------------------------------------------------
template <int N, int DT, int EM = 1>
__global__ void __launch_bounds__((Tile<N, EM>::THREADS))
k_rows_coef_fft(const typename Store<DT>::T *__restrict__ coef, const float *__restrict__ scales,
                float2 *__restrict__ U, int H, int R, int b0, int p0, int np, ThrArgs thr,
                const float2 *__restrict__ tw) {
  constexpr int NT = Tile<N, EM>::NT, M = Tile<N, EM>::M, E = Tile<N, EM>::E;
  __shared__ float2 lds[M * row_lds_len<N>()];
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int row = blockIdx.x * M + m;
  const bool ok = row < H;
  const int rr = ok ? row : 0;
  const int pp = blockIdx.y, bl = blockIdx.z, b = b0 + bl;
  const int ia = 2 * (p0 + pp), ib = ia + 1;
  const bool has_b = ib < R;
  const size_t plane = (size_t)H * N;
  float sa = 1.f, sb = 1.f;
  if (DT != 0) {
    sa = scales[(size_t)b * R + ia];
    if (has_b) sb = scales[(size_t)b * R + ib];
  }
  float da = 0.f, db = 0.f;
  if (thr.sigma) {
    const float sg = thr.sigma[b];
    const int ja = thr.jof[ia];
    if (ja >= 0) da = (thr.K[ja] * sg) * thr.l2[ia];
    if (has_b) {
      const int jb = thr.jof[ib];
      if (jb >= 0) db = (thr.K[jb] * sg) * thr.l2[ib];
    }
  }
  using Raw = typename Store<DT>::Raw;
  const Raw *ca = (const Raw *)(coef + ((size_t)b * R + ia) * plane + (size_t)rr * N);
  const Raw *cb = (const Raw *)(coef + ((size_t)b * R + (has_b ? ib : ia)) * plane + (size_t)rr * N);
  Raw ra[E], rb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ra[e] = coef_load(ca + t + e * NT);
    rb[e] = coef_load(cb + t + e * NT);   // a valid plane; ignored without a partner
  }
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    float a = Store<DT>::dec_raw(ra[e]) * sa;
    float bb = has_b ? Store<DT>::dec_raw(rb[e]) * sb : 0.f;
    if (!(fabsf(a) >= da)) a = 0.f;
    if (!(fabsf(bb) >= db)) bb = 0.f;
    v[e] = make_float2(a, bb);
  }
  row_fft<N, EM, false>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
  if (ok) {
    float2 *Uo = U + ((size_t)bl * np + pp) * plane + (size_t)row * N;
#pragma unroll
    for (int e = 0; e < E; ++e) Uo[t + e * NT] = v[e];
  }
}


// k_rows_coef_fft with the row-group loop and next-row prefetch (both
// coefficient rows of the pair) of k_rows_thr, used for 16-bit storage
// (32 x 512^2 FP16: step 2.24 -> 2.18 ms)
// Body of the prefetching inverse coefficient row pass for one block (as
// rows_coef_pf_body): shared by k_rows_coef_fft_pf and the multi-class pass.
template <int N, int DT, int EM, int M>
__device__ __forceinline__ void rows_coef_fft_pf_body(
    float2 *lds, const typename Store<DT>::T *__restrict__ coef, const float *__restrict__ scales,
    float2 *__restrict__ U, int H, int R, int b0, int p0, int np, const ThrArgs &thr,
    const float2 *__restrict__ tw, int gx, int G, int pp, int bl) {
  constexpr int NT = Tile<N, EM>::NT, E = Tile<N, EM>::E;
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int b = b0 + bl;
  const int ia = 2 * (p0 + pp), ib = ia + 1;
  const bool has_b = ib < R;
  const size_t plane = (size_t)H * N;
  float sa = 1.f, sb = 1.f;
  if (DT != 0) {
    sa = scales[(size_t)b * R + ia];
    if (has_b) sb = scales[(size_t)b * R + ib];
  }
  float da = 0.f, db = 0.f;
  if (thr.sigma) {
    const float sg = thr.sigma[b];
    const int ja = thr.jof[ia];
    if (ja >= 0) da = (thr.K[ja] * sg) * thr.l2[ia];
    if (has_b) {
      const int jb = thr.jof[ib];
      if (jb >= 0) db = (thr.K[jb] * sg) * thr.l2[ib];
    }
  }
  using Raw = typename Store<DT>::Raw;
  const Raw *ca0 = (const Raw *)(coef + ((size_t)b * R + ia) * plane);
  const Raw *cb0 = (const Raw *)(coef + ((size_t)b * R + (has_b ? ib : ia)) * plane);
  float2 *Up = U + ((size_t)bl * np + pp) * plane;
  const int nrg = (H + M - 1) / M;
  Raw na[E], nb_[E];
  auto load = [&](int rg) {
    const int row = rg * M + m;
    const size_t o = (size_t)(row < H ? row : 0) * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      na[e] = coef_load(ca0 + o + t + e * NT);
      nb_[e] = coef_load(cb0 + o + t + e * NT);   // a valid plane; ignored without a partner
    }
  };
  if (gx < nrg) load(gx);
  for (int rg = gx; rg < nrg; rg += G) {
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float a = Store<DT>::dec_raw(na[e]) * sa;
      float bb = has_b ? Store<DT>::dec_raw(nb_[e]) * sb : 0.f;
      if (!(fabsf(a) >= da)) a = 0.f;
      if (!(fabsf(bb) >= db)) bb = 0.f;
      v[e] = make_float2(a, bb);
    }
    if (rg + G < nrg) load(rg + G);
    row_fft<N, EM, false>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
    const int row = rg * M + m;
    if (row < H) {
      float2 *Uo = Up + (size_t)row * N;
#pragma unroll
      for (int e = 0; e < E; ++e) Uo[t + e * NT] = v[e];
    }
  }
}

template <int N, int DT, int EM = 1>
__global__ void __launch_bounds__((Tile<N, EM>::THREADS / 2 > 0 ? Tile<N, EM>::THREADS / 2 : 1))
k_rows_coef_fft_pf(const typename Store<DT>::T *__restrict__ coef, const float *__restrict__ scales,
                   float2 *__restrict__ U, int H, int R, int b0, int p0, int np, ThrArgs thr,
                   const float2 *__restrict__ tw) {
  constexpr int M = Tile<N, EM>::M / 2 > 0 ? Tile<N, EM>::M / 2 : 1;
  __shared__ float2 lds[M * row_lds_len<N>()];
  rows_coef_fft_pf_body<N, DT, EM, M>(lds, coef, scales, U, H, R, b0, p0, np, thr, tw,
                                      (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y,
                                      (int)blockIdx.z);
}


// ---------------------------------------------------------------------------
// Multi-class coefficient row passes (uneven batches): one launch covers the
// row blocks of every size class of a schedule step.  The flat block index
// is the work list: class c owns blocks [block0_c, block0_c+1), listed
// largest class first, and a block of class c decodes (row group, pair,
// image) from its local index as the single-class launch's grid would.  A
// block has 512 threads; a class of line length N runs 512 / NT lines per
// block with the wavefront-local line FFT of its plan (1024-point lines use
// the 16-values-per-thread plan), and the dynamic LDS holds the largest
// class's rows.
// ---------------------------------------------------------------------------
constexpr int kMultiThreads = 512;

template <int N, int DT, int EM, bool FWD>
__device__ __forceinline__ void multi_row_class(const MultiRowClass &k, float2 *lds, int gx,
                                                int pp, int bl) {
  constexpr int M = kMultiThreads / Plan<N, EM>::NT;
  using CT = typename Store<DT>::T;
  if constexpr (FWD)
    rows_coef_pf_body<N, DT, EM, M>(lds, k.T, (CT *)k.coef, k.scales, k.H, k.R, k.b0, k.p0, k.np,
                                    k.inv_hw, k.tw, gx, k.G, pp, bl);
  else
    rows_coef_fft_pf_body<N, DT, EM, M>(lds, (const CT *)k.coef, k.scales, k.U, k.H, k.R, k.b0,
                                        k.p0, k.np, k.thr, k.tw, gx, k.G, pp, bl);
}

#define SL_MULTI_ROW_LENGTHS(X) X(64, 1) X(96, 1) X(128, 1) X(192, 1) X(256, 1) X(384, 1) \
  X(512, 1) X(768, 1) X(1024, 2)

template <int DT, bool FWD>
__global__ void __launch_bounds__(kMultiThreads) k_rows_multi(MultiRows a) {
  extern __shared__ float2 mlds[];
  int c = 0;
  while (c + 1 < a.n && (int)blockIdx.x >= a.c[c + 1].block0) ++c;
  const MultiRowClass &k = a.c[c];
  const int local = (int)blockIdx.x - k.block0;
  const int gx = local % k.G, pp = (local / k.G) % k.np, bl = local / (k.G * k.np);
  switch (k.W) {
#define X(N, EM)                                                   \
  case N:                                                          \
    multi_row_class<N, DT, EM, FWD>(k, mlds, gx, pp, bl);          \
    break;
    SL_MULTI_ROW_LENGTHS(X)
#undef X
  }
}

// lines per block and LDS bytes of a class in the multi-class row pass (0 if
// its length has no wavefront-local plan here)
static int multi_row_lines(int W, size_t *lds_bytes) {
  switch (W) {
#define X(N, EM)                                                                           \
  case N:                                                                                  \
    if (lds_bytes)                                                                         \
      *lds_bytes = (size_t)(kMultiThreads / Plan<N, EM>::NT) * row_lds_len<N>() * sizeof(float2); \
    return kMultiThreads / Plan<N, EM>::NT;
    SL_MULTI_ROW_LENGTHS(X)
#undef X
    default:
      return 0;
  }
}

bool multi_rows_supported(const Sys2D &s) {
  return multi_row_lines(s.W, nullptr) > 0 && (s.W != 1024 || s.line_em == 2);
}

void multi_rows_class_geometry(const Sys2D &s, const Chunk &c, MultiRowClass &k) {
  const int M = multi_row_lines(s.W, nullptr);
  const int nrg = (s.H + M - 1) / M;
  int G = nrg / 8 > 1 ? nrg / 8 : 1;
  if ((long)G * c.np * c.nb < 8L * s.num_cu) G = nrg;
  k.W = s.W;
  k.H = s.H;
  k.R = s.R;
  k.b0 = c.b0;
  k.p0 = c.p0;
  k.np = c.np;
  k.G = G;
  k.nblocks = G * c.np * c.nb;
  k.tw = s.twW;
  k.inv_hw = 1.0f / ((float)s.H * (float)s.W);
}

hipError_t launch_rows_multi(MultiRows &a, int dtype, bool forward, hipStream_t st) {
  if (a.n < 1 || a.n > kMaxMultiClasses) return hipErrorInvalidValue;
  // largest classes first: their blocks are dispatched first
  for (int i = 1; i < a.n; ++i)
    for (int j = i; j > 0 && (long)a.c[j].nblocks * a.c[j].W > (long)a.c[j - 1].nblocks * a.c[j - 1].W; --j) {
      const MultiRowClass t = a.c[j];
      a.c[j] = a.c[j - 1];
      a.c[j - 1] = t;
    }
  size_t lds = 0;
  int total = 0;
  for (int i = 0; i < a.n; ++i) {
    size_t b = 0;
    if (multi_row_lines(a.c[i].W, &b) == 0) return hipErrorInvalidValue;
    lds = b > lds ? b : lds;
    a.c[i].block0 = total;
    total += a.c[i].nblocks;
  }
  if (total < 1) return hipSuccess;
  const dim3 grid(total), block(kMultiThreads);
  if (forward) {
    if (dtype == 1) hipLaunchKernelGGL((k_rows_multi<1, true>), grid, block, lds, st, a);
    else if (dtype == 2) hipLaunchKernelGGL((k_rows_multi<2, true>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((k_rows_multi<0, true>), grid, block, lds, st, a);
  } else {
    if (dtype == 1) hipLaunchKernelGGL((k_rows_multi<1, false>), grid, block, lds, st, a);
    else if (dtype == 2) hipLaunchKernelGGL((k_rows_multi<2, false>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((k_rows_multi<0, false>), grid, block, lds, st, a);
  }
  return hipGetLastError();
}

// Denoising without materialised coefficients: the forward transform's last
// row pass and the inverse transform's first row pass on one row of a pair
// plane.  T holds the column-transformed pair (c_a + i c_b before its row
// IDFT); the row IDFT scaled by 1/n gives the float32 coefficients exactly as
// k_rows_coef stores them, the hard threshold of k_rows_coef_fft is applied,
// and the row DFT of the thresholded pair is written back in place (it is
// the U of the inverse's column pass).
// The blocks loop over row groups of their plane and load the next group's
// rows while transforming the current ones (with two FFTs per row the loads
// are otherwise exposed: 1.07 -> 0.65 ms on 32 x 512^2, R = 49).  Blocks are
// half the height of the other row passes' (the loop keeps its twiddles in
// registers).  The loop is uniform over the block, so the FFT's
// synchronisation is too; rows past H are computed on row 0's values and not
// stored.  NT_: the pair planes of the chunk exceed the 256 MiB Infinity
// Cache and are read and written with the non-temporal hint (fused denoise
// of 32 x 512^2 1.81 -> 1.75 ms, 192^3 video inpainting 3% faster; a single
// 512^2 image, whose planes stay in that cache, 2% slower with the hint).
template <int N>
struct PTile {
  static constexpr int NT = Tile<N>::NT, E = Tile<N>::E;
  static constexpr int M = Tile<N>::M / 2 > 0 ? Tile<N>::M / 2 : 1;
  static constexpr int THREADS = M * NT;
};

template <int N, bool NT_>
__global__ void __launch_bounds__(PTile<N>::THREADS)
k_rows_thr(float2 *__restrict__ T, int H, int R, int b0, int p0, int np, float inv_n,
           ThrArgs thr, const float2 *__restrict__ tw) {
  constexpr int NT = PTile<N>::NT, M = PTile<N>::M, E = PTile<N>::E;
  __shared__ float2 lds[M * row_lds_len<N>()];
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int pp = blockIdx.y, bl = blockIdx.z, b = b0 + bl;
  const int ia = 2 * (p0 + pp), ib = ia + 1;
  float da = 0.f, db = 0.f;
  {
    const float sg = thr.sigma[b];
    const int ja = thr.jof[ia];
    if (ja >= 0) da = (thr.K[ja] * sg) * thr.l2[ia];
    if (ib < R) {
      const int jb = thr.jof[ib];
      if (jb >= 0) db = (thr.K[jb] * sg) * thr.l2[ib];
    }
  }
  float2 *Tp = T + ((size_t)bl * np + pp) * (size_t)H * N;
  const int nrg = (H + M - 1) / M, G = (int)gridDim.x;
  float2 nx[E];
  auto load = [&](int rg) {
    const int row = rg * M + m;
    const float2 *src = Tp + (size_t)(row < H ? row : 0) * N;
#pragma unroll
    for (int e = 0; e < E; ++e) nx[e] = stream_load<NT_>(&src[t + e * NT]);
  };
  if ((int)blockIdx.x < nrg) load(blockIdx.x);
  for (int rg = blockIdx.x; rg < nrg; rg += G) {
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = nx[e];
    if (rg + G < nrg) load(rg + G);
    fft_line<N, true>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float a = v[e].x * inv_n, bb = ib < R ? v[e].y * inv_n : 0.f;
      if (!(fabsf(a) >= da)) a = 0.f;
      if (!(fabsf(bb) >= db)) bb = 0.f;
      v[e] = make_float2(a, bb);
    }
    fft_line<N, false>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
    const int row = rg * M + m;
    if (row < H) {
      float2 *dst = Tp + (size_t)row * N;
#pragma unroll
      for (int e = 0; e < E; ++e) stream_store<NT_>(&dst[t + e * NT], v[e]);
    }
  }
}

// Column tile of the inverse accumulation pass: MW columns per block (at
// most the generic column tile's width).  16 columns for batches; a single
// image takes 8 (512 threads, no register spills, twice the blocks): one
// 512^2 image, R = 49, 5% faster per inpainting iteration, while the
// 32-image batch is 34% slower with 8.  The one-image instance reads the
// pair planes without the non-temporal hint (they stay in the Infinity
// Cache).
constexpr int kInvWide = 16, kInvNarrow = 8;
template <int N, int MW, int EM = 1>
struct ITile {
  using PL = Plan<N, EM>;
  static constexpr int NT = PL::NT;
  static constexpr int E = PL::E;
  static constexpr int MC = EM == 1 ? CTile<N>::M : (NT * 16 <= 1024 ? 16 : 8);
  static constexpr int M = MC < MW ? MC : MW;
  static constexpr int THREADS = M * NT;
};

// Column tile and image group of an inverse-accumulation block.  A grid with
// gridDim.y > 1 is (tiles, groups) in the usual XCD-grouped tile order.  A
// grid flattened into x (groups = gridDim.x / tiles, 8 | tiles) hands the
// blocks of one tile for every image group to one XCD, consecutive in
// dispatch order, where they share the tile's filter columns in L2 (used
// for narrow planes: 32 x 512^2 accumulation 495 -> 470 us; with 128 tiles
// of 8 columns, 1024^2, it was slower).
__device__ __forceinline__ void acc_tile_group(int tiles, int &tile, int &grp) {
  if (gridDim.y > 1 || (tiles & 7) != 0) {
    tile = col_tile();
    grp = blockIdx.y;
    return;
  }
  const int L = blockIdx.x, groups = (int)gridDim.x / tiles;
  const int r = L & 7, u = L >> 3;
  grp = u % groups;
  tile = r * (tiles >> 3) + u / groups;
}

template <int N, int BT, int MW, int EM = 1>
__global__ void __launch_bounds__((ITile<N, MW, EM>::THREADS))
k_cols_fft_acc(const float2 *__restrict__ U, const float *__restrict__ filt,
               const float *__restrict__ psi, float2 *__restrict__ ACC, float2 *__restrict__ part,
               int Btot, int W, int R, int b0, int nb, int p0, int np, int first, int last,
               const float2 *__restrict__ tw) {
  constexpr int NT = ITile<N, MW, EM>::NT, M = ITile<N, MW, EM>::M, E = ITile<N, MW, EM>::E;
  using PL = typename ITile<N, MW, EM>::PL;
  __shared__ float2 lds[M * N];
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  int tile, grp;
  acc_tile_group((W + M - 1) / M, tile, grp);
  const int col = tile * M + m;
  const bool ok = col < W;
  const int cc = ok ? col : 0;
  const size_t plane = (size_t)N * W;
  // Thread (m, t) owns rows t + e NT of column cc.  Every access is a
  // wave-uniform base (plane, row step e NT) plus one 32-bit lane byte offset
  // (row t, column cc): no per-value addresses stay live across the pair loop.
  const unsigned lo = ((unsigned)t * W + cc) * 8u, lo4 = lo / 2;
  const size_t sb8 = (size_t)NT * W * 8, sb4 = sb8 / 2;
  auto at8 = [&](const float2 *base, int e) -> const float2 * {
    return (const float2 *)((const char *)base + e * sb8 + lo);
  };
  auto at4 = [&](const float *base, int e) -> const float * {
    return (const float *)((const char *)base + e * sb4 + lo4);
  };
  // pair group z sums pairs [q0, q1) of the chunk into its own partial sum:
  // ACC for z = 0, part[z - 1] ([Btot] planes each) otherwise; with several
  // groups k_cols_acc_finish adds the partial sums after the last chunk.  A
  // group with no pair in this chunk still initialises its partial sum.
  const int per = (np + (int)gridDim.z - 1) / (int)gridDim.z;
  const int q0 = (int)blockIdx.z * per, q1 = min(np, q0 + per);
  float2 *dst = blockIdx.z == 0 ? ACC : part + (size_t)(blockIdx.z - 1) * Btot * plane;
  float2 acc[BT][E];
#pragma unroll
  for (int bt = 0; bt < BT; ++bt) {
    const int bl = grp * BT + bt;
    const float2 *accp = dst + (size_t)(b0 + (bl < nb ? bl : 0)) * plane;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[bt][e] = first ? make_float2(0.f, 0.f) : *at8(accp, e);
  }
  for (int pp = q0; pp < q1; ++pp) {
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const float *fa = filt + (size_t)ia * plane;
    const float *fb = filt + (size_t)(ib < R ? ib : ia) * plane;
    float a[E], bb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = *at4(fa, e);
      bb[e] = ib < R ? *at4(fb, e) : 0.f;
    }
#pragma unroll
    for (int bt = 0; bt < BT; ++bt) {
      const int bl = grp * BT + bt;
      const float2 *Ui = U + ((size_t)(bl < nb ? bl : 0) * np + pp) * plane;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = stream_load<SL_NT_STREAM && MW != kInvNarrow>(at8(Ui, e));
      fft_line_p<PL, false>(v, t, LdsLine{lds + m, M}, tw);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        // (psi_a - i psi_b) * v
        acc[bt][e].x += a[e] * v[e].x + bb[e] * v[e].y;
        acc[bt][e].y += a[e] * v[e].y - bb[e] * v[e].x;
      }
    }
  }
#pragma unroll
  for (int bt = 0; bt < BT; ++bt) {
    const int bl = grp * BT + bt;
    if (last) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float d = *at4(psi, e);
        acc[bt][e] = make_float2(acc[bt][e].x / d, acc[bt][e].y / d);
      }
      fft_line_p<PL, true>(acc[bt], t, LdsLine{lds + m, M}, tw);
    }
    if (ok && bl < nb) {
      float2 *accp = dst + (size_t)(b0 + bl) * plane;
#pragma unroll
      for (int e = 0; e < E; ++e) *(float2 *)at8(accp, e) = acc[bt][e];
    }
  }
}

// ACC += part[0] + ... + part[G-2] over n4 groups of 4 floats (two complex
// values), summed in group order
__global__ void __launch_bounds__(256)
k_acc_sum_parts(float4 *__restrict__ ACC, const float4 *__restrict__ part, int G, size_t n4) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
    float4 v = ACC[i];
    for (int z = 1; z < G; ++z) {
      const float4 u = part[(size_t)(z - 1) * n4 + i];
      v = make_float4(v.x + u.x, v.y + u.y, v.z + u.z, v.w + u.w);
    }
    ACC[i] = v;
  }
}

// ACC[b] = column IDFT(ACC[b] / Psi_hat), in place: every thread reads its
// own column samples before the FFT.
template <int N>
__global__ void __launch_bounds__(CTile<N>::THREADS)
k_cols_acc_finish(float2 *__restrict__ ACC, const float *__restrict__ psi, int W,
                  const float2 *__restrict__ tw) {
  constexpr int NT = CTile<N>::NT, M = CTile<N>::M, E = CTile<N>::E;
  using PL = typename CTile<N>::PL;
  __shared__ float2 lds[M * N];
  const int m = threadIdx.x % M, t = threadIdx.x / M;
  const int col = col_tile() * M + m;
  const bool ok = col < W;
  const int cc = ok ? col : 0;
  const size_t plane = (size_t)N * W;
  const int b = blockIdx.y;
  float2 *accp = ACC + (size_t)b * plane + cc;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = accp[(size_t)(t + e * NT) * W];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const float d = psi[(size_t)(t + e * NT) * W + cc];
    v[e] = make_float2(v[e].x / d, v[e].y / d);
  }
  fft_line_p<PL, true>(v, t, LdsLine{lds + m, M}, tw);
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) accp[(size_t)(t + e * NT) * W] = v[e];
  }
}

template <int N>
__global__ void __launch_bounds__(Tile<N>::THREADS)
k_rows_real_ifft(const float2 *__restrict__ V, float *__restrict__ x, int H, float inv_hw,
                 const float2 *__restrict__ tw) {
  constexpr int NT = Tile<N>::NT, M = Tile<N>::M, E = Tile<N>::E;
  __shared__ float2 lds[M * row_lds_len<N>()];
  const int t = threadIdx.x % NT, m = threadIdx.x / NT;
  const int row = blockIdx.x * M + m, b = blockIdx.y;
  const bool ok = row < H;
  const size_t off = ((size_t)b * H + (ok ? row : 0)) * N;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = V[off + t + e * NT];
  fft_line<N, true>(v, t, LdsLine{lds + m * row_lds_len<N>(), 0}, tw);
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) x[off + t + e * NT] = v[e].x * inv_hw;
  }
}

// ---------------------------------------------------------------------------
// launchers: runtime length -> template instance
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Plane passes of a volume: the y and x line FFTs of one z-slice of a pair
// volume in LDS (the slice, rows padded as the row kernels pad them), so the
// slice crosses HBM once instead of once per axis.  They run the same plans
// and line FFTs as the y column pass (k_cols_fft) and the x row passes
// (k_rows_coef, k_rows_coef_fft, k_rows_thr), on the same values, so results
// are bitwise those of the separate passes.  Slices of H x W with
// H * row_lds_len(W) * 8 bytes of LDS (128 x 128: 144 KiB).
// ---------------------------------------------------------------------------
template <int H, int W>
struct PlaneTile {
  static constexpr int RL = row_lds_len<W>();
  using PC = typename CTile<H>::PL;   // the y pass's plan
  static constexpr int NTC = PC::NT, EC = PC::E;
  static constexpr int NTR = Plan<W>::NT, ER = Plan<W>::E;
  static constexpr int mn(int a, int b) { return a < b ? a : b; }
  // threads: every column (row) of a pass has its own NTC (NTR) threads
  static constexpr int THREADS = mn(1024, mn(NTC * W, NTR * H));
  static constexpr int MC = THREADS / NTC, MR = THREADS / NTR;
  static constexpr size_t LDS = (size_t)H * RL * sizeof(float2);
  static constexpr bool OK = LDS <= 150 * 1024 && THREADS % 64 == 0 && W % MC == 0 &&
                             H % MR == 0 && THREADS % NTC == 0 && THREADS % NTR == 0;
};

template <int H, int W>
__device__ __forceinline__ LdsLine plane_col(float2 *pl, int x) {
  return LdsLine{pl + x + (x >> 3), PlaneTile<H, W>::RL};
}
template <int H, int W>
__device__ __forceinline__ LdsLine plane_row(float2 *pl, int y) {
  return LdsLine{pl + y * PlaneTile<H, W>::RL, 0};
}

// y-line FFT of every column of the slice in LDS, in place
template <int H, int W, bool INV>
__device__ __forceinline__ void plane_cols(float2 *pl, const float2 *__restrict__ twH) {
  using PT = PlaneTile<H, W>;
  const int m = threadIdx.x % PT::MC, t = threadIdx.x / PT::MC;
#pragma unroll 1
  for (int c0 = 0; c0 < W; c0 += PT::MC) {
    const LdsLine col = plane_col<H, W>(pl, c0 + m);
    float2 v[PT::EC];
#pragma unroll
    for (int e = 0; e < PT::EC; ++e) v[e] = col[t + e * PT::NTC];
    fft_line_p<typename PT::PC, INV>(v, t, col, twH);
    __syncthreads();   // every read of the last exchange precedes the write-back
#pragma unroll
    for (int e = 0; e < PT::EC; ++e) col[t + e * PT::NTC] = v[e];
  }
  __syncthreads();
}

// forward: z-IDFT'd slice -> y IDFT -> x IDFT -> coefficients of the pair.
// The slice's plane fills most of a CU's LDS, so one block per CU runs and
// nothing else overlaps its phases: the block is persistent over (slice,
// pair, image) items and software-pipelined instead.  Each column iteration
// reads its columns from HBM straight into registers (no staging copy) and
// issues the loads of the next column iteration, the last one those of the
// next item, before its own transform; the row pass's stores drain while the
// next item starts.  128 x 128 x 128, R = 99: 534 -> 353 us per forward.
template <int H, int W, int DT>
__global__ void __launch_bounds__((PlaneTile<H, W>::THREADS))
k_plane_coef(const float2 *__restrict__ T, typename Store<DT>::T *__restrict__ coef,
             const float *__restrict__ scales, int D, int R, int b0, int p0, int np, int nb,
             float inv_n, const float2 *__restrict__ twH, const float2 *__restrict__ twW) {
  using PT = PlaneTile<H, W>;
  constexpr int NCI = W / PT::MC;      // column iterations per slice
  __shared__ float2 pl[H * PT::RL];
  const int items = D * np * nb;
  const size_t slice = (size_t)H * W, vol = slice * D;
  const int mc = threadIdx.x % PT::MC, tc = threadIdx.x / PT::MC;
  // column (ci, mc) of item i, values y = tc + e NTC: wave-uniform bases,
  // one 32-bit lane offset
  const unsigned lo = (unsigned)(tc * W + mc) * (unsigned)sizeof(float2);
  auto fetch = [&](float2 (&v)[PT::EC], int i, int ci) {
    const int z = i % D, pp = (i / D) % np, bl = i / (D * np);
    const char *Tb = (const char *)(T + ((size_t)bl * np + pp) * vol + (size_t)z * slice + ci * PT::MC);
#pragma unroll
    for (int e = 0; e < PT::EC; ++e)
      v[e] = *(const float2 *)(Tb + (size_t)e * PT::NTC * W * sizeof(float2) + lo);
  };
  float2 cur[PT::EC], nxt[PT::EC];
  int i = blockIdx.x;
  if (i < items) fetch(cur, i, 0);
  for (; i < items; i += gridDim.x) {
    const int z = i % D, pp = (i / D) % np, bl = i / (D * np), b = b0 + bl;
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    __syncthreads();   // the previous slice's row pass has left LDS
#pragma unroll 1
    for (int ci = 0; ci < NCI; ++ci) {
      const bool last = ci + 1 == NCI;
      const int ni = last ? i + (int)gridDim.x : i;
      if (ni < items) fetch(nxt, ni, last ? 0 : ci + 1);
      const LdsLine col = plane_col<H, W>(pl, ci * PT::MC + mc);
      fft_line_p<typename PT::PC, true>(cur, tc, col, twH);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < PT::EC; ++e) col[tc + e * PT::NTC] = cur[e];
#pragma unroll
      for (int e = 0; e < PT::EC; ++e) cur[e] = nxt[e];
    }
    __syncthreads();
    float sa = inv_n, sb = inv_n;
    if (DT != 0) {
      sa = inv_n / scales[(size_t)b * R + ia];
      if (ib < R) sb = inv_n / scales[(size_t)b * R + ib];
    }
    using Raw = typename Store<DT>::Raw;
    Raw *ca = (Raw *)(coef + ((size_t)b * R + ia) * vol + (size_t)z * slice);
    Raw *cb = (Raw *)(coef + ((size_t)b * R + (ib < R ? ib : ia)) * vol + (size_t)z * slice);
    const int t = threadIdx.x % PT::NTR, m = threadIdx.x / PT::NTR;
#pragma unroll 1
    for (int r0 = 0; r0 < H; r0 += PT::MR) {
      const int y = r0 + m;
      float2 v[PT::ER];
      const LdsLine row = plane_row<H, W>(pl, y);
#pragma unroll
      for (int e = 0; e < PT::ER; ++e) v[e] = row[t + e * PT::NTR];
      fft_line<W, true>(v, t, row, twW);
#pragma unroll
      for (int e = 0; e < PT::ER; ++e)
        coef_store(ca + (size_t)y * W + t + e * PT::NTR, Store<DT>::enc_raw(v[e].x * sa));
      if (ib < R) {
#pragma unroll
        for (int e = 0; e < PT::ER; ++e)
          coef_store(cb + (size_t)y * W + t + e * PT::NTR, Store<DT>::enc_raw(v[e].y * sb));
      }
    }
  }
}

// inverse: coefficients of the pair (decoded, thresholded) -> x DFT -> y DFT
// -> U slice for the z pass.  Persistent and pipelined like the forward: each
// row iteration issues the coefficient loads of the next one (the last, of
// the next item) before its transform, and the column pass stores U straight
// from registers.  128 x 128 x 128, R = 99: 479 -> 354 us per inverse.
template <int H, int W, int DT>
__global__ void __launch_bounds__((PlaneTile<H, W>::THREADS))
k_plane_coef_fft(const typename Store<DT>::T *__restrict__ coef, const float *__restrict__ scales,
                 float2 *__restrict__ U, int D, int R, int b0, int p0, int np, int nb, ThrArgs thr,
                 const float2 *__restrict__ twH, const float2 *__restrict__ twW) {
  using PT = PlaneTile<H, W>;
  constexpr int NRI = H / PT::MR, NCI = W / PT::MC;
  using Raw = typename Store<DT>::Raw;
  __shared__ float2 pl[H * PT::RL];
  const int items = D * np * nb;
  const size_t slice = (size_t)H * W, vol = slice * D;
  const int t = threadIdx.x % PT::NTR, m = threadIdx.x / PT::NTR;
  // raw coefficients of row iteration ri of item i (both subbands of the pair)
  auto fetch = [&](Raw (&ra)[PT::ER], Raw (&rb)[PT::ER], int i, int ri) {
    const int z = i % D, pp = (i / D) % np, bl = i / (D * np), b = b0 + bl;
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const size_t o = (size_t)z * slice + (size_t)(ri * PT::MR + m) * W + t;
    const Raw *ca = (const Raw *)(coef + ((size_t)b * R + ia) * vol + o);
    const Raw *cb = (const Raw *)(coef + ((size_t)b * R + (ib < R ? ib : ia)) * vol + o);
#pragma unroll
    for (int e = 0; e < PT::ER; ++e) {
      ra[e] = coef_load(ca + e * PT::NTR);
      rb[e] = coef_load(cb + e * PT::NTR);   // ignored without a partner
    }
  };
  Raw ca_[PT::ER], cb_[PT::ER], na[PT::ER], nb_[PT::ER];
  int i = blockIdx.x;
  if (i < items) fetch(ca_, cb_, i, 0);
  const int mc = threadIdx.x % PT::MC, tc = threadIdx.x / PT::MC;
  for (; i < items; i += gridDim.x) {
    const int z = i % D, pp = (i / D) % np, bl = i / (D * np), b = b0 + bl;
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const bool has_b = ib < R;
    float sa = 1.f, sb = 1.f;
    if (DT != 0) {
      sa = scales[(size_t)b * R + ia];
      if (has_b) sb = scales[(size_t)b * R + ib];
    }
    float da = 0.f, db = 0.f;
    if (thr.sigma) {
      const float sg = thr.sigma[b];
      const int ja = thr.jof[ia];
      if (ja >= 0) da = (thr.K[ja] * sg) * thr.l2[ia];
      if (has_b) {
        const int jb = thr.jof[ib];
        if (jb >= 0) db = (thr.K[jb] * sg) * thr.l2[ib];
      }
    }
    __syncthreads();   // the previous slice's column pass has left LDS
#pragma unroll
    for (int ri = 0; ri < NRI; ++ri) {
      const bool last = ri + 1 == NRI;
      const int ni = last ? i + (int)gridDim.x : i;
      if (ni < items) fetch(na, nb_, ni, last ? 0 : ri + 1);
      float2 v[PT::ER];
#pragma unroll
      for (int e = 0; e < PT::ER; ++e) {
        float a = Store<DT>::dec_raw(ca_[e]) * sa;
        float bb = has_b ? Store<DT>::dec_raw(cb_[e]) * sb : 0.f;
        if (!(fabsf(a) >= da)) a = 0.f;
        if (!(fabsf(bb) >= db)) bb = 0.f;
        v[e] = make_float2(a, bb);
      }
      const LdsLine row = plane_row<H, W>(pl, ri * PT::MR + m);
      fft_line<W, false>(v, t, row, twW);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < PT::ER; ++e) row[t + e * PT::NTR] = v[e];
#pragma unroll
      for (int e = 0; e < PT::ER; ++e) {
        ca_[e] = na[e];
        cb_[e] = nb_[e];
      }
    }
    __syncthreads();
    // y DFT of every column, stored to U straight from registers
    float2 *Us = U + ((size_t)bl * np + pp) * vol + (size_t)z * slice;
#pragma unroll 1
    for (int ci = 0; ci < NCI; ++ci) {
      const int x = ci * PT::MC + mc;
      const LdsLine col = plane_col<H, W>(pl, x);
      float2 v[PT::EC];
#pragma unroll
      for (int e = 0; e < PT::EC; ++e) v[e] = col[tc + e * PT::NTC];
      fft_line_p<typename PT::PC, false>(v, tc, col, twH);
#pragma unroll
      for (int e = 0; e < PT::EC; ++e) Us[(size_t)(tc + e * PT::NTC) * W + x] = v[e];
    }
  }
}

// fused denoise: y IDFT, x IDFT, scale, hard threshold, x DFT, y DFT of one
// slice, in place
template <int H, int W>
__global__ void __launch_bounds__((PlaneTile<H, W>::THREADS))
k_plane_thr(float2 *__restrict__ T, int D, int R, int b0, int p0, int np, float inv_n,
            ThrArgs thr, const float2 *__restrict__ twH, const float2 *__restrict__ twW) {
  using PT = PlaneTile<H, W>;
  __shared__ float2 pl[H * PT::RL];
  const int z = blockIdx.x, pp = blockIdx.y, bl = blockIdx.z, b = b0 + bl;
  const int ia = 2 * (p0 + pp), ib = ia + 1;
  float da = 0.f, db = 0.f;
  {
    const float sg = thr.sigma[b];
    const int ja = thr.jof[ia];
    if (ja >= 0) da = (thr.K[ja] * sg) * thr.l2[ia];
    if (ib < R) {
      const int jb = thr.jof[ib];
      if (jb >= 0) db = (thr.K[jb] * sg) * thr.l2[ib];
    }
  }
  const size_t slice = (size_t)H * W, vol = slice * D;
  float2 *Ts = T + ((size_t)bl * np + pp) * vol + (size_t)z * slice;
  for (int k = threadIdx.x; k < H * W; k += PT::THREADS) {
    const int y = k / W, x = k % W;
    pl[y * PT::RL + x + (x >> 3)] = Ts[k];
  }
  __syncthreads();
  plane_cols<H, W, true>(pl, twH);
  const int t = threadIdx.x % PT::NTR, m = threadIdx.x / PT::NTR;
#pragma unroll 1
  for (int r0 = 0; r0 < H; r0 += PT::MR) {
    const int y = r0 + m;
    const LdsLine row = plane_row<H, W>(pl, y);
    float2 v[PT::ER];
#pragma unroll
    for (int e = 0; e < PT::ER; ++e) v[e] = row[t + e * PT::NTR];
    fft_line<W, true>(v, t, row, twW);
#pragma unroll
    for (int e = 0; e < PT::ER; ++e) {
      float a = v[e].x * inv_n, bb = ib < R ? v[e].y * inv_n : 0.f;
      if (!(fabsf(a) >= da)) a = 0.f;
      if (!(fabsf(bb) >= db)) bb = 0.f;
      v[e] = make_float2(a, bb);
    }
    fft_line<W, false>(v, t, row, twW);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PT::ER; ++e) row[t + e * PT::NTR] = v[e];
  }
  __syncthreads();
  plane_cols<H, W, false>(pl, twH);
  for (int k = threadIdx.x; k < H * W; k += PT::THREADS) {
    const int y = k / W, x = k % W;
    Ts[k] = pl[y * PT::RL + x + (x >> 3)];
  }
}

// ---------------------------------------------------------------------------
// Half-plane passes of a volume: z-slices too large for one CU's LDS (192 x
// 192: 288 KiB) are split in y by one decimation-in-frequency step.  With
// Hh = H / 2 and w = exp(-2 pi i / H), the y transform of a column t is
//   Y[2k + h] = DFT_Hh( (t[m] + (-1)^h t[m + Hh]) w^(+-m h) )[k],   m < Hh,
// (the sign of the twiddle follows the direction of the transform), so half h
// of the slice needs Hh combined rows (Hh x W complex in LDS, rows padded one
// element per 16) and yields every second output row, whole and contiguous.
// Both halves read the full slice; the grid gives the two halves of a slice
// workgroup ids 8 apart, which the dispatcher sends to the same XCD at about
// the same time, so the second read finds the slice in that XCD's L2.
// Forward: z-IDFT'd slice -> combine -> y IDFT (Hh) -> x IDFT -> coefficient
// rows 2k + h.  Inverse: coefficient rows m and m + Hh (decoded, thresholded)
// -> combine -> x DFT -> twiddle -> y DFT (Hh) -> U rows 2k + h.
// ---------------------------------------------------------------------------
template <int H, int W>
struct HalfTile {
  static constexpr int HH = H / 2;
  static constexpr int RL = W + W / 16;
  using PC = Plan<HH>;                        // the y pass's plan (half length)
  static constexpr int NTC = PC::NT, EC = PC::E;
  static constexpr int NTR = Plan<W>::NT, ER = Plan<W>::E;
  static constexpr bool fits(int th) {
    return th % 64 == 0 && th % NTC == 0 && th % NTR == 0 && W % (th / NTC) == 0 &&
           HH % (th / NTR) == 0;
  }
  // at most 512 threads: the pipelined passes hold two iterations' raw rows
  // (m and m + Hh) in registers, which needs the 256 VGPRs of 2 waves per SIMD
  static constexpr int pick() {
    for (int th = 512; th >= 64; th -= 64)
      if (fits(th)) return th;
    return 0;
  }
  static constexpr int THREADS = pick();
  static constexpr int MC = THREADS ? THREADS / NTC : 1, MR = THREADS ? THREADS / NTR : 1;
  static constexpr size_t LDS = (size_t)HH * RL * sizeof(float2);
  static constexpr bool OK = H % 2 == 0 && THREADS > 0 && LDS <= 156 * 1024 && W % 16 == 0;
};

// Item i of a half-plane pass -> (slice, half h); a slice indexes (z, pair,
// image).  The grid is persistent (G workgroups, G a multiple of 16);
// workgroup g takes items g, g + G, ...  Workgroups g and g + 8 sit on the
// same XCD (round-robin dispatch), so in every full round the map gives them
// the two halves of one slice: both read that slice at about the same time
// and the second read comes from the XCD's L2.  A last, partial round (an
// even number of items) pairs neighbouring workgroups instead.
__device__ __forceinline__ void half_item(int i, int G, int items, int &slice, int &h) {
  const int r = i / G, g = i % G;           // round, workgroup
  if ((r + 1) * G <= items) {
    h = (g >> 3) & 1;
    slice = r * (G >> 1) + (g >> 4) * 8 + (g & 7);
  } else {
    h = g & 1;
    slice = r * (G >> 1) + (g >> 1);
  }
}

// Forward.  Persistent and software-pipelined like the plane passes: column
// iteration ci holds the combined (DIF) values of its columns in registers,
// the raw rows m and m + Hh of the next column iteration (or of the next
// item) are loaded before the transform.
template <int H, int W, int DT>
__global__ void __launch_bounds__((HalfTile<H, W>::THREADS))
k_hplane_coef(const float2 *__restrict__ T, typename Store<DT>::T *__restrict__ coef,
              const float *__restrict__ scales, int D, int R, int b0, int p0, int np, int nb,
              float inv_n, const float2 *__restrict__ twH, const float2 *__restrict__ twW) {
  using HT = HalfTile<H, W>;
  constexpr int HH = HT::HH, NCI = W / HT::MC;
  __shared__ float2 pl[HH * HT::RL];
  __shared__ float2 twd[HH];   // DIF twiddles w^m (the loop-top barrier orders them)
  for (int k = threadIdx.x; k < HH; k += HT::THREADS) twd[k] = twH[k];
  const int G = gridDim.x;
  const int nslice = D * np * nb, items = 2 * nslice;
  const size_t slice = (size_t)H * W, vol = slice * D;
  const int mc = threadIdx.x % HT::MC, tc = threadIdx.x / HT::MC;
  const unsigned lo = (unsigned)(tc * W + mc) * (unsigned)sizeof(float2);
  // raw rows m = tc + e NTC and m + Hh of column ci of item i
  auto fetch = [&](float2 (&ra)[HT::EC], float2 (&rc)[HT::EC], int i, int ci) {
    int sl, h;
    half_item(i, G, items, sl, h);
    const int z = sl % D, pp = (sl / D) % np, bl = sl / (D * np);
    const char *Tb =
        (const char *)(T + ((size_t)bl * np + pp) * vol + (size_t)z * slice + ci * HT::MC);
#pragma unroll
    for (int e = 0; e < HT::EC; ++e) {
      ra[e] = *(const float2 *)(Tb + (size_t)e * HT::NTC * W * sizeof(float2) + lo);
      rc[e] = *(const float2 *)(Tb + ((size_t)e * HT::NTC + HH) * W * sizeof(float2) + lo);
    }
  };
  float2 ca_[HT::EC], cc_[HT::EC], na[HT::EC], nc[HT::EC];
  int i = blockIdx.x;
  if (i < items) fetch(ca_, cc_, i, 0);
  for (; i < items; i += G) {
    int sl, h;
    half_item(i, G, items, sl, h);
    const int z = sl % D, pp = (sl / D) % np, bl = sl / (D * np), b = b0 + bl;
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    __syncthreads();   // the previous item's row pass has left LDS
#pragma unroll 1
    for (int ci = 0; ci < NCI; ++ci) {
      const bool last = ci + 1 == NCI;
      const int ni = last ? i + G : i;
      if (ni < items) fetch(na, nc, ni, last ? 0 : ci + 1);
      float2 v[HT::EC];
#pragma unroll
      for (int e = 0; e < HT::EC; ++e)
        v[e] = h ? cmulconj(csub(ca_[e], cc_[e]), twd[tc + e * HT::NTC]) : cadd(ca_[e], cc_[e]);
      const int x = ci * HT::MC + mc;
      const LdsLine col{pl + x + (x >> 4), HT::RL};
      fft_line_p<typename HT::PC, true>(v, tc, col, TwStep<2>{twH});
      __syncthreads();
#pragma unroll
      for (int e = 0; e < HT::EC; ++e) col[tc + e * HT::NTC] = v[e];
#pragma unroll
      for (int e = 0; e < HT::EC; ++e) {
        ca_[e] = na[e];
        cc_[e] = nc[e];
      }
    }
    __syncthreads();
    float sa = inv_n, sb = inv_n;
    if (DT != 0) {
      sa = inv_n / scales[(size_t)b * R + ia];
      if (ib < R) sb = inv_n / scales[(size_t)b * R + ib];
    }
    using Raw = typename Store<DT>::Raw;
    Raw *ca = (Raw *)(coef + ((size_t)b * R + ia) * vol + (size_t)z * slice);
    Raw *cb = (Raw *)(coef + ((size_t)b * R + (ib < R ? ib : ia)) * vol + (size_t)z * slice);
    const int t = threadIdx.x % HT::NTR, m = threadIdx.x / HT::NTR;
#pragma unroll 1
    for (int r0 = 0; r0 < HH; r0 += HT::MR) {
      const int r = r0 + m, y = 2 * r + h;
      float2 v[HT::ER];
      const LdsLine row{pl + r * HT::RL, -1};
#pragma unroll
      for (int e = 0; e < HT::ER; ++e) v[e] = row[t + e * HT::NTR];
      fft_line<W, true>(v, t, row, twW);
#pragma unroll
      for (int e = 0; e < HT::ER; ++e)
        coef_store(ca + (size_t)y * W + t + e * HT::NTR, Store<DT>::enc_raw(v[e].x * sa));
      if (ib < R) {
#pragma unroll
        for (int e = 0; e < HT::ER; ++e)
          coef_store(cb + (size_t)y * W + t + e * HT::NTR, Store<DT>::enc_raw(v[e].y * sb));
      }
    }
  }
}

// Inverse, pipelined over row iterations; U rows 2k + h leave straight from
// the column transform's registers.
template <int H, int W, int DT>
__global__ void __launch_bounds__((HalfTile<H, W>::THREADS))
k_hplane_coef_fft(const typename Store<DT>::T *__restrict__ coef, const float *__restrict__ scales,
                  float2 *__restrict__ U, int D, int R, int b0, int p0, int np, int nb,
                  ThrArgs thr, const float2 *__restrict__ twH, const float2 *__restrict__ twW) {
  using HT = HalfTile<H, W>;
  constexpr int HH = HT::HH, NRI = HH / HT::MR, NCI = W / HT::MC;
  using Raw = typename Store<DT>::Raw;
  __shared__ float2 pl[HH * HT::RL];
  const int G = gridDim.x;
  const int nslice = D * np * nb, items = 2 * nslice;
  const size_t slice = (size_t)H * W, vol = slice * D;
  const int t = threadIdx.x % HT::NTR, m = threadIdx.x / HT::NTR;
  // raw rows r and r + Hh (r = ri MR + m) of both subbands of item i
  auto fetch = [&](Raw (&q)[4][HT::ER], int i, int ri) {
    int sl, h;
    half_item(i, G, items, sl, h);
    const int z = sl % D, pp = (sl / D) % np, bl = sl / (D * np), b = b0 + bl;
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const size_t o = (size_t)z * slice + (size_t)(ri * HT::MR + m) * W + t;
    const Raw *ca = (const Raw *)(coef + ((size_t)b * R + ia) * vol + o);
    const Raw *cb = (const Raw *)(coef + ((size_t)b * R + (ib < R ? ib : ia)) * vol + o);
#pragma unroll
    for (int e = 0; e < HT::ER; ++e) {
      q[0][e] = coef_load(ca + e * HT::NTR);
      q[1][e] = coef_load(cb + e * HT::NTR);   // ignored without a partner
      q[2][e] = coef_load(ca + (size_t)HH * W + e * HT::NTR);
      q[3][e] = coef_load(cb + (size_t)HH * W + e * HT::NTR);
    }
  };
  Raw cur[4][HT::ER], nxt[4][HT::ER];
  int i = blockIdx.x;
  if (i < items) fetch(cur, i, 0);
  const int mc = threadIdx.x % HT::MC, tc = threadIdx.x / HT::MC;
  for (; i < items; i += G) {
    int sl, h;
    half_item(i, G, items, sl, h);
    const int z = sl % D, pp = (sl / D) % np, bl = sl / (D * np), b = b0 + bl;
    const int ia = 2 * (p0 + pp), ib = ia + 1;
    const bool has_b = ib < R;
    float sa = 1.f, sb = 1.f;
    if (DT != 0) {
      sa = scales[(size_t)b * R + ia];
      if (has_b) sb = scales[(size_t)b * R + ib];
    }
    float da = 0.f, db = 0.f;
    if (thr.sigma) {
      const float sg = thr.sigma[b];
      const int ja = thr.jof[ia];
      if (ja >= 0) da = (thr.K[ja] * sg) * thr.l2[ia];
      if (has_b) {
        const int jb = thr.jof[ib];
        if (jb >= 0) db = (thr.K[jb] * sg) * thr.l2[ib];
      }
    }
    auto val = [&](Raw ra, Raw rb) {
      float a = Store<DT>::dec_raw(ra) * sa;
      float bb = has_b ? Store<DT>::dec_raw(rb) * sb : 0.f;
      if (!(fabsf(a) >= da)) a = 0.f;
      if (!(fabsf(bb) >= db)) bb = 0.f;
      return make_float2(a, bb);
    };
    __syncthreads();   // the previous item's column pass has left LDS
#pragma unroll 1
    for (int ri = 0; ri < NRI; ++ri) {
      const bool last = ri + 1 == NRI;
      const int ni = last ? i + G : i;
      if (ni < items) fetch(nxt, ni, last ? 0 : ri + 1);
      const int r = ri * HT::MR + m;
      float2 v[HT::ER];
#pragma unroll
      for (int e = 0; e < HT::ER; ++e) {
        const float2 p = val(cur[0][e], cur[1][e]), q = val(cur[2][e], cur[3][e]);
        v[e] = h ? csub(p, q) : cadd(p, q);
      }
      const LdsLine row{pl + r * HT::RL, -1};
      fft_line<W, false>(v, t, row, twW);
      if (h) {
        const float2 w = twH[r];
#pragma unroll
        for (int e = 0; e < HT::ER; ++e) v[e] = cmul(v[e], w);
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < HT::ER; ++e) row[t + e * HT::NTR] = v[e];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < HT::ER; ++e) cur[k][e] = nxt[k][e];
    }
    __syncthreads();
    float2 *Us = U + ((size_t)bl * np + pp) * vol + (size_t)z * slice;
#pragma unroll 1
    for (int ci = 0; ci < NCI; ++ci) {
      const int x = ci * HT::MC + mc;
      const LdsLine col{pl + x + (x >> 4), HT::RL};
      float2 v[HT::EC];
#pragma unroll
      for (int e = 0; e < HT::EC; ++e) v[e] = col[tc + e * HT::NTC];
      fft_line_p<typename HT::PC, false>(v, tc, col, TwStep<2>{twH});
#pragma unroll
      for (int e = 0; e < HT::EC; ++e) Us[(size_t)(2 * (tc + e * HT::NTC) + h) * W + x] = v[e];
    }
  }
}

#define SL_FOR_EACH_N(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool lines_supported(int n) {
  switch (n) {
#define X(N) case N:
    SL_FOR_EACH_N(X)
#undef X
    return true;
    default:
      return false;
  }
}

template <int N>
static dim3 row_grid(int H, int y, int z = 1) {
  return dim3((H + Tile<N>::M - 1) / Tile<N>::M, y, z);
}
template <int N>
static dim3 col_grid(int W, int y) {
  return dim3((W + CTile<N>::M - 1) / CTile<N>::M, y, 1);
}

hipError_t launch_rows_real_fft_mix(const Sys2D &s, const MixArgs &mix, float2 *A, int B,
                                    hipStream_t st) {
  switch (s.W) {
#define X(N)                                                                                  \
  case N:                                                                                     \
    if (mix.first)                                                                            \
      hipLaunchKernelGGL((k_rows_real_fft<N, 1>), row_grid<N>(s.H, B), dim3(Tile<N>::THREADS), \
                         0, st, nullptr, A, nullptr, s.H, s.twW, mix, B);                     \
    else                                                                                      \
      hipLaunchKernelGGL((k_rows_real_fft<N, 2>), row_grid<N>(s.H, B), dim3(Tile<N>::THREADS), \
                         0, st, nullptr, A, nullptr, s.H, s.twW, mix, B);                     \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_real_fft(const Sys2D &s, const float *x, float2 *A, unsigned *xmax, int B,
                                hipStream_t st) {
  switch (s.W) {
#define X(N)                                                                                  \
  case N:                                                                                     \
    hipLaunchKernelGGL((k_rows_real_fft<N, 0>), row_grid<N>(s.H, B), dim3(Tile<N>::THREADS), 0, \
                       st, x, A, xmax, s.H, s.twW, MixArgs{}, 0);                             \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cols_fft(const Sys2D &s, const float2 *A, float2 *F, int B, bool inverse,
                           hipStream_t st, bool stream) {
  switch (s.H) {
#define X(N)                                                                                  \
  case N:                                                                                     \
    if (inverse && stream)                                                                    \
      hipLaunchKernelGGL((k_cols_fft<N, true, true>), col_grid<N>(s.W, B),                    \
                         dim3(CTile<N>::THREADS), 0, st, A, F, s.W, s.twH);                   \
    else if (inverse)                                                                         \
      hipLaunchKernelGGL((k_cols_fft<N, true, false>), col_grid<N>(s.W, B),                   \
                         dim3(CTile<N>::THREADS), 0, st, A, F, s.W, s.twH);                   \
    else if (stream)                                                                          \
      hipLaunchKernelGGL((k_cols_fft<N, false, true>), col_grid<N>(s.W, B),                   \
                         dim3(CTile<N>::THREADS), 0, st, A, F, s.W, s.twH);                   \
    else                                                                                      \
      hipLaunchKernelGGL((k_cols_fft<N, false, false>), col_grid<N>(s.W, B),                  \
                         dim3(CTile<N>::THREADS), 0, st, A, F, s.W, s.twH);                   \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Pair groups of a column pass whose grid (column tiles x image groups) has
// `blocks` blocks: 1 when the grid fills the compute units, otherwise about
// `per_cu` blocks per compute unit, at most `cap` groups, none of them empty.
// The forward pass splits finer (its groups only re-read the spectrum); the
// inverse pass adds one partial-sum plane per extra group.
static int pair_groups(const Sys2D &s, int blocks, int np, int per_cu, int cap) {
  const int num_cu = s.num_cu;
  if (!s.split_pairs || np <= 1 || blocks >= num_cu) return 1;
  int g = (per_cu * num_cu + blocks - 1) / blocks;
  g = g < np ? g : np;
  g = g < cap ? g : cap;
  const int per = (np + g - 1) / g;
  return (np + per - 1) / per;
}

// images per block of the inverse accumulation: the system's choice, else
// two (one for a single image, which does not fill a two-image block)
static int inv_bt(const Sys2D &s, int nb) {
  if (s.inv_images == 1 || s.inv_images == kInvBT) return s.inv_images;
  return nb >= 2 ? kInvBT : 1;
}

// columns per block of the inverse accumulation pass
template <int N>
static int inv_tile_m(const Sys2D &s, int nb) {
  if constexpr (em2_length<N>()) {
    if (s.line_em == 2) return ITile<N, kInvNarrow, 2>::M;
  }
  return nb == 1 ? ITile<N, kInvNarrow>::M : ITile<N, kInvWide>::M;
}

int inv_pair_groups(const Sys2D &s, int nb, int np) {
  if (SL_COL_V3_INV || !lines_supported(s.H)) return 1;
  int M = 0;
  switch (s.H) {
#define X(N) \
  case N:    \
    M = inv_tile_m<N>(s, nb); \
    break;
    SL_FOR_EACH_N(X)
#undef X
  }
  const int bt = inv_bt(s, nb);
  return pair_groups(s, ((s.W + M - 1) / M) * ((nb + bt - 1) / bt), np, 2, 16);
}

template <int N, int MW, int EM = 1>
static void launch_fwd3(const Sys2D &s, const float2 *F, float2 *T, Chunk c, hipStream_t st) {
  using FT = FTile<N, MW, EM>;
  // 1024-point columns run 8 per block (64-byte row segments); two images
  // per block halve the filter reads per image and double the work between
  // barriers (24 x 1024^2, R = 33: 1.71 -> 1.44 ms per forward column pass)
  constexpr int BT = (N == 1024 && MW == kFwdWide) ? 2 : kFwdBT;
  const int tiles = (s.W + FT::M - 1) / FT::M, ny = (c.nb + BT - 1) / BT;
  hipLaunchKernelGGL((k_cols_filter_ifft3<N, BT, MW, EM>),
                     dim3(tiles, ny, pair_groups(s, tiles * ny, c.np, 4, 32)), dim3(FT::THREADS),
                     0, st, F, s.filt, T, s.W, s.R, c.b0, c.nb, c.p0, c.np, s.twH);
}

hipError_t launch_cols_filter_ifft(const Sys2D &s, const float2 *F, float2 *T, Chunk c,
                                   hipStream_t st) {
  switch (s.H) {
#define X(N)                                                                                 \
  case N:                                                                                    \
    if (SL_COL_V3_FWD && c.nb == 1)                                                            \
      launch_fwd3<N, kFwdNarrow>(s, F, T, c, st);                                              \
    else if (SL_COL_V3_FWD)                                                                    \
      launch_fwd3<N, kFwdWide>(s, F, T, c, st);                                                \
    else                                                                                       \
      hipLaunchKernelGGL((k_cols_filter_ifft<N, kFwdBT>), col_grid<N>(s.W, (c.nb + kFwdBT - 1) / kFwdBT), \
                         dim3(CTile<N>::THREADS), 0, st, F, s.filt, T, s.W, s.R, c.b0, c.nb, c.p0, \
                         c.np, s.twH);                                                         \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N, int DT, int EM>
static void rows_coef_em(const Sys2D &s, const float2 *T, void *coef, const float *scales, Chunk c,
                         float inv_hw, hipStream_t st) {
  using CT = typename Store<DT>::T;
  using TL = Tile<N, EM>;
  if (DT != 0) {
    constexpr int MP = TL::M / 2 > 0 ? TL::M / 2 : 1;
    const int nrg = (s.H + MP - 1) / MP;
    int G = nrg / 8 > 1 ? nrg / 8 : 1;
    if ((long)G * c.np * c.nb < 8L * s.num_cu) G = nrg;
    hipLaunchKernelGGL((k_rows_coef_pf<N, DT, EM>), dim3(G, c.np, c.nb), dim3(MP * TL::NT), 0, st, T,
                       (CT *)coef, scales, s.H, s.R, c.b0, c.p0, c.np, inv_hw, s.twW);
  } else {
    hipLaunchKernelGGL((k_rows_coef<N, DT, EM>), dim3((s.H + TL::M - 1) / TL::M, c.np, c.nb),
                       dim3(TL::THREADS), 0, st, T, (CT *)coef, scales, s.H, s.R, c.b0, c.p0, c.np,
                       inv_hw, s.twW);
  }
}

template <int N, int DT>
static void rows_coef_n(const Sys2D &s, const float2 *T, void *coef, const float *scales, Chunk c,
                        float inv_hw, hipStream_t st) {
  if constexpr (em2_length<N>()) {
    if (s.line_em == 2) return rows_coef_em<N, DT, 2>(s, T, coef, scales, c, inv_hw, st);
  }
  rows_coef_em<N, DT, 1>(s, T, coef, scales, c, inv_hw, st);
}

template <int DT>
static hipError_t rows_coef_dt(const Sys2D &s, const float2 *T, void *coef, const float *scales,
                               Chunk c, hipStream_t st) {
  const float inv_hw = 1.0f / ((float)s.H * (float)s.W);
  switch (s.W) {
#define X(N)                                                   \
  case N:                                                      \
    rows_coef_n<N, DT>(s, T, coef, scales, c, inv_hw, st);     \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_coef(const Sys2D &s, const float2 *T, void *coef, const float *scales,
                            Chunk c, hipStream_t st) {
  if (s.dtype == 1) return rows_coef_dt<1>(s, T, coef, scales, c, st);
  if (s.dtype == 2) return rows_coef_dt<2>(s, T, coef, scales, c, st);
  return rows_coef_dt<0>(s, T, coef, scales, c, st);
}

hipError_t launch_scales(const Sys2D &s, const unsigned *xmax, float *scales, int B,
                         hipStream_t st) {
  int n = B * s.R;
  hipLaunchKernelGGL(k_scales, dim3((n + 255) / 256), dim3(256), 0, st, xmax, s.l1, scales, B, s.R);
  return hipGetLastError();
}

hipError_t launch_div_psi(float2 *F, const float *psi, size_t npix, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_div_psi, dim3((unsigned)((npix + 255) / 256), B), dim3(256), 0, st, F, psi,
                     npix);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned *p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

template <int N, int DT, int EM>
static void rows_coef_fft_em(const Sys2D &s, const void *coef, const float *scales, float2 *U,
                             Chunk c, const ThrArgs &thr, hipStream_t st) {
  using CT = typename Store<DT>::T;
  using TL = Tile<N, EM>;
  if (DT != 0) {
    constexpr int MP = TL::M / 2 > 0 ? TL::M / 2 : 1;
    const int nrg = (s.H + MP - 1) / MP;
    int G = nrg / 8 > 1 ? nrg / 8 : 1;
    if ((long)G * c.np * c.nb < 8L * s.num_cu) G = nrg;
    hipLaunchKernelGGL((k_rows_coef_fft_pf<N, DT, EM>), dim3(G, c.np, c.nb), dim3(MP * TL::NT), 0,
                       st, (const CT *)coef, scales, U, s.H, s.R, c.b0, c.p0, c.np, thr, s.twW);
  } else {
    hipLaunchKernelGGL((k_rows_coef_fft<N, DT, EM>), dim3((s.H + TL::M - 1) / TL::M, c.np, c.nb),
                       dim3(TL::THREADS), 0, st, (const CT *)coef, scales, U, s.H, s.R, c.b0, c.p0,
                       c.np, thr, s.twW);
  }
}

template <int N, int DT>
static void rows_coef_fft_n(const Sys2D &s, const void *coef, const float *scales, float2 *U,
                            Chunk c, const ThrArgs &thr, hipStream_t st) {
  if constexpr (em2_length<N>()) {
    if (s.line_em == 2) return rows_coef_fft_em<N, DT, 2>(s, coef, scales, U, c, thr, st);
  }
  rows_coef_fft_em<N, DT, 1>(s, coef, scales, U, c, thr, st);
}

template <int DT>
static hipError_t rows_coef_fft_dt(const Sys2D &s, const void *coef, const float *scales,
                                   float2 *U, Chunk c, const ThrArgs &thr, hipStream_t st) {
  switch (s.W) {
#define X(N)                                                     \
  case N:                                                        \
    rows_coef_fft_n<N, DT>(s, coef, scales, U, c, thr, st);      \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_coef_fft(const Sys2D &s, const void *coef, const float *scales, float2 *U,
                                Chunk c, const ThrArgs &thr, hipStream_t st) {
  if (s.dtype == 1) return rows_coef_fft_dt<1>(s, coef, scales, U, c, thr, st);
  if (s.dtype == 2) return rows_coef_fft_dt<2>(s, coef, scales, U, c, thr, st);
  return rows_coef_fft_dt<0>(s, coef, scales, U, c, thr, st);
}

hipError_t launch_rows_thr(const Sys2D &s, float2 *T, float inv_n, Chunk c, const ThrArgs &thr,
                           hipStream_t st) {
  const bool stream = (size_t)c.nb * c.np * s.H * s.W * sizeof(float2) > ((size_t)256 << 20);
  switch (s.W) {
#define X(N)                                                                                   \
  case N: {                                                                                    \
    /* about 8 row groups per block, unless that leaves the GPU short of blocks */             \
    const int nrg = (s.H + PTile<N>::M - 1) / PTile<N>::M;                                     \
    int G = nrg / 8 > 1 ? nrg / 8 : 1;                                                         \
    if ((long)G * c.np * c.nb < 8L * s.num_cu) G = nrg;                                        \
    if (stream)                                                                                \
      hipLaunchKernelGGL((k_rows_thr<N, true>), dim3(G, c.np, c.nb), dim3(PTile<N>::THREADS), 0, \
                         st, T, s.H, s.R, c.b0, c.p0, c.np, inv_n, thr, s.twW);                \
    else                                                                                       \
      hipLaunchKernelGGL((k_rows_thr<N, false>), dim3(G, c.np, c.nb), dim3(PTile<N>::THREADS), \
                         0, st, T, s.H, s.R, c.b0, c.p0, c.np, inv_n, thr, s.twW);             \
    break;                                                                                     \
  }
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// With the EM = 2 line plan, 1024-point columns of the inverse accumulation
// run 8 per block with 64 threads each (512 threads, 16 values per thread):
// the EM = 1 instances (8 columns x 128 threads) spill registers at the
// 128-VGPR cap of a 1024-thread block.  Two images per block when the batch
// has them (one filter read for both: 24 x 1024^2, R = 33, 1.91 -> 1.70 ms).
template <int N>
static bool cols_fft_acc_em2(const Sys2D &s, const float2 *U, float2 *ACC, float2 *part, int G,
                             int Btot, Chunk c, bool first, bool last, hipStream_t st) {
  if constexpr (em2_length<N>()) {
    if (s.line_em == 2 && !SL_COL_V3_INV) {
      using IT = ITile<N, kInvNarrow, 2>;
      if (c.nb >= 2 && inv_bt(s, c.nb) == 2)
        hipLaunchKernelGGL((k_cols_fft_acc<N, 2, kInvNarrow, 2>),
                           dim3((s.W + IT::M - 1) / IT::M, (c.nb + 1) / 2, G), dim3(IT::THREADS), 0,
                           st, U, s.filt, s.psi, ACC, part, Btot, s.W, s.R, c.b0, c.nb, c.p0,
                           c.np, (int)first, (int)(last && G == 1), s.twH);
      else
        hipLaunchKernelGGL((k_cols_fft_acc<N, 1, kInvNarrow, 2>),
                           dim3((s.W + IT::M - 1) / IT::M, c.nb, G), dim3(IT::THREADS), 0, st, U,
                           s.filt, s.psi, ACC, part, Btot, s.W, s.R, c.b0, c.nb, c.p0, c.np,
                           (int)first, (int)(last && G == 1), s.twH);
      return true;
    }
  }
  return false;
}

// grid of the batched inverse accumulation: flattened (see acc_tile_group)
// when the plane has at most 32 column tiles and a multiple of 8
static dim3 acc_grid(int W, int M, int groups, int G) {
  const int tiles = (W + M - 1) / M;
  if (groups > 1 && tiles % 8 == 0 && tiles <= 32) return dim3(tiles * groups, 1, G);
  return dim3(tiles, groups, G);
}

hipError_t launch_cols_fft_acc(const Sys2D &s, const float2 *U, float2 *ACC, float2 *part,
                               int G, int Btot, Chunk c, bool first, bool last, hipStream_t st) {
  if (G < 1 || (G > 1 && (!part || SL_COL_V3_INV))) return hipErrorInvalidValue;
  switch (s.H) {
#define X(N)                                                                                    \
  case N:                                                                                       \
    if (cols_fft_acc_em2<N>(s, U, ACC, part, G, Btot, c, first, last, st))                     \
      break;                                                                                    \
    if (SL_COL_V3_INV)                                                                          \
      hipLaunchKernelGGL((k_cols_fft_acc3<N, kInvBT>), col_grid<N>(s.W, (c.nb + kInvBT - 1) / kInvBT), \
                         dim3(CTile<N>::THREADS), 0, st, U, s.filt, s.psi, ACC, s.W, s.R, c.b0, \
                         c.nb, c.p0, c.np, (int)first, (int)last, s.twH);                      \
    else if (c.nb == 1)                                                                         \
      hipLaunchKernelGGL((k_cols_fft_acc<N, 1, kInvNarrow>),                                    \
                         dim3((s.W + ITile<N, kInvNarrow>::M - 1) / ITile<N, kInvNarrow>::M, 1, G), \
                         dim3(ITile<N, kInvNarrow>::THREADS), 0, st, U, s.filt, s.psi, ACC, part, \
                         Btot, s.W, s.R, c.b0, c.nb, c.p0, c.np, (int)first,                    \
                         (int)(last && G == 1), s.twH);                                         \
    else if (inv_bt(s, c.nb) == 1)                                                              \
      hipLaunchKernelGGL((k_cols_fft_acc<N, 1, kInvWide>),                                      \
                         dim3((s.W + ITile<N, kInvWide>::M - 1) / ITile<N, kInvWide>::M, c.nb, G), \
                         dim3(ITile<N, kInvWide>::THREADS), 0, st, U, s.filt, s.psi, ACC, part, \
                         Btot, s.W, s.R, c.b0, c.nb, c.p0, c.np, (int)first,                    \
                         (int)(last && G == 1), s.twH);                                         \
    else                                                                                        \
      hipLaunchKernelGGL((k_cols_fft_acc<N, kInvBT, kInvWide>),                                 \
                         acc_grid(s.W, ITile<N, kInvWide>::M, (c.nb + kInvBT - 1) / kInvBT, G), \
                         dim3(ITile<N, kInvWide>::THREADS), 0, st, U, s.filt, s.psi, ACC, part, \
                         Btot, s.W, s.R, c.b0, c.nb, c.p0, c.np, (int)first,                    \
                         (int)(last && G == 1), s.twH);                                         \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cols_acc_finish(const Sys2D &s, float2 *ACC, const float2 *part, int G, int B,
                                  hipStream_t st) {
  // partial sums first, at full-device parallelism (a plane holds an even
  // number of complex values: two per float4)
  const size_t n4 = (size_t)B * s.H * s.W / 2;
  const size_t want = (n4 + 255) / 256;
  hipLaunchKernelGGL(k_acc_sum_parts, dim3((unsigned)(want < 8192 ? want : 8192)), dim3(256), 0,
                     st, (float4 *)ACC, (const float4 *)part, G, n4);
  switch (s.H) {
#define X(N)                                                                                  \
  case N:                                                                                     \
    hipLaunchKernelGGL(k_cols_acc_finish<N>, col_grid<N>(s.W, B), dim3(CTile<N>::THREADS), 0, \
                       st, ACC, s.psi, s.W, s.twH);                                           \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_real_ifft(const Sys2D &s, const float2 *V, float *x, int B, hipStream_t st) {
  const float inv_hw = 1.0f / ((float)s.H * (float)s.W);
  switch (s.W) {
#define X(N)                                                                                 \
  case N:                                                                                    \
    hipLaunchKernelGGL(k_rows_real_ifft<N>, row_grid<N>(s.H, B), dim3(Tile<N>::THREADS), 0, \
                       st, V, x, s.H, inv_hw, s.twW);                                        \
    break;
    SL_FOR_EACH_N(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- plane passes of volumes ------------------------------------------------
// (H, W) slices with an LDS plane kernel; other shapes use the line passes
#define SL_FOR_EACH_PLANE(X) X(64, 64) X(96, 96) X(128, 128) X(64, 128) X(128, 64) X(96, 128) X(128, 96)

template <int H, int W>
static constexpr bool plane_ok() { return PlaneTile<H, W>::OK; }

bool plane_supported(int H, int W) {
#define X(h, w) \
  if (H == h && W == w) return plane_ok<h, w>();
  SL_FOR_EACH_PLANE(X)
#undef X
  return false;
}

template <int DT>
static hipError_t plane_coef_dt(const Sys2D &s, int D, const float2 *T, void *coef,
                                const float *scales, Chunk c, float inv_n, hipStream_t st) {
  using CT = typename Store<DT>::T;
#define X(h, w)                                                                                 \
  if constexpr (plane_ok<h, w>())                                                               \
    if (s.H == h && s.W == w) {                                                                 \
      hipLaunchKernelGGL((k_plane_coef<h, w, DT>), dim3(std::min(s.num_cu, D * c.np * c.nb)), \
                         dim3(PlaneTile<h, w>::THREADS), 0, st, T, (CT *)coef, scales, D, s.R,  \
                         c.b0, c.p0, c.np, c.nb, inv_n, s.twH, s.twW);                          \
      return hipGetLastError();                                                                 \
    }
  SL_FOR_EACH_PLANE(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_plane_coef(const Sys2D &s, int D, const float2 *T, void *coef,
                             const float *scales, Chunk c, float inv_n, hipStream_t st) {
  switch (s.dtype) {
    case 0: return plane_coef_dt<0>(s, D, T, coef, scales, c, inv_n, st);
    case 1: return plane_coef_dt<1>(s, D, T, coef, scales, c, inv_n, st);
    case 2: return plane_coef_dt<2>(s, D, T, coef, scales, c, inv_n, st);
  }
  return hipErrorInvalidValue;
}

template <int DT>
static hipError_t plane_coef_fft_dt(const Sys2D &s, int D, const void *coef, const float *scales,
                                    float2 *U, Chunk c, const ThrArgs &thr, hipStream_t st) {
  using CT = typename Store<DT>::T;
#define X(h, w)                                                                                 \
  if constexpr (plane_ok<h, w>())                                                               \
    if (s.H == h && s.W == w) {                                                                 \
      hipLaunchKernelGGL((k_plane_coef_fft<h, w, DT>), dim3(std::min(s.num_cu, D * c.np * c.nb)), \
                         dim3(PlaneTile<h, w>::THREADS), 0, st, (const CT *)coef, scales, U, D, \
                         s.R, c.b0, c.p0, c.np, c.nb, thr, s.twH, s.twW);                       \
      return hipGetLastError();                                                                 \
    }
  SL_FOR_EACH_PLANE(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_plane_coef_fft(const Sys2D &s, int D, const void *coef, const float *scales,
                                 float2 *U, Chunk c, const ThrArgs &thr, hipStream_t st) {
  switch (s.dtype) {
    case 0: return plane_coef_fft_dt<0>(s, D, coef, scales, U, c, thr, st);
    case 1: return plane_coef_fft_dt<1>(s, D, coef, scales, U, c, thr, st);
    case 2: return plane_coef_fft_dt<2>(s, D, coef, scales, U, c, thr, st);
  }
  return hipErrorInvalidValue;
}

#define SL_FOR_EACH_HALF_PLANE(X) X(192, 192) X(192, 128) X(128, 192)

template <int H, int W>
static constexpr bool half_ok() { return HalfTile<H, W>::OK; }

// persistent grid of the half-plane passes: one workgroup per CU (their LDS
// allows no more), rounded down to whole rounds of 16 and at most the number
// of slices' halves; every round covers G / 2 whole slices
static int half_grid(const Sys2D &s, int D, Chunk c) {
  const int halves = 2 * D * c.np * c.nb;
  int G = std::max(16, s.num_cu / 16 * 16);
  while (G > 16 && G > halves) G -= 16;
  return G;
}

bool half_plane_supported(int H, int W) {
#define X(h, w) \
  if (H == h && W == w) return half_ok<h, w>();
  SL_FOR_EACH_HALF_PLANE(X)
#undef X
  return false;
}

template <int DT>
static hipError_t hplane_coef_dt(const Sys2D &s, int D, const float2 *T, void *coef,
                                 const float *scales, Chunk c, float inv_n, hipStream_t st) {
  using CT = typename Store<DT>::T;
#define X(h, w)                                                                                 \
  if constexpr (half_ok<h, w>())                                                                \
    if (s.H == h && s.W == w) {                                                                 \
      hipLaunchKernelGGL((k_hplane_coef<h, w, DT>), dim3(half_grid(s, D, c)),                  \
                         dim3(HalfTile<h, w>::THREADS), 0, st, T, (CT *)coef, scales, D, s.R,   \
                         c.b0, c.p0, c.np, c.nb, inv_n, s.twH, s.twW);                          \
      return hipGetLastError();                                                                 \
    }
  SL_FOR_EACH_HALF_PLANE(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_hplane_coef(const Sys2D &s, int D, const float2 *T, void *coef,
                              const float *scales, Chunk c, float inv_n, hipStream_t st) {
  switch (s.dtype) {
    case 0: return hplane_coef_dt<0>(s, D, T, coef, scales, c, inv_n, st);
    case 1: return hplane_coef_dt<1>(s, D, T, coef, scales, c, inv_n, st);
    case 2: return hplane_coef_dt<2>(s, D, T, coef, scales, c, inv_n, st);
  }
  return hipErrorInvalidValue;
}

template <int DT>
static hipError_t hplane_coef_fft_dt(const Sys2D &s, int D, const void *coef,
                                     const float *scales, float2 *U, Chunk c, const ThrArgs &thr,
                                     hipStream_t st) {
  using CT = typename Store<DT>::T;
#define X(h, w)                                                                                 \
  if constexpr (half_ok<h, w>())                                                                \
    if (s.H == h && s.W == w) {                                                                 \
      hipLaunchKernelGGL((k_hplane_coef_fft<h, w, DT>), dim3(half_grid(s, D, c)),              \
                         dim3(HalfTile<h, w>::THREADS), 0, st, (const CT *)coef, scales, U, D,  \
                         s.R, c.b0, c.p0, c.np, c.nb, thr, s.twH, s.twW);                       \
      return hipGetLastError();                                                                 \
    }
  SL_FOR_EACH_HALF_PLANE(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_hplane_coef_fft(const Sys2D &s, int D, const void *coef, const float *scales,
                                  float2 *U, Chunk c, const ThrArgs &thr, hipStream_t st) {
  switch (s.dtype) {
    case 0: return hplane_coef_fft_dt<0>(s, D, coef, scales, U, c, thr, st);
    case 1: return hplane_coef_fft_dt<1>(s, D, coef, scales, U, c, thr, st);
    case 2: return hplane_coef_fft_dt<2>(s, D, coef, scales, U, c, thr, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_plane_thr(const Sys2D &s, int D, float2 *T, float inv_n, Chunk c,
                            const ThrArgs &thr, hipStream_t st) {
#define X(h, w)                                                                                 \
  if constexpr (plane_ok<h, w>())                                                               \
    if (s.H == h && s.W == w) {                                                                 \
      hipLaunchKernelGGL((k_plane_thr<h, w>), dim3(D, c.np, c.nb),                      \
                         dim3(PlaneTile<h, w>::THREADS), 0, st, T, D, s.R, c.b0, c.p0, c.np,    \
                         inv_n, thr, s.twH, s.twW);                                             \
      return hipGetLastError();                                                                 \
    }
  SL_FOR_EACH_PLANE(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace sl

