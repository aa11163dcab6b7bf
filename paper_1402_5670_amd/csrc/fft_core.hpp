// Stockham FFT building blocks for CDNA4 (gfx950), FP32 arithmetic with
// twiddles tabulated on the host in FP64 and rounded to FP32.
//
// A length-N line is processed by NT threads, each owning E = N / NT
// complex values.  On entry and on exit thread t holds the element at line
// position t + e * NT in register v[e] (e = 0..E-1), so a pointwise operation
// between a forward and an inverse transform needs no data movement.  The
// first radix stage reads directly from registers, the last stage writes
// directly to registers; stages in between exchange through LDS.
//
// Stockham stage of radix r after a sub-transform length p (product of the
// earlier radices), for butterfly i in [0, N/r):
//     k = i mod p,   x_q = in[i + q N/r] * W_N^{q k N/(p r)},
//     y = DFT_r(x),  out[(i - k) r + k + q p] = y_q,
// with W_N = exp(-2 pi i / N) (conjugated for the inverse transform).
#pragma once

#include <hip/hip_runtime.h>

namespace sl {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward direction) or +i (inverse direction)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2 *x) {
  float2 a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2 *x) {
  const float s3 = 0.86602540378443864676f;   // sqrt(3)/2
  float2 s = cadd(x[1], x[2]);
  float2 d = csub(x[1], x[2]);
  float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
  float2 rd = rot90<INV>(d);                   // -i d (forward)
  x[0] = cadd(x[0], s);
  x[1] = make_float2(m.x + s3 * rd.x, m.y + s3 * rd.y);
  x[2] = make_float2(m.x - s3 * rd.x, m.y - s3 * rd.y);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 *x) {
  float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
  float2 t2 = cadd(x[1], x[3]), t3 = rot90<INV>(csub(x[1], x[3]));
  x[0] = cadd(t0, t2);
  x[2] = csub(t0, t2);
  x[1] = cadd(t1, t3);
  x[3] = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2 *x) {
  const float r = 0.70710678118654752440f;
  float2 b0 = cadd(x[0], x[4]), b4 = csub(x[0], x[4]);
  float2 b1 = cadd(x[1], x[5]), b5 = csub(x[1], x[5]);
  float2 b2 = cadd(x[2], x[6]), b6 = csub(x[2], x[6]);
  float2 b3 = cadd(x[3], x[7]), b7 = csub(x[3], x[7]);
  // odd half twiddles W8^1, W8^2, W8^3 (conjugated for the inverse)
  if (INV) {
    b5 = make_float2(r * (b5.x - b5.y), r * (b5.x + b5.y));
    b7 = make_float2(-r * (b7.x + b7.y), r * (b7.x - b7.y));
  } else {
    b5 = make_float2(r * (b5.x + b5.y), r * (b5.y - b5.x));
    b7 = make_float2(r * (b7.y - b7.x), -r * (b7.x + b7.y));
  }
  b6 = rot90<INV>(b6);
  float2 e[4] = {b0, b1, b2, b3};
  float2 o[4] = {b4, b5, b6, b7};
  dft4<INV>(e);
  dft4<INV>(o);
  x[0] = e[0]; x[2] = e[1]; x[4] = e[2]; x[6] = e[3];
  x[1] = o[0]; x[3] = o[1]; x[5] = o[2]; x[7] = o[3];
}

template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2 *x) {
  if constexpr (R == 2) dft2<INV>(x);
  else if constexpr (R == 3) dft3<INV>(x);
  else if constexpr (R == 4) dft4<INV>(x);
  else dft8<INV>(x);
}

// ---------------------------------------------------------------------------
// compile-time radix plans.  Powers of two: 8s first, then a 4 or a 2.
// Lengths with a factor 3: 4s first, then a 2, then 3s, so that a thread holds
// lcm(4, 3) = 12 values (radix-8 stages would make it lcm(8, 3) = 24 and
// double the registers per thread).
// ---------------------------------------------------------------------------
template <int N_, int EMUL = 1>
struct Plan {
  static constexpr int N = N_;
  static constexpr int count3() { int n = N, c = 0; while (n % 3 == 0) { n /= 3; ++c; } return c; }
  static constexpr int pow2() { int n = N; while (n % 3 == 0) n /= 3; return n; }
  static constexpr int log2p() { int n = pow2(), c = 0; while (n > 1) { n /= 2; ++c; } return c; }
  static constexpr int n3 = count3();
  static constexpr int hi = n3 ? 4 : 8;                          // leading radix
  static constexpr int nhi = n3 ? log2p() / 2 : log2p() / 3;     // its stage count
  static constexpr int rem2 = n3 ? log2p() % 2 : log2p() % 3;    // 0, 1 (radix 2) or 2 (radix 4)
  static constexpr int S = nhi + (rem2 ? 1 : 0) + n3;
  static constexpr int radix(int s) {
    return s < nhi ? hi : (rem2 && s == nhi) ? (rem2 == 1 ? 2 : 4) : 3;
  }
  static constexpr int lcm_radix() {
    int l = 1;
    for (int s = 0; s < S; ++s) {
      int r = radix(s);
      int a = l, b = r;
      while (b) { int t = a % b; a = b; b = t; }
      l = l / a * r;
    }
    return l;
  }
  static constexpr int E = lcm_radix() * EMUL;   // values per thread
  static constexpr int NT = N / E;          // threads per line
  static constexpr int pbefore(int s) { int p = 1; for (int q = 0; q < s; ++q) p *= radix(q); return p; }
  static_assert(pow2() * (N / pow2()) == N, "bad size");
};

// LDS addressing of one line.  Column tiles interleave M lines (element n of
// line m at base[n * M + m], stride_n = M), which keeps the 64 lanes of a
// wave on consecutive words.  Row tiles store a line contiguously with one
// pad element after every 8 (stride_n = 0 selects that layout): without it
// the radix-8 stage writes at stride 8 elements and 16 lanes share a bank.
// stride_n = -1 pads one element after every 16 (planes that would not fit
// LDS with the denser padding).  Every caller passes a constant stride_n.
struct LdsLine {
  float2 *base;
  int stride_n;
  __device__ __forceinline__ float2 &operator[](int n) const {
    if (stride_n > 0) return base[n * stride_n];
    if (stride_n == 0) return base[n + (n >> 3)];
    return base[n + (n >> 4)];
  }
};
// LDS elements of one padded row line of length N
template <int N>
constexpr int row_lds_len() { return N + N / 8; }

// Exchanges between radix stages need every thread of a line to have written
// its values before any thread reads.  When all threads of a line sit in one
// wavefront (row tiles with NT dividing 64), the wavefront's LDS operations
// execute in issue order and a code-motion fence suffices: waves of a block
// then run their lines independently.  Otherwise the block synchronises.
template <bool WAVE>
__device__ __forceinline__ void line_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Lines of NT threads lie inside one wavefront when NT divides 64.
template <int NT>
constexpr bool wave_lines() { return NT <= 64 && 64 % NT == 0; }

// Twiddle tables: a global table (read through the scalar-uniform pointer) or
// a copy staged in LDS by the calling kernel (TwLds), whose reads are not
// hoisted out of a caller's loop into registers.
struct TwLds {
  const float2 *p;
};
// Every S-th entry of a longer table: the twiddles of length N / S from
// those of length N.
template <int S>
struct TwStep {
  const float2 *p;
};
__device__ __forceinline__ float2 tw_at(const float2 *__restrict__ tw, int i) { return tw[i]; }
__device__ __forceinline__ float2 tw_at(TwLds tw, int i) { return tw.p[i]; }
template <int S>
__device__ __forceinline__ float2 tw_at(TwStep<S> tw, int i) { return tw.p[i * S]; }

template <class PL, int S_, bool INV, bool WAVE = false, class TW = const float2 *>
__device__ __forceinline__ void fft_stage(float2 (&v)[PL::E], int t, const LdsLine &lds, TW tw) {
  constexpr int N = PL::N;
  constexpr int E = PL::E, NT = PL::NT;
  constexpr int r = PL::radix(S_);
  constexpr int p = PL::pbefore(S_);
  constexpr int NB = E / r;          // butterflies per thread
  constexpr int stride = N / r;
  float2 x[NB][r];
  if constexpr (S_ == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int q = 0; q < r; ++q) x[b][q] = v[b + q * NB];
  } else {
    line_sync<WAVE>();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      int i = t + b * NT;
#pragma unroll
      for (int q = 0; q < r; ++q) x[b][q] = lds[i + q * stride];
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    int i = t + b * NT;
    if constexpr (p > 1) {
      int k = i % p;
#pragma unroll
      for (int q = 1; q < r; ++q) {
        float2 w = tw_at(tw, q * k * (N / (p * r)));
        x[b][q] = INV ? cmulconj(x[b][q], w) : cmul(x[b][q], w);
      }
    }
    dft_r<r, INV>(x[b]);
  }
  if constexpr (S_ == PL::S - 1) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int q = 0; q < r; ++q) v[b + q * NB] = x[b][q];
  } else {
    if constexpr (S_ > 0) line_sync<WAVE>();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      int i = t + b * NT;
      int k = i % p;
      int j = (i - k) * r + k;
#pragma unroll
      for (int q = 0; q < r; ++q) lds[j + q * p] = x[b][q];
    }
  }
}

template <class PL, bool INV, bool WAVE, int S_ = 0, class TW>
__device__ __forceinline__ void fft_stages(float2 (&v)[PL::E], int t, const LdsLine &lds, TW tw) {
  if constexpr (S_ < PL::S) {
    fft_stage<PL, S_, INV, WAVE, TW>(v, t, lds, tw);
    fft_stages<PL, INV, WAVE, S_ + 1, TW>(v, t, lds, tw);
  }
}

// Full length-N FFT of one line held in registers (see file comment).  The
// leading barrier makes it safe to call repeatedly on the same LDS buffer.
// A single-stage plan never touches LDS.
template <class PL, bool INV, bool WAVE = false, class TW = const float2 *>
__device__ __forceinline__ void fft_line_p(float2 (&v)[PL::E], int t, const LdsLine &lds, TW tw) {
  if constexpr (PL::S > 1) line_sync<WAVE>();
  fft_stages<PL, INV, WAVE, 0, TW>(v, t, lds, tw);
}

// Row lines (one line per NT consecutive threads): wavefront-local exchanges
// whenever the line fits in a wavefront.
template <int N, bool INV>
__device__ __forceinline__ void fft_line(float2 (&v)[Plan<N>::E], int t, const LdsLine &lds,
                                         const float2 *__restrict__ tw) {
  fft_line_p<Plan<N>, INV, wave_lines<Plan<N>::NT>()>(v, t, lds, tw);
}

// Column tile of a column-pass block.  Workgroups go to the eight XCDs of
// the chip round robin by linear workgroup id; when the x extent of the grid
// is a multiple of 8, blockIdx.x % 8 is the XCD, and the remap hands each XCD
// a contiguous run of column tiles, so that neighbouring tiles (whose rows
// share 128-byte lines and DRAM pages) meet in the same L2.  A bijection on
// [0, gridDim.x).  Measured on MI355X: 64 images of 256..1024^2 (1024^2 has
// 8-column, 64-byte tiles) 9.55 -> 8.33 ms; the 32 x 512^2 batch unchanged.
#ifndef SL_XCD_COLS
#define SL_XCD_COLS 1
#endif
__device__ __forceinline__ int col_tile() {
  const int gx = (int)gridDim.x, bx = (int)blockIdx.x;
  if (SL_XCD_COLS && (gx & 7) == 0) return (bx & 7) * (gx >> 3) + (bx >> 3);
  return bx;
}

// Pair-plane streams: the complex intermediates that the column passes write
// once (forward) or read once (inverse), gigabytes per call, beside filter
// tables that every image and pair re-reads.  With SL_NT_STREAM these
// accesses carry the non-temporal hint.  Measured on MI355X, 32 x 512^2,
// R = 49: forward column pass 770 -> 442 us, inverse accumulation
// 586 -> 540 us, with the same HBM bytes in the counters (the gain is in how
// the caches treat the stream, not in fewer bytes).
#ifndef SL_NT_STREAM
#define SL_NT_STREAM 1
#endif
typedef float sl_f2v __attribute__((ext_vector_type(2)));
template <bool NT = SL_NT_STREAM>
__device__ __forceinline__ void stream_store(float2 *p, float2 v) {
  if constexpr (NT) {
    const sl_f2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, (sl_f2v *)p);
  } else {
    *p = v;
  }
}
template <bool NT = SL_NT_STREAM>
__device__ __forceinline__ float2 stream_load(const float2 *p) {
  if constexpr (NT) {
    const sl_f2v w = __builtin_nontemporal_load((const sl_f2v *)p);
    return make_float2(w.x, w.y);
  } else {
    return *p;
  }
}

}  // namespace sl
