// XCD-cooperative 2D transform passes (Algorithms 1 and 2 of the paper by the
// convolution theorem, Section 4) for 512 x 512 planes on gfx950.
//
// The line passes (kernels2d.hip) exchange every subband-pair plane between
// their column and row FFTs through HBM: the complex intermediate is written
// and read once per direction, as many bytes again as the coefficients.  Here
// the 32 workgroups of one XCD transform one plane together and exchange it
// through a 2 MiB scratch plane that stays in that XCD's 4 MiB L2.
//
// Work split.  Workgroups reach the XCDs round robin; each reads its XCD id
// from the XCC_ID register and draws a rank r in [0, 32) from a per-XCD
// ticket.  XCD k transforms images k, k + 8, ... one after the other.  In the
// column phases workgroup r owns the 16 columns 16 r .. 16 r + 15 (64 threads
// per column, 8 values per thread), in the row phases the 16 rows 16 r ..
// 16 r + 15 (one row per wavefront).  The image spectrum F (forward) and the
// accumulator of Algorithm 2 (inverse) stay in the registers of the column
// owner for all subband pairs of the image.
//
// Synchronisation.  Two counters per XCD count arrivals: A after a phase
// wrote the scratch plane, B after a phase finished reading it.  Each wait is
// for the 32 arrivals of one generation (monotonic targets 32 n), polled with
// agent-scope loads of the counter.  Writers store normally (the stores are
// acknowledged by the L2 before the arrive); after a completed wait the
// reader invalidates its compute unit's L1 (which may hold stale lines of
// earlier planes) and loads normally from the XCD's L2.  The agent-scope
// release / acquire fences, which write back and invalidate the whole L2,
// are not used.  The phases are software pipelined so that the waits
// overlap FFT work: a workgroup arrives on A, computes the next pair's column
// FFT in registers, then waits for A; it arrives on B as soon as its scratch
// loads have landed, before its row FFT and stores.
//
// Every wait is bounded: after spin polls without the target it sets the
// XCD's abort word and the host-visible error flag and returns; the other
// workgroups of that XCD see the abort word at their next wait and return
// too, so the kernel always drains.  The host reports the flag as SL_EHIP.
#include <hip/hip_runtime.h>

#include "dispatch.hpp"
#include "fft_core.hpp"

namespace sl {

namespace {

constexpr int XN = 512;        // plane side
constexpr int XG = 32;         // workgroups per XCD (one per compute unit)
constexpr int XM = 16;         // rows / columns of a workgroup
constexpr int XT = 1024;       // threads per workgroup (16 waves, up to 128 VGPRs each)
constexpr int XCDS = 8;
constexpr int kCtr = 32;       // unsigned words per XCD counter line (128 bytes)
// LDS per workgroup: the FFT exchange (72 KiB), the column tile that
// persists over an image (64 KiB: F in the forward, the accumulator in the
// inverse, kept out of the registers that the pipelined phases need) and
// the twiddles, 140 KiB: one workgroup per compute unit
constexpr size_t kPadLds = 0;

using XPlan = Plan<XN>;        // one wave per row line, 64 threads per column line, 8 values
using XPlanC = XPlan;
static_assert(XPlan::E == 8 && XPlan::NT == 64 && XPlan::NT * XM == XT,
              "512-point lines: 64 threads x 8 values");
constexpr int CE = XPlanC::E, CNT = XPlanC::NT;   // column values per thread, threads per column
static_assert(XG * XM == XN, "one workgroup per 16 lines");

// counter line of an XCD: [0] rank ticket, [1] A arrivals, [2] B arrivals,
// [3] abort word
__device__ __forceinline__ unsigned xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;   // HW_REG_XCC_ID[3:0]
}

__device__ __forceinline__ void x_arrive(unsigned *cnt) {
  __builtin_amdgcn_s_waitcnt(0);   // this wave's stores and loads have completed
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool x_wait(unsigned *cnt, unsigned target, unsigned *abort, int spin,
                                       int *err) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    int res = 1;
    for (int i = 0;; ++i) {
      if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        res = 0;
        break;
      }
      if (i >= spin) {
        __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (err) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        res = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // Invalidate this compute unit's L1 (it may hold lines of the scratch
    // plane from an earlier phase), so that the phase's plain loads are served
    // by the XCD's L2, where the other workgroups' stores have landed: the L1
    // invalidation of a workgroup-scope acquire.  Loads with agent scope would
    // also miss the L1, but make the L2 write every dirty scratch line back to
    // memory (measured: a second coefficient tensor's worth of HBM writes).
    if (res) asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
    ok = res;
  }
  __syncthreads();
  return ok != 0;
}

// Buffer accesses: a uniform base in a resource descriptor (SGPRs), a 32-bit
// per-thread byte offset and a uniform byte offset, so that the strided
// element addresses of a line are not held in 64-bit registers; accesses
// past the descriptor's size read 0 and write nothing.  AUX: 0 plain, kNT
// the non-temporal hint (streams read or written once: input, filters,
// coefficients).
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned u2v __attribute__((ext_vector_type(2)));
constexpr int kNT = 2;
__device__ __forceinline__ Rsrc mkbuf(const void *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <int AUX>
__device__ __forceinline__ float2 bld2(Rsrc r, unsigned voff, unsigned soff) {
  const u2v v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
template <int AUX>
__device__ __forceinline__ void bst2(float2 x, Rsrc r, unsigned voff, unsigned soff) {
  const u2v v = {__float_as_uint(x.x), __float_as_uint(x.y)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, AUX);
}
template <int AUX>
__device__ __forceinline__ float bld1(Rsrc r, unsigned voff, unsigned soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}
template <int AUX>
__device__ __forceinline__ void bst1(float x, Rsrc r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, soff, AUX);
}

// Rank of this workgroup within its XCD (block-uniform); -1 aborts.
__device__ __forceinline__ int x_rank(unsigned *c, int *err) {
  __shared__ int s_rank;
  if (threadIdx.x == 0) {
    int r = (int)__hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (r >= XG) {
      // more workgroups on this XCD than it has compute units: not the
      // round-robin distribution the split assumes
      __hip_atomic_store(c + 3, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (err) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      r = -1;
    }
    s_rank = r;
  }
  __syncthreads();
  return s_rank;
}


}  // namespace

struct XcdArgs {
  const float *x;        // forward input [B][512][512]
  float *coef;           // [B][R][512][512] float32
  float *out;            // inverse output [B][512][512]
  const float *filt;     // [R][512][512]
  const float *psi;      // [512][512]
  const float2 *tw;      // 512 twiddles
  float2 *S;             // 8 scratch planes
  unsigned *ctr;         // 8 counter lines
  int *err;              // host-visible error flag (may be null)
  int B, R, spin;
  float inv_n;           // 1 / (512 * 512)
  ThrArgs thr;
};

// Element offsets of a workgroup's lines.  Row phases: wave w transforms row
// 16 r + w, thread t owns elements t + 64 e (per-thread offset of the row and
// lane, uniform offset 64 e).  Column phases: 64 threads per column, thread t
// owns rows t + 64 e (per-thread offset of the row and column, uniform
// offset 64 e rows).
struct XLines {
  int rm, rt, cm, ct;
  unsigned ro[1];   // element offset of the thread's first element in its row
  unsigned co;      // element offset of the thread's first element in its column
  __device__ XLines(int r) {
    rm = threadIdx.x >> 6;
    rt = threadIdx.x & 63;
    cm = threadIdx.x & 15;
    ct = threadIdx.x >> 4;
    ro[0] = (unsigned)(r * XM + rm) * XN + rt;
    co = (unsigned)ct * XN + r * XM + cm;
  }
  static constexpr unsigned row_step = 64, col_step = (unsigned)CNT * XN;   // elements
};

// Forward: x -> row DFT -> S -> column DFT (F, kept in LDS) -> per pair:
// F (psi_a + i psi_b) -> column IDFT -> S -> row IDFT -> c_a, c_b.
__global__ void __launch_bounds__(XT) k_xcd_fwd(XcdArgs a) {
  __shared__ float2 lds[XM * row_lds_len<XN>()];
  __shared__ float2 tile[XN * XM];
  __shared__ float2 twl[XN];
  const unsigned xcc = xcc_id();
  unsigned *c = a.ctr + xcc * kCtr;
  for (int i = threadIdx.x; i < XN; i += XT) twl[i] = a.tw[i];
  const int r = x_rank(c, a.err);   // its barrier also orders the twiddle stores
  if (r < 0) return;
  unsigned *cA = c + 1, *cB = c + 2, *abort = c + 3;
  const XLines L(r);
  const int ct = L.ct;
  const LdsLine rl[1] = {{lds + L.rm * row_lds_len<XN>(), 0}};
  const LdsLine cl{lds + L.cm, XM};
  float2 *ft = tile + ct * XM + L.cm;                        // F of (row ct + 64 e, col)
  const TwLds tw{twl};
  const size_t plane = (size_t)XN * XN;
  const unsigned pb4 = (unsigned)plane * 4;
  const Rsrc rS = mkbuf(a.S + (size_t)xcc * plane, (unsigned)plane * 8);
  const Rsrc rF = mkbuf(a.filt, (unsigned)a.R * pb4);
  const int P = (a.R + 1) / 2;
  unsigned nA = 0, nB = 0;

  // F (psi_a + i psi_b) for pair p, then the column IDFT, into V
  auto col_ifft = [&](int p, float2 (&V)[CE]) {
    const int ia = 2 * p, ib = ia + 1;
    const unsigned sa = (unsigned)ia * pb4, sb = (unsigned)(ib < a.R ? ib : ia) * pb4;
#pragma unroll
    for (int e = 0; e < CE; ++e) {
      const unsigned so = e * XLines::col_step * 4;
      const float fa_ = bld1<kNT>(rF, L.co * 4, sa + so);
      const float fb_ = ib < a.R ? bld1<kNT>(rF, L.co * 4, sb + so) : 0.f;
      const float2 f = ft[e * CNT * XM];
      V[e] = make_float2(f.x * fa_ - f.y * fb_, f.y * fa_ + f.x * fb_);
    }
    fft_line_p<XPlanC, true>(V, ct, cl, tw);
  };

  for (int b = (int)xcc; b < a.B; b += XCDS) {
    // rows of x: row DFT into the scratch plane
    if (!x_wait(cB, XG * nB, abort, a.spin, a.err)) return;
    {
      const Rsrc rx = mkbuf(a.x + (size_t)b * plane, pb4);
      float2 v[1][8];
#pragma unroll
      for (int h = 0; h < 1; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[h][e] = make_float2(bld1<kNT>(rx, L.ro[h] * 4, e * XLines::row_step * 4), 0.f);
#pragma unroll
      for (int h = 0; h < 1; ++h) fft_line_p<XPlan, false, true>(v[h], L.rt, rl[h], tw);
#pragma unroll
      for (int h = 0; h < 1; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) bst2<0>(v[h][e], rS, L.ro[h] * 8, e * XLines::row_step * 8);
    }
    x_arrive(cA);
    ++nA;
    // columns: the spectrum tile F of this workgroup, kept in LDS
    if (!x_wait(cA, XG * nA, abort, a.spin, a.err)) return;
    {
      float2 f[CE];
#pragma unroll
      for (int e = 0; e < CE; ++e) f[e] = bld2<0>(rS, L.co * 8, e * XLines::col_step * 8);
      x_arrive(cB);
      ++nB;
      fft_line_p<XPlanC, false>(f, ct, cl, tw);
#pragma unroll
      for (int e = 0; e < CE; ++e) ft[e * CNT * XM] = f[e];
    }
    __syncthreads();   // the F tile is complete before col_ifft reads it
    float2 V[CE];
    col_ifft(0, V);
    for (int p = 0; p < P; ++p) {
      if (!x_wait(cB, XG * nB, abort, a.spin, a.err)) return;
#pragma unroll
      for (int e = 0; e < CE; ++e) bst2<0>(V[e], rS, L.co * 8, e * XLines::col_step * 8);
      x_arrive(cA);
      ++nA;
      if (p + 1 < P) col_ifft(p + 1, V);   // overlaps the other workgroups' stores
      if (!x_wait(cA, XG * nA, abort, a.spin, a.err)) return;
      float2 u[1][8];
#pragma unroll
      for (int h = 0; h < 1; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) u[h][e] = bld2<0>(rS, L.ro[h] * 8, e * XLines::row_step * 8);
      x_arrive(cB);
      ++nB;
#pragma unroll
      for (int h = 0; h < 1; ++h) fft_line_p<XPlan, true, true>(u[h], L.rt, rl[h], tw);
      const int ia = 2 * p, ib = ia + 1;
      const Rsrc ra = mkbuf(a.coef + ((size_t)b * a.R + ia) * plane, pb4);
#pragma unroll
      for (int h = 0; h < 1; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          bst1<kNT>(u[h][e].x * a.inv_n, ra, L.ro[h] * 4, e * XLines::row_step * 4);
      if (ib < a.R) {
        const Rsrc rb = mkbuf(a.coef + ((size_t)b * a.R + ib) * plane, pb4);
#pragma unroll
        for (int h = 0; h < 1; ++h)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            bst1<kNT>(u[h][e].y * a.inv_n, rb, L.ro[h] * 4, e * XLines::row_step * 4);
      }
    }
  }
}

// Inverse: per pair, c_a + i c_b (hard threshold on load) -> row DFT -> S ->
// column DFT -> ACC += (psi_a - i psi_b) (...), ACC kept in LDS; then ACC /
// Psi_hat -> column IDFT -> S -> row IDFT -> real part / (512 * 512).
__global__ void __launch_bounds__(XT) k_xcd_inv(XcdArgs a) {
  __shared__ float2 lds[XM * row_lds_len<XN>()];
  __shared__ float2 tile[XN * XM];
  __shared__ float2 twl[XN];
  const unsigned xcc = xcc_id();
  unsigned *c = a.ctr + xcc * kCtr;
  for (int i = threadIdx.x; i < XN; i += XT) twl[i] = a.tw[i];
  const int r = x_rank(c, a.err);
  if (r < 0) return;
  unsigned *cA = c + 1, *cB = c + 2, *abort = c + 3;
  const XLines L(r);
  const int ct = L.ct;
  const LdsLine rl[1] = {{lds + L.rm * row_lds_len<XN>(), 0}};
  const LdsLine cl{lds + L.cm, XM};
  float2 *at = tile + ct * XM + L.cm;                        // ACC of (row ct + 64 e, col)
  const TwLds tw{twl};
  const size_t plane = (size_t)XN * XN;
  const unsigned pb4 = (unsigned)plane * 4;
  const Rsrc rS = mkbuf(a.S + (size_t)xcc * plane, (unsigned)plane * 8);
  const Rsrc rF = mkbuf(a.filt, (unsigned)a.R * pb4);
  const Rsrc rP = mkbuf(a.psi, pb4);
  const int P = (a.R + 1) / 2;
  unsigned nA = 0, nB = 0;

  // coefficient rows of pair p of image b, thresholded, row DFT, into U
  auto row_fft = [&](int b, int p, float2 (&U)[1][8]) {
    const int ia = 2 * p, ib = ia + 1;
    const bool has_b = ib < a.R;
    float da = 0.f, db = 0.f;
    if (a.thr.sigma) {
      const float sg = a.thr.sigma[b];
      const int ja = a.thr.jof[ia];
      if (ja >= 0) da = (a.thr.K[ja] * sg) * a.thr.l2[ia];
      if (has_b) {
        const int jb = a.thr.jof[ib];
        if (jb >= 0) db = (a.thr.K[jb] * sg) * a.thr.l2[ib];
      }
    }
    const Rsrc ra = mkbuf(a.coef + ((size_t)b * a.R + ia) * plane, pb4);
    const Rsrc rb = mkbuf(a.coef + ((size_t)b * a.R + (has_b ? ib : ia)) * plane, pb4);
    float va[1][8], vb[1][8];
#pragma unroll
    for (int h = 0; h < 1; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        va[h][e] = bld1<kNT>(ra, L.ro[h] * 4, e * XLines::row_step * 4);
        vb[h][e] = bld1<kNT>(rb, L.ro[h] * 4, e * XLines::row_step * 4);   // ignored without a partner
      }
#pragma unroll
    for (int h = 0; h < 1; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float x0 = va[h][e], x1 = has_b ? vb[h][e] : 0.f;
        if (!(fabsf(x0) >= da)) x0 = 0.f;
        if (!(fabsf(x1) >= db)) x1 = 0.f;
        U[h][e] = make_float2(x0, x1);
      }
#pragma unroll
    for (int h = 0; h < 1; ++h) fft_line_p<XPlan, false, true>(U[h], L.rt, rl[h], tw);
  };

  for (int b = (int)xcc; b < a.B; b += XCDS) {
#pragma unroll
    for (int e = 0; e < CE; ++e) at[e * CNT * XM] = make_float2(0.f, 0.f);
    float2 U[1][8];
    row_fft(b, 0, U);
    for (int p = 0; p < P; ++p) {
      if (!x_wait(cB, XG * nB, abort, a.spin, a.err)) return;
#pragma unroll
      for (int h = 0; h < 1; ++h)
#pragma unroll
        for (int e = 0; e < 8; ++e) bst2<0>(U[h][e], rS, L.ro[h] * 8, e * XLines::row_step * 8);
      x_arrive(cA);
      ++nA;
      if (p + 1 < P) row_fft(b, p + 1, U);    // overlaps the other workgroups' stores
      if (!x_wait(cA, XG * nA, abort, a.spin, a.err)) return;
      float2 w[CE];
#pragma unroll
      for (int e = 0; e < CE; ++e) w[e] = bld2<0>(rS, L.co * 8, e * XLines::col_step * 8);
      x_arrive(cB);
      ++nB;
      fft_line_p<XPlanC, false>(w, ct, cl, tw);
      const int ia = 2 * p, ib = ia + 1;
      const unsigned sa = (unsigned)ia * pb4, sb = (unsigned)(ib < a.R ? ib : ia) * pb4;
#pragma unroll
      for (int e = 0; e < CE; ++e) {
        const unsigned so = e * XLines::col_step * 4;
        const float fva = bld1<kNT>(rF, L.co * 4, sa + so);
        const float fvb = ib < a.R ? bld1<kNT>(rF, L.co * 4, sb + so) : 0.f;
        // (psi_a - i psi_b) * w
        float2 acc = at[e * CNT * XM];
        acc.x += fva * w[e].x + fvb * w[e].y;
        acc.y += fva * w[e].y - fvb * w[e].x;
        at[e * CNT * XM] = acc;
      }
    }
    // dual-frame division and the column IDFT
    float2 v[CE];
#pragma unroll
    for (int e = 0; e < CE; ++e) {
      const float d = bld1<0>(rP, L.co * 4, e * XLines::col_step * 4);
      const float2 acc = at[e * CNT * XM];
      v[e] = make_float2(acc.x / d, acc.y / d);
    }
    fft_line_p<XPlanC, true>(v, ct, cl, tw);
    if (!x_wait(cB, XG * nB, abort, a.spin, a.err)) return;
#pragma unroll
    for (int e = 0; e < CE; ++e) bst2<0>(v[e], rS, L.co * 8, e * XLines::col_step * 8);
    x_arrive(cA);
    ++nA;
    if (!x_wait(cA, XG * nA, abort, a.spin, a.err)) return;
    float2 u[1][8];
#pragma unroll
    for (int h = 0; h < 1; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e) u[h][e] = bld2<0>(rS, L.ro[h] * 8, e * XLines::row_step * 8);
    x_arrive(cB);
    ++nB;
#pragma unroll
    for (int h = 0; h < 1; ++h) fft_line_p<XPlan, true, true>(u[h], L.rt, rl[h], tw);
    const Rsrc rx = mkbuf(a.out + (size_t)b * plane, pb4);
#pragma unroll
    for (int h = 0; h < 1; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        bst1<0>(u[h][e].x * a.inv_n, rx, L.ro[h] * 4, e * XLines::row_step * 4);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
size_t xcd_scratch_bytes() { return (size_t)XCDS * XN * XN * sizeof(float2) + XCDS * kCtr * 4; }

// Whether this device and launch shape can run the cooperative passes: every
// workgroup of the grid must be resident at once (one per compute unit).
bool xcd_supported(const Sys2D &s, int B) {
  if (s.H != XN || s.W != XN || s.dtype != 0 || B < XCDS) return false;
  if (s.num_cu != XCDS * XG) return false;
  static int occ_f = -1, occ_i = -1;
  if (occ_f < 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, (const void *)k_xcd_fwd, XT, kPadLds) !=
        hipSuccess)
      occ_f = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_i, (const void *)k_xcd_inv, XT, kPadLds) !=
        hipSuccess)
      occ_i = 0;
  }
  return occ_f >= 1 && occ_i >= 1;
}

static XcdArgs xcd_args(const Sys2D &s, void *scratch, int *err, int B, int spin) {
  XcdArgs a{};
  a.filt = s.filt;
  a.psi = s.psi;
  a.tw = s.twW;
  a.S = (float2 *)scratch;
  a.ctr = (unsigned *)((char *)scratch + (size_t)XCDS * XN * XN * sizeof(float2));
  a.err = err;
  a.B = B;
  a.R = s.R;
  a.spin = spin;
  a.inv_n = 1.0f / (float)(XN * XN);
  return a;
}

hipError_t launch_xcd_fwd(const Sys2D &s, const float *x, float *coef, void *scratch, int *err,
                          int B, int spin, hipStream_t st) {
  XcdArgs a = xcd_args(s, scratch, err, B, spin);
  a.x = x;
  a.coef = coef;
  hipError_t e = launch_zero_u32(a.ctr, XCDS * kCtr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xcd_fwd, dim3(XCDS * XG), dim3(XT), kPadLds, st, a);
  return hipGetLastError();
}

hipError_t launch_xcd_inv(const Sys2D &s, const float *coef, const ThrArgs &thr, float *x,
                          void *scratch, int *err, int B, int spin, hipStream_t st) {
  XcdArgs a = xcd_args(s, scratch, err, B, spin);
  a.coef = (float *)coef;
  a.out = x;
  a.thr = thr;
  hipError_t e = launch_zero_u32(a.ctr, XCDS * kCtr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xcd_inv, dim3(XCDS * XG), dim3(XT), kPadLds, st, a);
  return hipGetLastError();
}

}  // namespace sl
