// Host-side launchers of the device passes (internal to libshearlet).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sl {

constexpr int kMaxScales = 8;

// Hard-threshold parameters fused into the first inverse pass.
struct ThrArgs {
  const float *sigma;   // [B] device, or null = no thresholding
  const float *l2;      // [R] device ||psi_i||_2 (float32)
  const int *jof;       // [R] device scale index (-1 = lowpass)
  float K[kMaxScales];
};

// Per-call view of the 2D system tables.
struct Sys2D {
  int H, W, R, dtype;
  int num_cu;               // compute units of the device (grid sizing)
  int inv_images;           // images per inverse accumulation block: 0 = by
                            // batch (2, or 1 for a single image), or 1 / 2
  int split_pairs;          // 1: small grids split the pair loop over blocks
  int line_em;              // line plan of the coefficient row passes: 1, or 2
                            // (twice the values per thread) for 1024-point rows
  const float *filt;        // [R][H][W]
  const float *psi;         // [H][W]  Psi_hat
  const float *l1;          // [R]
  const float2 *twH, *twW;  // twiddles exp(-2 pi i m / N), N = H and N = W
};

// Chunk of (images, subband pairs) processed between two passes.
struct Chunk {
  int b0, nb, p0, np;
};

bool lines_supported(int n);

// Forward passes --------------------------------------------------------------
// x [B][H][W] real -> A [B][H][W] complex (row DFT); xmax[b] = max |x_b| bits
hipError_t launch_rows_real_fft(const Sys2D &s, const float *x, float2 *A, unsigned *xmax, int B,
                                hipStream_t st);
// Inpainting input of one iteration (Algorithm 3), formed while the rows are
// loaded: x = fm where mask != 0, else f (0 when first: the iteration starts
// from f = 0 and f is not read).  The launch also writes the iteration's
// threshold scale sigma[b] = delta_init[b] * fac, b < B.
struct MixArgs {
  const float *fm;
  const uint8_t *mask;
  const float *f;
  int first;
  const float *delta_init;
  float fac;
  float *sigma;
};
// launch_rows_real_fft with x formed by MixArgs (no max-|x|)
hipError_t launch_rows_real_fft_mix(const Sys2D &s, const MixArgs &mix, float2 *A, int B,
                                    hipStream_t st);
// A -> F (column DFT, or inverse DFT without scaling when inverse is set);
// stream marks A and F as pair-plane streams read or written once (accessed
// with the non-temporal hint)
hipError_t launch_cols_fft(const Sys2D &s, const float2 *A, float2 *F, int B, bool inverse,
                           hipStream_t st, bool stream = false);
// F, filters -> T[chunk] (filter pair multiply + column inverse DFT)
hipError_t launch_cols_filter_ifft(const Sys2D &s, const float2 *F, float2 *T, Chunk c,
                                   hipStream_t st);
// T[chunk] -> coefficients (row inverse DFT, pair split, storage encode)
hipError_t launch_rows_coef(const Sys2D &s, const float2 *T, void *coef, const float *scales,
                            Chunk c, hipStream_t st);
// scales[b][i] from xmax and l1 norms (F16 / BF16 storage)
hipError_t launch_scales(const Sys2D &s, const unsigned *xmax, float *scales, int B,
                         hipStream_t st);
hipError_t launch_zero_u32(unsigned *p, int n, hipStream_t st);
hipError_t launch_div_psi(float2 *F, const float *psi, size_t npix, int B, hipStream_t st);

// Inverse passes --------------------------------------------------------------
// coefficients -> U[chunk] (decode, threshold, pair pack, row DFT)
hipError_t launch_rows_coef_fft(const Sys2D &s, const void *coef, const float *scales, float2 *U,
                                Chunk c, const ThrArgs &thr, hipStream_t st);
// T[chunk] -> T[chunk] in place: row IDFT, scale inv_n, hard threshold, row DFT
// (denoising without materialised coefficients)
hipError_t launch_rows_thr(const Sys2D &s, float2 *T, float inv_n, Chunk c, const ThrArgs &thr,
                           hipStream_t st);
// U[chunk] -> ACC (column DFT, multiply by the filter pair, sum over pairs);
// the last chunk divides by Psi_hat and applies the column inverse DFT.
// With G > 1 pair groups (inv_pair_groups) group z sums into part[z - 1]
// ([G - 1][Btot] planes), and launch_cols_acc_finish completes the sum, the
// division and the column inverse DFT after the last chunk.
int inv_pair_groups(const Sys2D &s, int nb, int np);
hipError_t launch_cols_fft_acc(const Sys2D &s, const float2 *U, float2 *ACC, float2 *part, int G,
                               int Btot, Chunk c, bool first, bool last, hipStream_t st);
hipError_t launch_cols_acc_finish(const Sys2D &s, float2 *ACC, const float2 *part, int G, int B,
                                  hipStream_t st);
// ACC -> x (row inverse DFT, real part, 1/(HW))
hipError_t launch_rows_real_ifft(const Sys2D &s, const float2 *V, float *x, int B, hipStream_t st);

// ---- multi-class coefficient row passes (uneven batches) ---------------------
// One launch runs the coefficient row pass of several size classes: the
// forward's row IDFT and coefficient store (T -> coef, as launch_rows_coef)
// or the inverse's coefficient load, threshold and row DFT (coef -> U, as
// launch_rows_coef_fft).  Every class must have the same storage type.
constexpr int kMaxMultiClasses = 8;
struct MultiRowClass {
  const float2 *T;        // forward input (chunk pair planes)
  float2 *U;              // inverse output (chunk pair planes)
  void *coef;
  const float *scales;
  const float2 *tw;       // twiddles of the row length
  ThrArgs thr;            // inverse threshold
  float inv_hw;
  int W, H, R, b0, p0, np, G, nblocks, block0;
};
struct MultiRows {
  MultiRowClass c[kMaxMultiClasses];
  int n;
};
bool multi_rows_supported(const Sys2D &s);
// fills the geometry fields of k for chunk c of the class with view s
void multi_rows_class_geometry(const Sys2D &s, const Chunk &c, MultiRowClass &k);
hipError_t launch_rows_multi(MultiRows &a, int dtype, bool forward, hipStream_t st);

// ---- XCD-cooperative passes (xcd2d.hip) --------------------------------------
// 512 x 512 planes, float32 coefficients: the 32 workgroups of each XCD
// transform one image at a time and exchange every plane through a scratch
// plane in the XCD's L2.  scratch holds xcd_scratch_bytes() (8 planes and 8
// counter lines); err (host-visible, may be null) is set when a bounded wait
// gives up, in which case the results are invalid.
bool xcd_supported(const Sys2D &s, int B);
size_t xcd_scratch_bytes();
// x -> coefficients (Algorithm 1)
hipError_t launch_xcd_fwd(const Sys2D &s, const float *x, float *coef, void *scratch, int *err,
                          int B, int spin, hipStream_t st);
// coefficients (hard threshold on load if thr.sigma) -> x (Algorithm 2)
hipError_t launch_xcd_inv(const Sys2D &s, const float *coef, const ThrArgs &thr, float *x,
                          void *scratch, int *err, int B, int spin, hipStream_t st);

// ---- 3D --------------------------------------------------------------------
// Filter of one subband generated from its factors (see kernels3d.hip):
//   lowpass (cone 0): tab[g_off + x] * tab[p1_off + y] * tab[p2_off + z]
//   otherwise: g[xi_am] * plane1[xi_s1][xi_am] * plane2[xi_s2][xi_am] with
//   axes numbered 1 = x (W), 2 = y (H), 3 = z (D) and planes of row length n_main.
// Filters of subband pair p (a = 2p, b = 2p + 1) along the z line of voxel
// column (y, x): psi(z) = C[c + y W + x] * X[x + z W] * Y[y + z H] (float2:
// the value for a, the value for b), with X or Y absent (= 1) when the
// offset is negative.  Offsets count float2 elements of Sys3D::tab.
struct ZPair {
  long long c, x, y;
};

struct Sys3D {
  int D, H, W, R, dtype;
  int num_cu;                 // compute units of the device (grid sizing)
  const ZPair *pairs;         // [(R + 1) / 2]
  const float2 *tab;          // per-pair factor blocks
  const float *psi;           // [D][H][W] Psi_hat
  const float2 *twD;
};

// zdft: F carries the x and y transforms only and the kernel takes its DFT
// along z itself
hipError_t launch_z_filter_ifft(const Sys3D &s, const float2 *F, float2 *T, Chunk c, bool zdft,
                                hipStream_t st);

// Plane passes: the y and x line FFTs of each z-slice of a chunk's pair
// volumes in LDS (s: the slice view, H x W with twiddles of both lengths;
// D slices per volume).  plane_supported(H, W) tells which slice shapes
// have them.  Results equal the separate line passes bit for bit.
bool plane_supported(int H, int W);
// T (after the z IDFT) -> y IDFT -> x IDFT -> coefficients (as rows_coef)
hipError_t launch_plane_coef(const Sys2D &s, int D, const float2 *T, void *coef,
                             const float *scales, Chunk c, float inv_n, hipStream_t st);
// coefficients (decode, threshold) -> x DFT -> y DFT -> U (for z_fft_acc)
hipError_t launch_plane_coef_fft(const Sys2D &s, int D, const void *coef, const float *scales,
                                 float2 *U, Chunk c, const ThrArgs &thr, hipStream_t st);
// T -> y IDFT, x IDFT, scale, threshold, x DFT, y DFT -> T (fused denoise)
// Half-plane passes: slices too large for LDS, split in y into two halves
// (one decimation-in-frequency step); forward and inverse only.  Results
// agree with the line passes to float32 rounding.
bool half_plane_supported(int H, int W);
hipError_t launch_hplane_coef(const Sys2D &s, int D, const float2 *T, void *coef,
                              const float *scales, Chunk c, float inv_n, hipStream_t st);
hipError_t launch_hplane_coef_fft(const Sys2D &s, int D, const void *coef, const float *scales,
                                  float2 *U, Chunk c, const ThrArgs &thr, hipStream_t st);
hipError_t launch_plane_thr(const Sys2D &s, int D, float2 *T, float inv_n, Chunk c,
                            const ThrArgs &thr, hipStream_t st);
hipError_t launch_z_fft_acc(const Sys3D &s, const float2 *U, float2 *ACC, Chunk c, bool first,
                            bool last, hipStream_t st);

}  // namespace sl
