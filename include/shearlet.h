/*
 * shearlet.h -- C ABI of the MI355X digital shearlet transform library
 * (libshearlet.so).  Undecimated 2D and 3D digital shearlet transform with
 * compactly supported shearlets as defined in "ShearLab 3D: Faithful Digital
 * Shearlet Transforms based on Compactly Supported Shearlets" (Kutyniok,
 * Lim, Reisenhofer, 2014).
 *
 * Conventions shared by every call
 *   - Arrays are row-major with x1 fastest: a 2D signal is [H][W] = [N2][N1],
 *     a 3D signal is [D][H][W] = [N3][N2][N1]; a batch adds a leading [B].
 *   - The coefficient tensor is subband-major: [B][R][H][W] (2D) or
 *     [B][R][D][H][W] (3D), each subband plane contiguous.  (The paper's
 *     MATLAB example stores rows x cols x R with the subband index last,
 *     Section 4.3; the layout here keeps each plane contiguous for streaming.)
 *   - Subband order: index 0 is the lowpass; then for each scale j = 0..J-1
 *     (coarse to fine) 2D: cone 1 for k = -L..L, cone 2 for k = -L+1..L-1
 *     (k = -L..L with full_system), L = 2^{shear_levels[j]};
 *     3D: pyramids 1, 2, 3, each with k1 outer and k2 inner in -L..L,
 *     pyramid 2 skipping |k1| = L and pyramid 3 skipping |k1| = L or |k2| = L
 *     unless full_system (Section 4.4).
 *   - Pointers named *_dev are device pointers (hipMalloc'ed by the caller,
 *     e.g. through PyTorch); pointers named *_host are host memory.  The
 *     caller owns every buffer it passes; the library owns sl_system.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     GPU calls are asynchronous on that stream; argument errors are
 *     returned synchronously, kernel faults surface at the caller's next
 *     synchronisation.
 *   - Every call returns an sl_status (0 = success) and never aborts;
 *     sl_last_error() describes the last failure of the calling thread.
 */
#ifndef SHEARLET_H_
#define SHEARLET_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SL_OK = 0,
  SL_EINVAL = -1,        /* bad argument or configuration                   */
  SL_ENOMEM = -2,        /* allocation failed or workspace too small        */
  SL_EUNSUPPORTED = -3,  /* a dimension the device FFT does not support      */
  SL_EILLCOND = -4,      /* min Psi_hat / max Psi_hat < 1e-6                */
  SL_EHIP = -5           /* a HIP runtime call failed                       */
};

enum { SL_F32 = 0, SL_F16 = 1, SL_BF16 = 2 };   /* coefficient storage type */

/* Shearlet system parameters (Algorithm 1's inputs, Section 4.1; the
 * MATLAB interface of Section 4.3).                                          */
typedef struct {
  int ndim;                   /* 2 or 3                                        */
  int64_t dims[3];            /* [H, W] or [D, H, W]; each 2^a or 3*2^a, 8..1024 */
  int n_scales;               /* J >= 1 (nScales)                               */
  const int *shear_levels;    /* host, length J, d_j in 0..4, coarse to fine    */
  const double *qmf;          /* host, odd length, symmetric 1D lowpass h with
                                 centre tap in the middle; NULL = the 9-tap
                                 maximally flat h_ShearLab (Section 5.1)        */
  int qmf_len;
  const double *dir_filter;   /* host [dir_rows][dir_cols] taps of the fan
                                 filter P, rows along x2, odd sizes, centred,
                                 point-symmetric; NULL = the maximally flat
                                 half-band fan D_2((cos 2pi eta2 -
                                 cos 2pi eta1)/2) (eq. nonsep, Section 5.1)     */
  int dir_rows, dir_cols;
  int full_system;            /* 1 keeps the seam filters (Section 4.4)         */
  int coeff_dtype;            /* SL_F32, SL_F16 or SL_BF16                      */
} sl_config;

/* One subband: cone 0 = lowpass; 1, 2 = 2D cones; 1, 2, 3 = 3D pyramids.     */
typedef struct {
  int cone, j, k1, k2;
  double l2norm;              /* ||psi_i||_2 on the grid = sqrt(mean psi_hat^2) */
  double l1norm;              /* ||psi_i||_1 on the grid (3D: Young bound)      */
} sl_subband;

typedef struct sl_system sl_system;

/* ---- host-only calls (no GPU needed) ------------------------------------ */

int sl_abi_version(void);
const char *sl_last_error(void);

/* Number of subbands R of a configuration (Sections 4.1 and 4.4).           */
int sl_config_num_subbands(const sl_config *cfg, int *R_out);

/* FP64 closed form of the frequency-domain filter bank on the DFT grid,
 * evaluated on the host (Sections 3.2.2, 3.3.2, 3.4):
 *   filters_host [R][dims...]  psi_hat_i (may be NULL),
 *   dual_host    [dims...]     Psi_hat = sum_i psi_hat_i^2 (may be NULL),
 *   subbands_host[R]           indices and norms (may be NULL).
 * Returns SL_EILLCOND when Psi_hat is not bounded away from zero.           */
int sl_build_filters_host(const sl_config *cfg, double *filters_host,
                          double *dual_host, sl_subband *subbands_host);

/* FP64 undecimated separable wavelet bank on the DFT grid (2D only): the 2D
 * digital wavelet transform of Section 3.4 built from the QMF cascades of
 * eq. lowhigh, without its subsampling (the stationary wavelet transform
 * that Section 5's image decomposition pairs with the shearlets).  Subband
 * order: lowpass h_J (x) h_J, then for j = 0..J-1 (coarse to fine) cone 1 =
 * g_{J-j} along x1 times h_{J-j} along x2, cone 2 = h_{J-j} along x1 times
 * g_{J-j} along x2, cone 3 = g_{J-j} along both; k1 = k2 = 0; R = 3 J + 1.
 * Reads dims, n_scales, qmf and coeff_dtype of cfg (ndim must be 2); the
 * shear levels, fan filter and full_system do not apply.  Outputs as for
 * sl_build_filters_host.                                                    */
int sl_build_wavelet_filters_host(const sl_config *cfg, double *filters_host,
                                  double *dual_host, sl_subband *subbands_host);

/* ---- system (host build + device upload) -------------------------------- */

/* Build the filter bank on the host in FP64, round to FP32 and upload the
 * tables plus FFT twiddles (computed in FP64, rounded to FP32) to the
 * current HIP device.  *out is owned by the library.                        */
int sl_build_system(const sl_config *cfg, sl_system **out);
/* A system holding the wavelet bank of sl_build_wavelet_filters_host: every
 * transform call accepts it like a 2D shearlet system (the pair packing,
 * thresholds and dual-frame inverse only need real, even filters).         */
int sl_build_wavelet_system(const sl_config *cfg, sl_system **out);
void sl_free_system(sl_system *s);
int sl_system_num_subbands(const sl_system *s, int *R_out);
int sl_system_subband(const sl_system *s, int i, sl_subband *out);

/* The filter bank of a built system in FP64, as evaluated before it was
 * rounded to float32 for the device (the same closed form as
 * sl_build_filters_host / sl_build_wavelet_filters_host on the system's
 * configuration): filters_host [R][dims] psi_hat_i on the DFT grid (R times
 * the sample count doubles, caller-owned); dual_host [dims] the dual-frame
 * weight Psi_hat = sum_i psi_hat_i^2 of eq. frame_filter.  Host memory only;
 * no GPU work.  SL_EINVAL for NULL arguments.                               */
int sl_get_filters(const sl_system *s, double *filters_host);
int sl_get_dual_weight(const sl_system *s, double *dual_host);

/* Device bytes of workspace needed by forward/inverse/denoise for a batch.
 * Every workspace pointer must be 16-byte aligned (SL_EINVAL otherwise).   */
int sl_workspace_size(const sl_system *s, int batch, size_t *bytes_out);

/* ---- transforms --------------------------------------------------------- */

/* Forward transform (Algorithm 1): c_i = IDFT(psi_hat_i .* DFT(x)).
 *   x_dev      [B][dims] float32
 *   coeffs_dev [B][R][dims] of the system's coefficient type
 *   scales_dev [B][R] float32 written for SL_F16/SL_BF16 storage (the stored
 *              value is c / scale); may be NULL for SL_F32
 *   workspace_dev of at least sl_workspace_size(s, B) bytes.                */
int sl_forward(const sl_system *s, const float *x_dev, int batch, void *coeffs_dev,
               float *scales_dev, void *workspace_dev, size_t workspace_bytes,
               void *stream);

/* Inverse transform (Algorithm 2 with the dual filters of eq. dual_filter):
 *   x = IDFT( sum_i DFT(c_i) .* psi_hat_i / Psi_hat ).
 * If sigma_dev is not NULL every detail coefficient is hard-thresholded on
 * load (eq. hard_tresholding): kept iff |c| >= K[j] * sigma[b] * ||psi_i||_2,
 * computed in float32 as (K[j] * sigma[b]) * l2norm_i; the lowpass is kept.
 *   sigma_dev [B] float32 or NULL;  K_host [J] float32 (ignored if no sigma). */
int sl_inverse(const sl_system *s, const void *coeffs_dev, const float *scales_dev,
               int batch, const float *sigma_dev, const float *K_host, float *x_dev,
               void *workspace_dev, size_t workspace_bytes, void *stream);

/* A trained learned-shrinkage network (see the learned-shrinkage calls
 * below): its float32 master parameters [J][SL_CNN_PARAMS] and the bfloat16
 * operand pack sl_cnn_pack built from them.  Both device buffers stay owned
 * by the caller.                                                            */
typedef struct {
  const float *params_dev;
  const void *packed_dev;
} sl_shrinkage_model;

/* Denoising T^-1 S T x: sl_forward into coeffs_dev (caller-provided,
 * [B][R][dims]), the shrinkage S, then the inverse (Section 5.3).
 *   model == NULL: S is the hard threshold of eq. hard_tresholding inside
 *     sl_inverse (kept iff |c| >= K[j] sigma[b] ||psi_i||_2, lowpass kept);
 *     sigma_dev and K_host are required and the workspace is
 *     sl_workspace_size(s, B) bytes.
 *   model != NULL: S multiplies every detail coefficient by the network's
 *     gain (sl_cnn_apply, the lowpass kept) and sl_inverse reconstructs
 *     without a threshold, so the result equals sl_forward, sl_cnn_apply and
 *     sl_inverse called in turn; K_host is ignored (may be NULL), the system
 *     must be a 2D SL_F32 one, and the workspace is
 *     sl_denoise_workspace_size(s, B, 1, ...) bytes (it holds the shrunk
 *     coefficients besides the transform's workspace).
 * Errors: SL_EINVAL for NULL or misaligned buffers or an unsupported system,
 * SL_ENOMEM for a short workspace.                                          */
int sl_denoise_workspace_size(const sl_system *s, int batch, int with_model, size_t *bytes_out);
int sl_denoise(const sl_system *s, const float *x_dev, int batch, const float *sigma_dev,
               const float *K_host, const sl_shrinkage_model *model, void *coeffs_dev,
               float *scales_dev, float *out_dev, void *workspace_dev, size_t workspace_bytes,
               void *stream);

/* Hard-threshold denoising without materialising the coefficients: the
 * forward transform's last row DFT, the threshold of eq. hard_tresholding
 * (delta = K_j sigma_b ||psi_i||_2, lowpass kept) and the inverse transform's
 * first row DFT run in one pass over each pair of subbands, so the K-fold
 * coefficient tensor never reaches memory.  Arithmetic is float32 throughout:
 * the result equals sl_denoise on an SL_F32 system (for F16/BF16 systems it
 * omits their storage rounding).  x_dev, out_dev [B][dims] float32;
 * sigma_dev [B] device; K_host [J] host; workspace as sl_workspace_size.     */
int sl_denoise_fused(const sl_system *s, const float *x_dev, int batch, const float *sigma_dev,
                     const float *K_host, float *out_dev, void *workspace_dev,
                     size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and kernels as sl_denoise_fused, with the workspace taken from
 * a static device array of SL_NOALLOC_SCRATCH_BYTES (128 MiB) that the
 * library holds on every GPU it runs on until the process ends, instead of a
 * caller buffer.  Allocates nothing.  The call needs sl_workspace_size(s, B)
 * <= SL_NOALLOC_SCRATCH_BYTES (one 512 x 512 image with R = 49 fits; larger
 * batches need a smaller chunk, sl_system_set_chunk_bytes) and returns
 * SL_ENOMEM otherwise, before any GPU work.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (several streams or threads)
 * race and must be serialised by the caller.  Nothing in the array needs to
 * start at zero; it keeps the last call's contents.  Arguments and other
 * errors as for sl_denoise_fused; must be called with the system's device
 * current.                                                                  */
#define SL_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int sl_denoise_fused_noalloc(const sl_system *s, const float *x_dev, int batch,
                             const float *sigma_dev, const float *K_host, float *out_dev,
                             void *stream);

/* Inpainting by iterative hard thresholding (Algorithm 3; Section 5, image
 * and video inpainting).  From f = 0 and with the mask M (1 = known sample),
 * iteration t = 0..iterations-1 computes
 *   g = M .* (f_masked - f) + f            (f_masked where M = 1, f elsewhere)
 *   f = T^-1 T_delta_t T g                  (as sl_denoise_fused: subband i
 *                                            kept iff |c_i| >= delta_t ||psi_i||_2,
 *                                            the lowpass kept)
 *   delta_t = delta_init[b] * lambda^t,    lambda = delta_min^(1/(iterations-1)),
 * so the last iteration thresholds at delta_init * delta_min.  The threshold
 * scale of iteration t is float32(delta_init[b] * float32(lambda^t)), lambda^t
 * computed in double; everything else is float32.
 *   f_masked_dev [B][dims] float32 (16-byte aligned); mask_dev [B][dims]
 *     bytes, nonzero = known (4-byte aligned); delta_init_dev [B] float32;
 *   t_begin, t_end: run iterations t_begin..t_end-1 of the schedule only
 *     (0 <= t_begin <= t_end <= iterations).  f_dev [B][dims] float32
 *     (16-byte aligned) holds on entry the estimate after t_begin iterations
 *     (not read when t_begin = 0) and on exit the estimate after t_end, so a
 *     long run can be split into segments with identical results;
 *   use_graph: nonzero captures the launches of the call into a HIP graph,
 *     instantiated on the first call and replayed by later calls with the
 *     same arguments (pointers included); a system keeps the 4 most recent
 *     graphs until sl_free_system.  Calls that share a system must not run
 *     concurrently from several threads while building graphs.
 *   workspace_dev of at least sl_inpaint_workspace_size(s, B) bytes
 *     (16-byte aligned).
 * Errors: SL_EINVAL for NULL or misaligned buffers, a bad iteration range
 * or delta_min < 0; SL_ENOMEM for a short workspace; SL_EHIP for a launch
 * or graph failure (the estimate is then undefined).                       */
int sl_inpaint_workspace_size(const sl_system *s, int batch, size_t *bytes_out);
int sl_inpaint(const sl_system *s, const float *f_masked_dev, const unsigned char *mask_dev,
               int batch, const float *delta_init_dev, double delta_min, int iterations,
               int t_begin, int t_end, float *f_dev, int use_graph, void *workspace_dev,
               size_t workspace_bytes, void *stream);

/* Image decomposition by iterative thresholding with two transforms
 * (Algorithm 4; Section 5, image decomposition).  From f0 = f1 = 0, iteration
 * t = 0..iterations-1 computes, from the estimates of the iteration's start,
 *   f_res = f - (f0 + f1)
 *   f0 = T0^-1 T_delta_t T0 (f_res + f0)     (system s0, e.g. shearlets)
 *   f1 = T1^-1 T_delta_t T1 (f_res + f1)     (system s1, e.g. wavelets)
 * with f_res + f0 = f - f1 and f_res + f1 = f - f0 formed directly, T_delta
 * and the schedule delta_t as in sl_inpaint (each system thresholds subband
 * i at delta_t ||psi_i||_2 and keeps its lowpass).  s0 and s1 must have the
 * same dims and device.
 *   f_dev [B][dims] float32; delta_init_dev [B] float32;
 *   f0_dev, f1_dev [B][dims] float32, distinct: on entry the estimates after
 *     t_begin iterations (not read when t_begin = 0), on exit after t_end;
 *   use_graph: as in sl_inpaint; the graphs are kept by s0, keyed by s1's
 *     identity (a system built later never reuses them);
 *   all buffers 16-byte aligned; workspace_dev of at least
 *     sl_decompose_workspace_size(s0, s1, B) bytes.
 * Errors as in sl_inpaint, plus SL_EINVAL for systems of different dims.   */
int sl_decompose_workspace_size(const sl_system *s0, const sl_system *s1, int batch,
                                size_t *bytes_out);
int sl_decompose(const sl_system *s0, const sl_system *s1, const float *f_dev, int batch,
                 const float *delta_init_dev, double delta_min, int iterations, int t_begin,
                 int t_end, float *f0_dev, float *f1_dev, int use_graph, void *workspace_dev,
                 size_t workspace_bytes, void *stream);

/* Adjoint of sl_inverse: c_i = IDFT(psi_hat_i / Psi_hat .* DFT(r)) for every
 * subband, i.e. the forward transform with the dual filters of eq.
 * dual_filter.  Used to back-propagate an image-domain loss through the
 * reconstruction.  Requires SL_F32 storage.                                  */
int sl_inverse_adjoint(const sl_system *s, const float *r_dev, int batch, float *coeffs_dev,
                       void *workspace_dev, size_t workspace_bytes, void *stream);

/* Bytes of the intermediate chunk of subband-pair planes that one pass
 * launch processes (default 2 GiB or $SL_CHUNK_MB).  Changing it changes
 * sl_workspace_size.                                                        */
int sl_system_set_chunk_bytes(sl_system *s, size_t bytes);
size_t sl_system_chunk_bytes(const sl_system *s);

/* Column tile shape of a 2D system's passes (a schedule choice; results are
 * the same up to float32 summation order):
 *   inv_images  images per inverse-accumulation block: 0 = two, or one for
 *               a single image (default); 1 or 2 forces that shape;
 *   split_pairs 1 (default): when the column grid leaves compute units idle,
 *               the subband-pair loop of the column passes is split over
 *               blocks (the inverse then sums per-group partial planes, which
 *               sl_workspace_size includes); 0 keeps one group.
 * SL_EINVAL for other values.  Changing them can change sl_workspace_size. */
int sl_system_set_block_shape(sl_system *s, int inv_images, int split_pairs);
int sl_system_block_shape(const sl_system *s, int *inv_images, int *split_pairs);

/* Line plan of the 2D passes (a schedule choice; results are the same up to
 * float32 rounding order): values_factor 1 (default) or 2, the number of
 * values each thread holds relative to the default plan.  With 2, the
 * coefficient row passes transform a 1024-point row with one wavefront (16
 * values per thread, radix exchanges without block barriers) instead of
 * two, and the inverse accumulation transforms 1024-point columns with 64
 * threads each in 512-thread blocks; other lengths and passes keep the
 * default plan.  Autotuned per size class by sl_multi_autotune.  SL_EINVAL
 * for other values.                                                         */
int sl_system_set_line_plan(sl_system *s, int values_factor);
int sl_system_line_plan(const sl_system *s, int *values_factor);

/* XCD-cooperative passes (2D, 512 x 512, SL_F32, batches of at least 8, on a
 * device of 8 XCDs x 32 compute units).  The 32 workgroups of each XCD
 * transform one image at a time and exchange every subband-pair plane
 * between the column and row FFTs through a scratch plane kept in that XCD's
 * L2, instead of through HBM; results agree with the line passes to float32
 * rounding (Algorithms 1 and 2 are computed the same way).  With enable = 1
 * (or $SL_XCD=1 at system build) sl_forward and sl_inverse take them where
 * supported; the default is 0, the line passes, which measured faster on
 * MI355X (32 x 512^2, R = 49: 2.35 against 2.67 ms per forward + inverse).
 * Their waits for the other workgroups of an XCD are bounded by spin_limit
 * polls (0 = the default, about 2^20); a wait that gives up aborts the pass
 * (invalid results) and the next call on the system returns SL_EHIP.
 * sl_system_xcd_active tells whether a call with this batch and a workspace
 * of sl_workspace_size bytes runs them.  SL_EINVAL for bad arguments.        */
int sl_system_set_xcd(sl_system *s, int enable, int spin_limit);
int sl_system_xcd_active(const sl_system *s, int batch, int *active);

/* ---- uneven batches (several image sizes in one schedule) ----------------
 * The forward (and inverse) transform of a batch of images of different
 * sizes: sl_multi_run with what = 1 is the uneven-batch forward call
 * (Algorithm 1 applied to every image with the system of its size), what = 2
 * the inverse (Algorithm 2), 3 both.  A multi-batch groups n_classes size classes: class s has its own system
 * (not owned; must outlive the multi-batch) and counts[s] images stored
 * contiguously ([counts[s]][dims_s]).  The buffer arguments below are arrays
 * of n_classes device pointers, one per class.  what: 1 = forward,
 * 2 = inverse (hard threshold if sigma_dev is not NULL: per class [counts]),
 * 3 = both.  One workspace of sl_multi_workspace_size bytes serves all
 * classes (disjoint slots, so classes may run concurrently).               */
typedef struct sl_multi sl_multi;
int sl_multi_create(sl_system *const *systems, const int *counts, int n_classes,
                    sl_multi **out);
void sl_multi_free(sl_multi *m);
int sl_multi_workspace_size(sl_multi *m, size_t *bytes_out);
int sl_multi_run(sl_multi *m, int what, const float *const *x_dev, void *const *coeffs_dev,
                 float *const *scales_dev, const float *const *sigma_dev, const float *K_host,
                 float *const *out_dev, void *workspace_dev, size_t workspace_bytes,
                 void *stream);
/* Times forward + inverse for each class over its schedule candidates and
 * keeps the fastest: chunk sizes of 32..2048 MiB that fit the class's
 * current workspace slot and, for 2D classes, the block shape of
 * sl_system_set_block_shape (one or two images per inverse-accumulation
 * block, pair-loop split on or off) and, for classes with 1024-point lines,
 * the line plan of sl_system_set_line_plan.  Cached by size, R, batch and
 * storage type in the text file cache_path, if given (one line per class:
 * key, chunk bytes, images per block, split, line plan).                    */
int sl_multi_autotune(sl_multi *m, const float *const *x_dev, void *const *coeffs_dev,
                      float *const *scales_dev, float *const *out_dev, void *workspace_dev,
                      size_t workspace_bytes, const char *cache_path, void *stream);
/* Schedule of a multi-batch: per_class = 0 (default) runs, where every class
 * supports it (2D, one storage type, row lengths with a wavefront-local line
 * plan; 1024-point classes need line plan 2), the multi-class schedule: each
 * class's spectrum and column passes, and for every step one coefficient
 * row launch whose flat work list holds the row blocks of all classes
 * (largest class first); otherwise, or with per_class = 1, each class runs
 * its own passes (as separate graph branches in sl_multi_graph_build).
 * sl_multi_autotune times both and keeps the faster.  sl_multi_schedule
 * reports whether the multi-class schedule is in use.                      */
int sl_multi_set_schedule(sl_multi *m, int per_class);
int sl_multi_schedule(sl_multi *m, int *multi_class_rows);
/* Captures one run (same arguments as sl_multi_run) into a HIP graph (one
 * branch per class in the per-class schedule, one sequence in the
 * multi-class schedule); sl_multi_graph_launch replays it on a stream.  The
 * buffers are baked into the graph.  Per-pass timing must be off.          */
int sl_multi_graph_build(sl_multi *m, int what, const float *const *x_dev,
                         void *const *coeffs_dev, float *const *scales_dev,
                         const float *const *sigma_dev, const float *K_host,
                         float *const *out_dev, void *workspace_dev, size_t workspace_bytes);
int sl_multi_graph_launch(sl_multi *m, void *stream);

/* ---- learned shrinkage (an extension beyond the paper) -------------------
 * A per-scale CNN maps each detail coefficient plane c (with the noise level
 * sigma of its image) to gains g in [0, 1]:
 *   x0 = (|c| / (sigma ||psi_i||_2), sigma * 255 / 50),
 *   g  = sigmoid(conv3(relu(conv2(relu(conv1(x0)))))),  3x3 convolutions
 *   with zero padding, 2 -> 32 -> 32 -> 1 channels; output g * c.
 * Parameters: params_dev [J][SL_CNN_PARAMS] float32, one blob per scale:
 *   W1[32][2][9] b1[32] W2[32][32][9] b2[32] W3[1][32][9] b3[1], weights
 *   indexed [out][in][3 dy + dx].  The matrix-core kernels read bfloat16
 *   operand copies built by sl_cnn_pack (call it after every update); they
 *   accumulate in float32.  Coefficients must be SL_F32; 2D systems only.    */
#define SL_CNN_PARAMS 10145
size_t sl_cnn_packed_bytes(int J);
int sl_cnn_pack(const float *params_dev, int J, void *packed_dev, void *stream);
/* Workspace bytes of sl_cnn_apply (training = 0) or sl_cnn_backward (1).     */
int sl_cnn_workspace_size(const sl_system *s, int batch, int training, size_t *bytes_out);
/* coeffs_out = g .* coeffs for every detail subband, lowpass copied;
 * gains_dev [B][R][dims] float32 (lowpass slot untouched) may be NULL.       */
int sl_cnn_apply(const sl_system *s, const float *params_dev, const void *packed_dev,
                 const float *coeffs_dev, const float *sigma_dev, int batch,
                 float *coeffs_out_dev, float *gains_dev, void *workspace_dev,
                 size_t workspace_bytes, void *stream);
/* Gradient of a loss with respect to params_dev, given dL/d(coeffs_out)
 * (dcoeffs_dev, [B][R][dims] float32) and the input coefficients:
 * grads_dev [J][SL_CNN_PARAMS] float32 (overwritten).  Recomputes the
 * forward pass; deterministic.                                              */
int sl_cnn_backward(const sl_system *s, const float *params_dev, const void *packed_dev,
                    const float *coeffs_dev, const float *sigma_dev, int batch,
                    const float *dcoeffs_dev, float *grads_dev, void *workspace_dev,
                    size_t workspace_bytes, void *stream);
/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8) on n
 * float32 parameters with moment buffers m_dev, v_dev; step counts from 1.   */
int sl_cnn_adam(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int n,
                float lr, int step, void *stream);
/* out = scale * (a - b) over n floats and loss_dev[0] = sum (a - b)^2 (a
 * fixed-order reduction): the gradient of a squared-error image loss.
 * loss_dev must hold SL_SQERR_SCRATCH floats (the rest is scratch).          */
#define SL_SQERR_SCRATCH 1025
int sl_sq_error_grad(const float *a_dev, const float *b_dev, size_t n, float scale,
                     float *out_dev, float *loss_dev, void *stream);

/* ---- training-data synthesis (not part of the paper's method) -----------
 * Renders n cartoon images [n][H][W] float32: shapes_dev is the packed shape
 * table [n][1 + max_shapes * 24] (background, then per shape: type 0/1/2,
 * value, ellipse cx cy a b cos sin | polygon count and up to 8 vertices),
 * painted in order with membership tested at pixel centres.  If noisy_dev
 * is not NULL it receives clean + sigma[n] * N(0,1) noise from a
 * counter-based generator keyed by (noise_seed, image, pixel).              */
int sl_render_cartoons(const float *shapes_dev, int n, int H, int W, int max_shapes,
                       const float *sigma_dev, uint64_t noise_seed, float *clean_dev,
                       float *noisy_dev, void *stream);

/* ---- diagnostics: per-pass device timing ---------------------------------
 * When enabled, every kernel launch of the transforms is bracketed by a pair
 * of HIP events recorded on the launch stream; sl_timing_query synchronises
 * those events and returns the summed elapsed time and the launch count of
 * one pass.  Passes are numbered 0..sl_timing_num_passes()-1 and named by
 * sl_timing_pass_name.  Process-wide state; not thread-safe.                */
int sl_timing_enable(int on);
int sl_timing_reset(void);
int sl_timing_num_passes(void);
const char *sl_timing_pass_name(int pass);
int sl_timing_query(int pass, double *total_ms_out, int *launches_out);

#ifdef __cplusplus
}
#endif

#endif /* SHEARLET_H_ */
