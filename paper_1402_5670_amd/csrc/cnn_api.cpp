// C ABI of the learned-shrinkage network (declared in include/shearlet.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

#include "../../include/shearlet.h"
#include "cnn.hpp"
#include "system.hpp"

namespace sl {
hipError_t render_cartoons(const float *shapes, int n, int H, int W, int max_shapes,
                           const float *sigma, uint64_t seed, float *clean, float *noisy,
                           hipStream_t st);
}

namespace {

using sl::kCnnParams;

constexpr size_t kPackLayer2 = 9 * 2 * 512;   // u16 per scale, two output blocks
constexpr size_t kPackLayer1 = 9 * 1 * 512;   // one output block
constexpr size_t kPackK1 = 2 * 512;             // layer 1, taps packed into K
constexpr size_t kPackTaps3 = 512;              // layer 3, taps on the M axis
constexpr int kWgradLen = 9 * 32 * 32 + 32;
constexpr int kWgradBlocks = 512;
constexpr int kErrBlocks = SL_SQERR_SCRATCH - 1;

size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct Packed {
  const uint16_t *w1, *w2, *w3, *w2t, *w3t, *w1k, *w3m;
};

Packed packed_view(const void *base, int J) {
  const uint16_t *p = (const uint16_t *)base;
  Packed v;
  v.w1 = p;
  v.w2 = v.w1 + J * kPackLayer2;
  v.w3 = v.w2 + J * kPackLayer2;
  v.w2t = v.w3 + J * kPackLayer1;
  v.w3t = v.w2t + J * kPackLayer2;
  v.w1k = v.w3t + J * kPackLayer2;
  v.w3m = v.w1k + J * kPackK1;
  return v;
}

sl::CnnPlanes planes(const sl_system *s, int B, const float *sigma) {
  sl::CnnPlanes pl{};
  pl.R = s->R;
  pl.J = s->cfg.J;
  pl.B = B;
  pl.p0 = 0;
  int acc = 0;
  for (int j = 0; j < pl.J; ++j) {
    int n = 0, first = -1;
    for (int i = 1; i < s->R; ++i)
      if (s->subs[i].j == j) {
        if (first < 0) first = i;
        ++n;
      }
    pl.start[j] = acc;
    pl.nsub[j] = n;
    pl.first[j] = first < 0 ? 1 : first;
    acc += B * n;
  }
  pl.start[pl.J] = acc;
  pl.sigma = sigma;
  pl.l2 = s->d_l2;
  return pl;
}

size_t act_bytes(const sl_system *s, int planes) {
  return al((size_t)planes * (size_t)s->cfg.npix() * 32 * 2);
}

// SL_CNN_LAYERWISE=1 selects the layer-by-layer inference (activations in
// HBM) instead of the fused tile kernel; both compute the same network.
bool layerwise() {
  const char *e = std::getenv("SL_CNN_LAYERWISE");
  return e && std::atoi(e) != 0;
}

int apply_chunk(const sl_system *s, int B) {
  const int P = B * (s->R - 1);
  const char *env = std::getenv("SL_CNN_CHUNK_MB");
  const size_t cap = (size_t)(env ? std::max(1, std::atoi(env)) : 4096) << 20;
  const size_t per = 2 * (size_t)s->cfg.npix() * 32 * 2;
  return (int)std::max<size_t>(1, std::min<size_t>((size_t)P, cap / per));
}

int check(const sl_system *s, int B, const void *a, const void *b) {
  if (!s) return sl::set_error(SL_EINVAL, "system is NULL");
  if (B < 1 || B > 65535) return sl::set_error(SL_EINVAL, "batch must be in 1..65535");
  if (!a || !b) return sl::set_error(SL_EINVAL, "NULL buffer");
  if (s->cfg.dtype != SL_F32) return sl::set_error(SL_EINVAL, "the CNN needs SL_F32 coefficients");
  if (s->cfg.J > sl::kMaxScales) return sl::set_error(SL_EUNSUPPORTED, "too many scales");
  if (s->R < 2) return sl::set_error(SL_EINVAL, "no detail subbands");
  if (s->cfg.ndim != 2) return sl::set_error(SL_EUNSUPPORTED, "the CNN works on 2D systems");
  return SL_OK;
}

void plane_hw(const sl_system *s, int &H, int &W) {
  H = (int)s->cfg.dims[0];
  W = (int)s->cfg.dims[1];
}

#define CK(expr)                                                  \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return sl::hip_error(e_, #expr);        \
  } while (0)

}  // namespace

extern "C" {

size_t sl_cnn_packed_bytes(int J) {
  // w1, w2, w2t, w3t: two output blocks each; w3: one; w1k: packed layer 1;
  // w3m: layer 3 with the taps as output rows
  if (J < 1) return 0;
  return (size_t)J * (4 * kPackLayer2 + kPackLayer1 + kPackK1 + kPackTaps3) * sizeof(uint16_t);
}

int sl_cnn_pack(const float *params_dev, int J, void *packed_dev, void *stream) {
  if (!params_dev || !packed_dev || J < 1 || J > sl::kMaxScales)
    return sl::set_error(SL_EINVAL, "bad arguments to sl_cnn_pack");
  hipStream_t st = (hipStream_t)stream;
  uint16_t *base = (uint16_t *)packed_dev;
  Packed v = packed_view(packed_dev, J);
  CK(sl::cnn_pack(params_dev, J, 1, 0, base, 2, st));
  CK(sl::cnn_pack(params_dev, J, 2, 0, (uint16_t *)v.w2, 2, st));
  CK(sl::cnn_pack(params_dev, J, 3, 0, (uint16_t *)v.w3, 1, st));
  CK(sl::cnn_pack(params_dev, J, 2, 1, (uint16_t *)v.w2t, 2, st));
  CK(sl::cnn_pack(params_dev, J, 3, 1, (uint16_t *)v.w3t, 2, st));
  CK(sl::cnn_pack(params_dev, J, 1, 2, (uint16_t *)v.w1k, 2, st));
  CK(sl::cnn_pack(params_dev, J, 3, 3, (uint16_t *)v.w3m, 1, st));
  return SL_OK;
}

int sl_cnn_workspace_size(const sl_system *s, int batch, int training, size_t *bytes_out) {
  if (!s || !bytes_out || batch < 1) return sl::set_error(SL_EINVAL, "bad arguments");
  const int P = batch * (s->R - 1);
  if (!training) {
    *bytes_out = layerwise() ? 2 * act_bytes(s, apply_chunk(s, batch)) : 256;
  } else {
    const int J = s->cfg.J;
    *bytes_out = 5 * act_bytes(s, P) + al((size_t)batch * s->R * s->cfg.npix() * 4) +
                 al((size_t)kWgradBlocks * kWgradLen * 4) + al((size_t)3 * J * kWgradLen * 4);
  }
  return SL_OK;
}

int sl_cnn_apply(const sl_system *s, const float *params_dev, const void *packed_dev,
                 const float *coeffs_dev, const float *sigma_dev, int batch,
                 float *coeffs_out_dev, float *gains_dev, void *workspace_dev,
                 size_t workspace_bytes, void *stream) {
  int rc = check(s, batch, coeffs_dev, coeffs_out_dev);
  if (rc) return rc;
  if (!params_dev || !packed_dev || !sigma_dev || !workspace_dev)
    return sl::set_error(SL_EINVAL, "NULL argument");
  size_t need = 0;
  sl_cnn_workspace_size(s, batch, 0, &need);
  if (workspace_bytes < need)
    return sl::set_error(SL_ENOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t st = (hipStream_t)stream;
  int H, W;
  plane_hw(s, H, W);
  const int J = s->cfg.J, P = batch * (s->R - 1), Pc = apply_chunk(s, batch);
  Packed pk = packed_view(packed_dev, J);
  sl::CnnPlanes pl0 = planes(s, batch, sigma_dev);
  if (!layerwise()) {
    CK(sl::cnn_copy_lowpass(coeffs_dev, coeffs_out_dev, batch, s->R, (int)s->cfg.npix(), st));
    CK(sl::cnn_fused(coeffs_dev, pl0, P, H, W, pk.w1k, pk.w2, pk.w3m, params_dev, coeffs_out_dev,
                     gains_dev, s->num_cu, st));
    return SL_OK;
  }
  uint16_t *A = (uint16_t *)workspace_dev;
  uint16_t *Bf = (uint16_t *)((char *)workspace_dev + act_bytes(s, Pc));
  sl::CnnPlanes pl = planes(s, batch, sigma_dev);
  CK(sl::cnn_copy_lowpass(coeffs_dev, coeffs_out_dev, batch, s->R, (int)s->cfg.npix(), st));
  for (int p0 = 0; p0 < P; p0 += Pc) {
    const int n = std::min(Pc, P - p0);
    pl.p0 = p0;
    CK(sl::cnn_x0(coeffs_dev, pl, n, H, W, A, st));
    CK(sl::cnn_conv(A, pk.w1, 2, params_dev + sl::kOffB1, kCnnParams, pl, n, H, W, sl::CONV_RELU,
                    Bf, nullptr, nullptr, nullptr, nullptr, st));
    CK(sl::cnn_conv(Bf, pk.w2, 2, params_dev + sl::kOffB2, kCnnParams, pl, n, H, W, sl::CONV_RELU,
                    A, nullptr, nullptr, nullptr, nullptr, st));
    CK(sl::cnn_conv(A, pk.w3, 1, params_dev + sl::kOffB3, kCnnParams, pl, n, H, W, sl::CONV_GAIN,
                    nullptr, nullptr, coeffs_dev, coeffs_out_dev, gains_dev, st));
  }
  return SL_OK;
}

int sl_cnn_backward(const sl_system *s, const float *params_dev, const void *packed_dev,
                    const float *coeffs_dev, const float *sigma_dev, int batch,
                    const float *dcoeffs_dev, float *grads_dev, void *workspace_dev,
                    size_t workspace_bytes, void *stream) {
  int rc = check(s, batch, coeffs_dev, dcoeffs_dev);
  if (rc) return rc;
  if (!params_dev || !packed_dev || !sigma_dev || !workspace_dev || !grads_dev)
    return sl::set_error(SL_EINVAL, "NULL argument");
  size_t need = 0;
  sl_cnn_workspace_size(s, batch, 1, &need);
  if (workspace_bytes < need)
    return sl::set_error(SL_ENOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t st = (hipStream_t)stream;
  int H, W;
  plane_hw(s, H, W);
  const int J = s->cfg.J, P = batch * (s->R - 1);
  Packed pk = packed_view(packed_dev, J);
  char *w = (char *)workspace_dev;
  const size_t ab = act_bytes(s, P);
  uint16_t *X0 = (uint16_t *)w;
  uint16_t *H1 = (uint16_t *)(w + ab);
  uint16_t *H2 = (uint16_t *)(w + 2 * ab);
  uint16_t *DZ = (uint16_t *)(w + 3 * ab);
  uint16_t *DA2 = (uint16_t *)(w + 4 * ab);
  float *G = (float *)(w + 5 * ab);
  float *part = (float *)(w + 5 * ab + al((size_t)batch * s->R * s->cfg.npix() * 4));
  float *dW = (float *)((char *)part + al((size_t)kWgradBlocks * kWgradLen * 4));
  sl::CnnPlanes pl = planes(s, batch, sigma_dev);
  // forward recompute
  CK(sl::cnn_x0(coeffs_dev, pl, P, H, W, X0, st));
  CK(sl::cnn_conv(X0, pk.w1, 2, params_dev + sl::kOffB1, kCnnParams, pl, P, H, W, sl::CONV_RELU,
                  H1, nullptr, nullptr, nullptr, nullptr, st));
  CK(sl::cnn_conv(H1, pk.w2, 2, params_dev + sl::kOffB2, kCnnParams, pl, P, H, W, sl::CONV_RELU,
                  H2, nullptr, nullptr, nullptr, nullptr, st));
  CK(sl::cnn_conv(H2, pk.w3, 1, params_dev + sl::kOffB3, kCnnParams, pl, P, H, W, sl::CONV_GAIN,
                  nullptr, nullptr, coeffs_dev, nullptr, G, st));
  // backward
  CK(sl::cnn_dz(dcoeffs_dev, coeffs_dev, G, pl, P, H, W, DZ, nullptr, st));
  CK(sl::cnn_conv(DZ, pk.w3t, 2, nullptr, 0, pl, P, H, W, sl::CONV_MASKED, DA2, H2, nullptr,
                  nullptr, nullptr, st));
  const int tiles_per_plane = ((W + 31) / 32) * ((H + 7) / 8);
  for (int j = 0; j < J; ++j)
    if (pl.start[j + 1] == pl.start[j]) return sl::set_error(SL_EINVAL, "a scale without planes");
  for (int j = 0; j < J; ++j) {
    const int a = pl.start[j], n = pl.start[j + 1] - pl.start[j];
    const int nb = std::min(kWgradBlocks, n * tiles_per_plane);
    CK(sl::cnn_wgrad(H2, DZ, H, W, a, n, nb, part, dW + (size_t)(3 * j + 2) * kWgradLen, 2, 1, st));
    CK(sl::cnn_wgrad(H1, DA2, H, W, a, n, nb, part, dW + (size_t)(3 * j + 1) * kWgradLen, 2, 2, st));
  }
  uint16_t *DA1 = DZ;
  CK(sl::cnn_conv(DA2, pk.w2t, 2, nullptr, 0, pl, P, H, W, sl::CONV_MASKED, DA1, H1, nullptr,
                  nullptr, nullptr, st));
  for (int j = 0; j < J; ++j) {
    const int a = pl.start[j], n = pl.start[j + 1] - pl.start[j];
    float *g1 = dW + (size_t)(3 * j) * kWgradLen;
    const int nb = std::min(kWgradBlocks, n * tiles_per_plane);
    CK(sl::cnn_wgrad(X0, DA1, H, W, a, n, nb, part, g1, 1, 2, st));
    CK(sl::cnn_grad_assemble(g1, dW + (size_t)(3 * j + 1) * kWgradLen,
                             dW + (size_t)(3 * j + 2) * kWgradLen, j, grads_dev, st));
  }
  return SL_OK;
}

int sl_cnn_adam(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int n,
                float lr, int step, void *stream) {
  if (!params_dev || !grads_dev || !m_dev || !v_dev || n < 1 || step < 1)
    return sl::set_error(SL_EINVAL, "bad arguments to sl_cnn_adam");
  CK(sl::cnn_adam(params_dev, grads_dev, m_dev, v_dev, n, lr, 0.9, 0.999, 1e-8, step,
                  (hipStream_t)stream));
  return SL_OK;
}

int sl_sq_error_grad(const float *a_dev, const float *b_dev, size_t n, float scale,
                     float *out_dev, float *loss_dev, void *stream) {
  if (!a_dev || !b_dev || !out_dev || !loss_dev || n == 0)
    return sl::set_error(SL_EINVAL, "bad arguments to sl_sq_error_grad");
  // loss_dev[1 .. SL_SQERR_SCRATCH) holds the per-block partial sums
  CK(sl::sq_error_grad(a_dev, b_dev, n, scale, out_dev, loss_dev + 1, kErrBlocks, loss_dev,
                       (hipStream_t)stream));
  return SL_OK;
}

int sl_render_cartoons(const float *shapes_dev, int n, int H, int W, int max_shapes,
                       const float *sigma_dev, uint64_t noise_seed, float *clean_dev,
                       float *noisy_dev, void *stream) {
  if (!shapes_dev || !clean_dev || n < 1 || n > 65535 || H < 1 || W < 1 || max_shapes < 0 ||
      (noisy_dev && !sigma_dev))
    return sl::set_error(SL_EINVAL, "bad arguments to sl_render_cartoons");
  CK(sl::render_cartoons(shapes_dev, n, H, W, max_shapes, sigma_dev, noise_seed, clean_dev,
                         noisy_dev, (hipStream_t)stream));
  return SL_OK;
}

}  // extern "C"
