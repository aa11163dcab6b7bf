// C ABI of libshearlet (declared in include/shearlet.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <map>
#include <string>
#include <vector>

#include "../../include/shearlet.h"
#include "dispatch.hpp"
#include "host_filters.hpp"
#include "inpaint.hpp"
#include "system.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return SL_EHIP;
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace

namespace sl {
size_t transform_workspace_bytes(const sl_system *s, int batch);
}


namespace {

template <class T>
int dev_upload(sl_system *s, const std::vector<T> &host, T **out) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(sizeof(T), host.size() * sizeof(T));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  s->allocs.push_back(p);
  if (!host.empty()) {
    e = hipMemcpy(p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  *out = (T *)p;
  return SL_OK;
}

// exp(-2 pi i m / N), m = 0..N-1, computed in FP64 and rounded to FP32
std::vector<float2> twiddles(int N) {
  std::vector<float2> t(N);
  for (int m = 0; m < N; ++m) {
    long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
    t[m].x = (float)(double)std::cos(a);
    t[m].y = (float)(double)std::sin(a);
  }
  return t;
}

void chunk_plan(const sl_system *s, int B, int &nb, int &np) {
  const int P = (s->R + 1) / 2;
  const size_t plane = 8ull * (size_t)s->cfg.npix();
  const size_t cap = s->chunk_cap;
  if ((size_t)B * P * plane <= cap) {
    nb = B;
    np = P;
  } else if ((size_t)B * plane <= cap) {
    nb = B;
    np = (int)std::max<size_t>(1, cap / ((size_t)B * plane));
  } else {
    nb = (int)std::max<size_t>(1, cap / plane);
    np = 1;
  }
  // grid limits: chunk images * pairs (times the depth in 3D) index grid.y
  const int depth = s->cfg.ndim == 3 ? (int)s->cfg.dims[0] : 1;
  while ((int64_t)nb * np * depth > 65535) {
    if (np > 1) np = (np + 1) / 2;
    else nb = (nb + 1) / 2;
  }
}

// Workspace: spectrum F (also the inverse's accumulator) [B] complex planes,
// a second accumulator [B] used by sl_denoise_fused (F must survive every
// chunk there), the chunk of pair planes, per-image max |x|.
// Partial sums of the 2D inverse accumulation when its pair loop is split
// into groups (small batches): [groups - 1][B] complex planes.
struct Layout {
  size_t off_F, off_acc, off_chunk, off_xmax, off_part, total;
};

int inv_groups(const sl_system *s, int B);

Layout layout(const sl_system *s, int B) {
  int nb, np;
  chunk_plan(s, B, nb, np);
  const size_t plane = 8ull * (size_t)s->cfg.npix();
  Layout L;
  L.off_F = 0;
  L.off_acc = align_up(plane * B);
  L.off_chunk = align_up(L.off_acc + plane * B);
  L.off_xmax = align_up(L.off_chunk + plane * (size_t)nb * np);
  L.off_part = align_up(L.off_xmax + 4ull * B);
  L.total = align_up(L.off_part + plane * B * (size_t)(inv_groups(s, B) - 1));
  return L;
}

// A 2D view of the system for the line kernels: H lines of length W.  In 3D
// the row view is (D*H) x W, the y view H x W per z-slice and the z view
// D x (H*W) per volume.
sl::Sys2D view2d(const sl_system *s, int H, int W, int nH, int nW) {
  sl::Sys2D v;
  v.H = H;
  v.W = W;
  v.R = s->R;
  v.dtype = s->cfg.dtype;
  v.filt = s->d_filt;
  v.psi = s->d_psi;
  v.l1 = s->d_l1;
  v.num_cu = s->num_cu;
  v.inv_images = s->inv_images;
  v.split_pairs = s->split_pairs;
  v.line_em = s->line_em;
  v.twH = nH ? s->d_tw.at(nH) : nullptr;
  v.twW = nW ? s->d_tw.at(nW) : nullptr;
  return v;
}

sl::Sys2D view2d(const sl_system *s) {
  int H = (int)s->cfg.dims[0], W = (int)s->cfg.dims[1];
  return view2d(s, H, W, H, W);
}

// The XCD-cooperative passes replace the line passes of a 2D forward or
// inverse when the device and shape support them and the chunk region of the
// workspace can hold their scratch planes.
bool use_xcd(const sl_system *s, int B, const Layout &L) {
  if (!s->xcd || s->cfg.ndim != 2 || !s->xcd_err_dev) return false;
  if (L.off_xmax - L.off_chunk < sl::xcd_scratch_bytes()) return false;
  return sl::xcd_supported(view2d(s), B);
}

int inv_groups(const sl_system *s, int B) {
  if (s->cfg.ndim != 2) return 1;
  int nb, np;
  chunk_plan(s, B, nb, np);
  return sl::inv_pair_groups(view2d(s), nb, np);
}

sl::Sys3D view3d(const sl_system *s) {
  sl::Sys3D v;
  v.D = (int)s->cfg.dims[0];
  v.H = (int)s->cfg.dims[1];
  v.W = (int)s->cfg.dims[2];
  v.R = s->R;
  v.dtype = s->cfg.dtype;
  v.num_cu = s->num_cu;
  v.pairs = s->d_zpairs;
  v.tab = s->d_ztab;
  v.psi = s->d_psi;
  v.twD = s->d_tw.at(v.D);
  return v;
}

int check_call(const sl_system *s, int batch, const void *a, const void *b, void *ws,
               size_t ws_bytes) {
  if (!s) return fail(SL_EINVAL, "system is NULL");
  if (batch < 1 || batch > 65535) return fail(SL_EINVAL, "batch must be in 1..65535");
  if (!a || !b || !ws) return fail(SL_EINVAL, "NULL buffer");
  if ((uintptr_t)ws & 15u) return fail(SL_EINVAL, "the workspace must be 16-byte aligned");
  size_t need = layout(s, batch).total;
  if (ws_bytes < need)
    return fail(SL_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->device)
    return fail(SL_EINVAL, "the current HIP device is not the system's device");
  if (s->xcd_err_host && *(volatile int *)s->xcd_err_host) {
    *(volatile int *)s->xcd_err_host = 0;
    return fail(SL_EHIP,
                "an XCD-cooperative pass of an earlier call gave up waiting for its workgroups; "
                "the results of that call are invalid");
  }
  return SL_OK;
}

#define SL_TRY(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

// ---- per-pass event timing ----------------------------------------------
enum Pass {
  P_ROWS_REAL_FFT = 0,
  P_COLS_FFT,
  P_COLS_FILTER_IFFT,
  P_ROWS_COEF,
  P_ROWS_COEF_FFT,
  P_COLS_FFT_ACC,
  P_ROWS_REAL_IFFT,
  P_AUX,
  P_ROWS_THR,
  P_XCD_FWD,
  P_XCD_INV,
  P_COUNT
};
const char *kPassNames[P_COUNT] = {"rows_real_fft",   "cols_fft",      "cols_filter_ifft",
                                   "rows_coef",       "rows_coef_fft", "cols_fft_acc",
                                   "rows_real_ifft",  "aux",           "rows_thr",
                                   "xcd_fwd",         "xcd_inv"};

struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[P_COUNT];
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void recycle() {
    for (auto &v : ev)
      for (auto &p : v) {
        pool.push_back(p.first);
        pool.push_back(p.second);
      }
    for (auto &v : ev) v.clear();
  }
} g_timing;

// set while a call captures a graph: no timing events go into it
thread_local bool g_capturing = false;

template <class F>
hipError_t timed(int pass, hipStream_t st, F &&launch) {
  if (!g_timing.on || g_capturing) return launch();
  hipEvent_t a = g_timing.get(), b = g_timing.get();
  (void)hipEventRecord(a, st);
  hipError_t e = launch();
  (void)hipEventRecord(b, st);
  g_timing.ev[pass].push_back({a, b});
  return e;
}

#define SL_LAUNCH(pass, st, expr) SL_TRY(timed(pass, st, [&]() { return (expr); }))

int forward3d(const sl_system *s, const float *x, int batch, void *coef, float *scales,
              float2 *F, float2 *T, unsigned *xmax, bool dual, hipStream_t st) {
  const int D = (int)s->cfg.dims[0], H = (int)s->cfg.dims[1], W = (int)s->cfg.dims[2];
  const bool scaled = s->cfg.dtype != SL_F32;
  const sl::Sys2D vr = view2d(s, D * H, W, 0, W);       // x lines
  const sl::Sys2D vy = view2d(s, H, W, H, 0);           // y lines per z-slice
  const sl::Sys2D vz = view2d(s, D, H * W, D, 0);       // z lines per volume
  const sl::Sys2D vp = view2d(s, H, W, H, W);           // z-slices in LDS
  const bool plane = s->plane3d && sl::plane_supported(H, W);
  const bool half = s->plane3d && !plane && sl::half_plane_supported(H, W);
  const float inv_vol = 1.0f / ((float)(D * H) * (float)W);
  const sl::Sys3D v3 = view3d(s);
  if (scaled) SL_LAUNCH(P_AUX, st, sl::launch_zero_u32(xmax, batch, st));
  SL_LAUNCH(P_ROWS_REAL_FFT, st, sl::launch_rows_real_fft(vr, x, F, scaled ? xmax : nullptr, batch, st));
  SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, F, F, batch * D, false, st));
  // the z pass takes the DFT along z itself, unless F must be divided by
  // Psi_hat first (the adjoint)
  const bool zdft = !dual;
  if (!zdft) SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vz, F, F, batch, false, st));
  if (dual) SL_LAUNCH(P_AUX, st, sl::launch_div_psi(F, s->d_psi, (size_t)s->cfg.npix(), batch, st));
  if (scaled) SL_LAUNCH(P_AUX, st, sl::launch_scales(vr, xmax, scales, batch, st));
  int nb, np;
  chunk_plan(s, batch, nb, np);
  const int P = (s->R + 1) / 2;
  for (int b0 = 0; b0 < batch; b0 += nb)
    for (int p0 = 0; p0 < P; p0 += np) {
      sl::Chunk c{b0, std::min(nb, batch - b0), p0, std::min(np, P - p0)};
      SL_LAUNCH(P_COLS_FILTER_IFFT, st, sl::launch_z_filter_ifft(v3, F, T, c, zdft, st));
      if (plane) {
        SL_LAUNCH(P_ROWS_COEF, st, sl::launch_plane_coef(vp, D, T, coef, scales, c, inv_vol, st));
      } else if (half) {
        SL_LAUNCH(P_ROWS_COEF, st, sl::launch_hplane_coef(vp, D, T, coef, scales, c, inv_vol, st));
      } else {
        SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, T, T, c.nb * c.np * D, true, st, true));
        SL_LAUNCH(P_ROWS_COEF, st, sl::launch_rows_coef(vr, T, coef, scales, c, st));
      }
    }
  return SL_OK;
}

int inverse3d(const sl_system *s, const void *coef, const float *scales, int batch,
              const sl::ThrArgs &thr, float *x, float2 *ACC, float2 *U, hipStream_t st) {
  const int D = (int)s->cfg.dims[0], H = (int)s->cfg.dims[1], W = (int)s->cfg.dims[2];
  const sl::Sys2D vr = view2d(s, D * H, W, 0, W);
  const sl::Sys2D vy = view2d(s, H, W, H, 0);
  const sl::Sys2D vp = view2d(s, H, W, H, W);
  const bool plane = s->plane3d && sl::plane_supported(H, W);
  const bool half = s->plane3d && !plane && sl::half_plane_supported(H, W);
  const sl::Sys3D v3 = view3d(s);
  int nb, np;
  chunk_plan(s, batch, nb, np);
  const int P = (s->R + 1) / 2;
  for (int b0 = 0; b0 < batch; b0 += nb)
    for (int p0 = 0; p0 < P; p0 += np) {
      sl::Chunk c{b0, std::min(nb, batch - b0), p0, std::min(np, P - p0)};
      if (plane) {
        SL_LAUNCH(P_ROWS_COEF_FFT, st, sl::launch_plane_coef_fft(vp, D, coef, scales, U, c, thr, st));
      } else if (half) {
        SL_LAUNCH(P_ROWS_COEF_FFT, st, sl::launch_hplane_coef_fft(vp, D, coef, scales, U, c, thr, st));
      } else {
        SL_LAUNCH(P_ROWS_COEF_FFT, st, sl::launch_rows_coef_fft(vr, coef, scales, U, c, thr, st));
        SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, U, U, c.nb * c.np * D, false, st, true));
      }
      SL_LAUNCH(P_COLS_FFT_ACC, st,
                sl::launch_z_fft_acc(v3, U, ACC, c, p0 == 0, p0 + c.np == P, st));
    }
  SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, ACC, ACC, batch * D, true, st));
  SL_LAUNCH(P_ROWS_REAL_IFFT, st, sl::launch_rows_real_ifft(vr, ACC, x, batch, st));
  return SL_OK;
}


// Forward transform, hard threshold and inverse transform without
// materialising the coefficients (the body of sl_denoise_fused and of every
// inpainting iteration).  Arguments are validated by the callers.
int denoise_fused_run(const sl_system *s, const float *x_dev, int batch, const sl::ThrArgs &thr,
                      float *out_dev, char *ws, hipStream_t st, const sl::MixArgs *mix = nullptr) {
  const Layout L = layout(s, batch);
  float2 *F = (float2 *)(ws + L.off_F);
  float2 *ACC = (float2 *)(ws + L.off_acc);
  float2 *T = (float2 *)(ws + L.off_chunk);
  const float inv_n = 1.0f / (float)s->cfg.npix();
  int nb, np;
  chunk_plan(s, batch, nb, np);
  const int P = (s->R + 1) / 2;
  if (s->cfg.ndim == 3) {
    const int D = (int)s->cfg.dims[0], H = (int)s->cfg.dims[1], W = (int)s->cfg.dims[2];
    const sl::Sys2D vr = view2d(s, D * H, W, 0, W);
    const sl::Sys2D vy = view2d(s, H, W, H, 0);
    const sl::Sys2D vp = view2d(s, H, W, H, W);
    const bool plane = s->plane3d && sl::plane_supported(H, W);
    const sl::Sys3D v3 = view3d(s);
    if (mix)
      SL_LAUNCH(P_ROWS_REAL_FFT, st, sl::launch_rows_real_fft_mix(vr, *mix, F, batch, st));
    else
      SL_LAUNCH(P_ROWS_REAL_FFT, st, sl::launch_rows_real_fft(vr, x_dev, F, nullptr, batch, st));
    SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, F, F, batch * D, false, st));
    for (int b0 = 0; b0 < batch; b0 += nb)
      for (int p0 = 0; p0 < P; p0 += np) {
        sl::Chunk c{b0, std::min(nb, batch - b0), p0, std::min(np, P - p0)};
        SL_LAUNCH(P_COLS_FILTER_IFFT, st, sl::launch_z_filter_ifft(v3, F, T, c, true, st));
        if (plane) {
          SL_LAUNCH(P_ROWS_THR, st, sl::launch_plane_thr(vp, D, T, inv_n, c, thr, st));
        } else {
          SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, T, T, c.nb * c.np * D, true, st, true));
          SL_LAUNCH(P_ROWS_THR, st, sl::launch_rows_thr(vr, T, inv_n, c, thr, st));
          SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, T, T, c.nb * c.np * D, false, st, true));
        }
        SL_LAUNCH(P_COLS_FFT_ACC, st,
                  sl::launch_z_fft_acc(v3, T, ACC, c, p0 == 0, p0 + c.np == P, st));
      }
    SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(vy, ACC, ACC, batch * D, true, st));
    SL_LAUNCH(P_ROWS_REAL_IFFT, st, sl::launch_rows_real_ifft(vr, ACC, out_dev, batch, st));
    return SL_OK;
  }
  const sl::Sys2D v = view2d(s);
  const int G = inv_groups(s, batch);
  float2 *part = (float2 *)(ws + L.off_part);
  if (mix)
    SL_LAUNCH(P_ROWS_REAL_FFT, st, sl::launch_rows_real_fft_mix(v, *mix, F, batch, st));
  else
    SL_LAUNCH(P_ROWS_REAL_FFT, st, sl::launch_rows_real_fft(v, x_dev, F, nullptr, batch, st));
  SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(v, F, F, batch, false, st));
  for (int b0 = 0; b0 < batch; b0 += nb)
    for (int p0 = 0; p0 < P; p0 += np) {
      sl::Chunk c{b0, std::min(nb, batch - b0), p0, std::min(np, P - p0)};
      SL_LAUNCH(P_COLS_FILTER_IFFT, st, sl::launch_cols_filter_ifft(v, F, T, c, st));
      SL_LAUNCH(P_ROWS_THR, st, sl::launch_rows_thr(v, T, inv_n, c, thr, st));
      SL_LAUNCH(P_COLS_FFT_ACC, st,
                sl::launch_cols_fft_acc(v, T, ACC, part, G, batch, c, p0 == 0, p0 + c.np == P, st));
    }
  if (G > 1) SL_LAUNCH(P_COLS_FFT_ACC, st, sl::launch_cols_acc_finish(v, ACC, part, G, batch, st));
  SL_LAUNCH(P_ROWS_REAL_IFFT, st, sl::launch_rows_real_ifft(v, ACC, out_dev, batch, st));
  return SL_OK;
}

// Inpainting workspace: the transform's, then sigma [B] float32 (the
// iteration's threshold scale).  The iteration's input is formed while the
// forward row pass loads it and is not stored.
struct InpaintLayout {
  size_t base, off_sigma, total;
};

InpaintLayout inpaint_layout(const sl_system *s, int B) {
  InpaintLayout L;
  L.base = layout(s, B).total;
  L.off_sigma = L.base;
  L.total = align_up(L.off_sigma + 4ull * B);
  return L;
}

struct InpaintArgs {
  const float *fm;
  const uint8_t *mask;
  int batch;
  const float *delta_init;
  double delta_min;
  int iterations, t_begin, t_end;
  float *f;
  char *ws;
};

// threshold factor of iteration t: lambda^t, lambda = delta_min^(1/(iterations-1))
float schedule_factor(double delta_min, int iterations, int t) {
  if (iterations <= 1 || t == 0) return 1.0f;
  const double lam = std::pow(delta_min, 1.0 / (double)(iterations - 1));
  return (float)std::pow(lam, (double)t);
}

int inpaint_launches(const sl_system *s, const InpaintArgs &a, hipStream_t st) {
  const InpaintLayout L = inpaint_layout(s, a.batch);
  float *sigma = (float *)(a.ws + L.off_sigma);
  sl::ThrArgs thr{};
  thr.sigma = sigma;
  thr.l2 = s->d_l2;
  thr.jof = s->d_jof;
  for (int j = 0; j < s->cfg.J; ++j) thr.K[j] = 1.0f;
  for (int t = a.t_begin; t < a.t_end; ++t) {
    // g = M f_masked + (1 - M) f, formed by the forward row pass
    const sl::MixArgs mix{a.fm, a.mask, a.f, t == 0 ? 1 : 0, a.delta_init,
                          schedule_factor(a.delta_min, a.iterations, t), sigma};
    int rc = denoise_fused_run(s, nullptr, a.batch, thr, a.f, a.ws, st, &mix);
    if (rc) return rc;
  }
  return SL_OK;
}


// Run `launches` on st directly, or (use_graph) replay the graph cached on
// `owner` under `key`, capturing and instantiating it on the first call.
int run_or_replay(const sl_system *owner, const std::vector<uint64_t> &key, bool use_graph,
                  hipStream_t st, const std::function<int(hipStream_t)> &launches) {
  if (!use_graph) return launches(st);
  auto *ms = const_cast<sl_system *>(owner);
  std::lock_guard<std::mutex> lock(ms->graph_mu);
  for (auto &gr : ms->graphs)
    if (gr.key == key) {
      SL_TRY(hipGraphLaunch(gr.exec, st));
      return SL_OK;
    }
  // capture on a private stream, instantiate, keep
  hipStream_t cs = nullptr;
  SL_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  g_capturing = true;
  int rc = launches(cs);
  g_capturing = false;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : hip_fail(e, "hipStreamEndCapture");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "hipGraphInstantiate");
  }
  if (ms->graphs.size() >= 4) {
    (void)hipGraphExecDestroy(ms->graphs.front().exec);
    (void)hipGraphDestroy(ms->graphs.front().graph);
    ms->graphs.erase(ms->graphs.begin());
  }
  ms->graphs.push_back({key, graph, exec});
  SL_TRY(hipGraphLaunch(exec, st));
  return SL_OK;
}

// Decomposition workspace: the larger of the two systems' transform
// workspaces (they run one after the other), then g0 and g1 [B][npix]
// float32 and sigma [B].
struct DecompLayout {
  size_t off_g0, off_g1, off_sigma, total;
};

DecompLayout decomp_layout(const sl_system *s0, const sl_system *s1, int B) {
  DecompLayout L;
  const size_t plane = 4ull * (size_t)s0->cfg.npix() * B;
  L.off_g0 = std::max(layout(s0, B).total, layout(s1, B).total);
  L.off_g1 = align_up(L.off_g0 + plane);
  L.off_sigma = align_up(L.off_g1 + plane);
  L.total = align_up(L.off_sigma + 4ull * B);
  return L;
}

sl::ThrArgs unit_thresholds(const sl_system *s, const float *sigma) {
  sl::ThrArgs thr{};
  thr.sigma = sigma;
  thr.l2 = s->d_l2;
  thr.jof = s->d_jof;
  for (int j = 0; j < s->cfg.J; ++j) thr.K[j] = 1.0f;
  return thr;
}

uint64_t bits_of(double v) {
  uint64_t b;
  std::memcpy(&b, &v, sizeof(b));
  return b;
}

}  // namespace

bool sl::multi2d_supported(const MultiClass2D *cls, int n) {
  if (n < 1 || n > kMaxMultiClasses) return false;
  for (int i = 0; i < n; ++i) {
    const sl_system *s = cls[i].s;
    if (!s || s->cfg.ndim != 2 || s->cfg.dtype != cls[0].s->cfg.dtype) return false;
    if (!sl::multi_rows_supported(view2d(s))) return false;
  }
  return true;
}

int sl::run_multi2d(const MultiClass2D *cls, int n, int what, const float *K, hipStream_t st) {
  if (!multi2d_supported(cls, n)) return fail(SL_EUNSUPPORTED, "classes not supported by run_multi2d");
  std::vector<std::vector<sl::Chunk>> chunks(n);
  size_t steps = 0;
  for (int i = 0; i < n; ++i) {
    const MultiClass2D &c = cls[i];
    int rc = check_call(c.s, c.B, c.x ? (const void *)c.x : c.coef, c.coef, c.ws, c.ws_bytes);
    if (rc) return rc;
    int nb, np;
    chunk_plan(c.s, c.B, nb, np);
    const int P = (c.s->R + 1) / 2;
    for (int b0 = 0; b0 < c.B; b0 += nb)
      for (int p0 = 0; p0 < P; p0 += np)
        chunks[i].push_back({b0, std::min(nb, c.B - b0), p0, std::min(np, P - p0)});
    steps = std::max(steps, chunks[i].size());
  }
  const int dtype = cls[0].s->cfg.dtype;
  if (what & 1) {
    // per class: row DFT of the images, column DFT, storage scales
    for (int i = 0; i < n; ++i) {
      const MultiClass2D &c = cls[i];
      const Layout L = layout(c.s, c.B);
      char *ws = (char *)c.ws;
      float2 *F = (float2 *)(ws + L.off_F);
      unsigned *xmax = (unsigned *)(ws + L.off_xmax);
      const sl::Sys2D v = view2d(c.s);
      const bool scaled = dtype != SL_F32;
      if (scaled && !c.scales) return fail(SL_EINVAL, "scales are required for F16/BF16 storage");
      if (scaled) SL_LAUNCH(P_AUX, st, sl::launch_zero_u32(xmax, c.B, st));
      SL_LAUNCH(P_ROWS_REAL_FFT, st,
                sl::launch_rows_real_fft(v, c.x, F, scaled ? xmax : nullptr, c.B, st));
      SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(v, F, F, c.B, false, st));
      if (scaled) SL_LAUNCH(P_AUX, st, sl::launch_scales(v, xmax, c.scales, c.B, st));
    }
    for (size_t k = 0; k < steps; ++k) {
      sl::MultiRows mr{};
      for (int i = 0; i < n; ++i) {
        if (k >= chunks[i].size()) continue;
        const MultiClass2D &c = cls[i];
        const Layout L = layout(c.s, c.B);
        char *ws = (char *)c.ws;
        const sl::Sys2D v = view2d(c.s);
        float2 *F = (float2 *)(ws + L.off_F), *T = (float2 *)(ws + L.off_chunk);
        SL_LAUNCH(P_COLS_FILTER_IFFT, st, sl::launch_cols_filter_ifft(v, F, T, chunks[i][k], st));
        sl::MultiRowClass &mc = mr.c[mr.n++];
        sl::multi_rows_class_geometry(v, chunks[i][k], mc);
        mc.T = T;
        mc.coef = c.coef;
        mc.scales = c.scales;
      }
      SL_LAUNCH(P_ROWS_COEF, st, sl::launch_rows_multi(mr, dtype, true, st));
    }
  }
  if (what & 2) {
    std::vector<int> groups(n);
    for (int i = 0; i < n; ++i) groups[i] = inv_groups(cls[i].s, cls[i].B);
    for (size_t k = 0; k < steps; ++k) {
      sl::MultiRows mr{};
      for (int i = 0; i < n; ++i) {
        if (k >= chunks[i].size()) continue;
        const MultiClass2D &c = cls[i];
        const Layout L = layout(c.s, c.B);
        const sl::Sys2D v = view2d(c.s);
        sl::MultiRowClass &mc = mr.c[mr.n++];
        sl::multi_rows_class_geometry(v, chunks[i][k], mc);
        mc.U = (float2 *)((char *)c.ws + L.off_chunk);
        mc.coef = c.coef;
        mc.scales = c.scales;
        mc.thr.sigma = c.sigma;
        mc.thr.l2 = c.s->d_l2;
        mc.thr.jof = c.s->d_jof;
        if (c.sigma) {
          if (!K) return fail(SL_EINVAL, "K is required with sigma");
          if (c.s->cfg.J > sl::kMaxScales) return fail(SL_EUNSUPPORTED, "too many scales");
          for (int j = 0; j < c.s->cfg.J; ++j) mc.thr.K[j] = K[j];
        }
      }
      SL_LAUNCH(P_ROWS_COEF_FFT, st, sl::launch_rows_multi(mr, dtype, false, st));
      for (int i = 0; i < n; ++i) {
        if (k >= chunks[i].size()) continue;
        const MultiClass2D &c = cls[i];
        const Layout L = layout(c.s, c.B);
        char *ws = (char *)c.ws;
        const sl::Sys2D v = view2d(c.s);
        const sl::Chunk &ch = chunks[i][k];
        const int P = (c.s->R + 1) / 2;
        SL_LAUNCH(P_COLS_FFT_ACC, st,
                  sl::launch_cols_fft_acc(v, (float2 *)(ws + L.off_chunk), (float2 *)(ws + L.off_F),
                                          (float2 *)(ws + L.off_part), groups[i], c.B, ch,
                                          ch.p0 == 0, ch.p0 + ch.np == P, st));
      }
    }
    for (int i = 0; i < n; ++i) {
      const MultiClass2D &c = cls[i];
      const Layout L = layout(c.s, c.B);
      char *ws = (char *)c.ws;
      const sl::Sys2D v = view2d(c.s);
      float2 *ACC = (float2 *)(ws + L.off_F);
      if (groups[i] > 1)
        SL_LAUNCH(P_COLS_FFT_ACC, st,
                  sl::launch_cols_acc_finish(v, ACC, (float2 *)(ws + L.off_part), groups[i], c.B, st));
      SL_LAUNCH(P_ROWS_REAL_IFFT, st, sl::launch_rows_real_ifft(v, ACC, c.out, c.B, st));
    }
  }
  return SL_OK;
}

int sl::set_error(int code, const std::string &msg) { return fail(code, msg); }
bool sl::set_capturing(bool on) {
  const bool was = g_capturing;
  g_capturing = on;
  return was;
}
int sl::hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }

size_t sl::transform_workspace_bytes(const sl_system *s, int batch) {
  return layout(s, batch).total;
}

extern "C" {

int sl_abi_version(void) { return 2; }

const char *sl_last_error(void) { return g_err.c_str(); }

int sl_config_num_subbands(const sl_config *cfg, int *R_out) {
  slh::Config c;
  std::string err;
  int rc = slh::parse_config(cfg, c, err);
  if (rc != SL_OK) return fail(rc, err);
  if (!R_out) return fail(SL_EINVAL, "R_out is NULL");
  *R_out = (int)slh::enumerate_subbands(c).size();
  return SL_OK;
}

int sl_build_filters_host(const sl_config *cfg, double *filters_host, double *dual_host,
                          sl_subband *subbands_host) {
  slh::Config c;
  std::string err;
  int rc = slh::parse_config(cfg, c, err);
  if (rc != SL_OK) return fail(rc, err);
  slh::Bank bank;
  rc = slh::build_bank(c, bank, filters_host, err);
  if (dual_host) std::copy(bank.dual.begin(), bank.dual.end(), dual_host);
  if (subbands_host)
    for (size_t i = 0; i < bank.subbands.size(); ++i) {
      const auto &s = bank.subbands[i];
      subbands_host[i] = {s.cone, s.j, s.k1, s.k2, bank.l2[i], bank.l1[i]};
    }
  if (rc != SL_OK) return fail(rc, err);
  return SL_OK;
}

}  // extern "C"

namespace {

// The wavelet bank reads dims, n_scales, the QMF and the storage type of a
// configuration; its shear levels and fan filter do not apply.
int parse_wavelet_config(const sl_config *cfg, slh::Config &c, std::string &err) {
  if (!cfg) {
    err = "cfg is NULL";
    return SL_EINVAL;
  }
  if (cfg->ndim != 2) {
    err = "the wavelet bank is two-dimensional";
    return SL_EINVAL;
  }
  sl_config w = *cfg;
  std::vector<int> zeros(std::max(1, cfg->n_scales), 0);
  w.shear_levels = zeros.data();
  w.dir_filter = nullptr;
  w.dir_rows = w.dir_cols = 0;
  w.full_system = 0;
  return slh::parse_config(&w, c, err);
}

int build_system_impl(const sl_config *cfg, bool wavelet, sl_system **out) {
  if (!out) return fail(SL_EINVAL, "out is NULL");
  *out = nullptr;
  static std::atomic<uint64_t> next_serial{1};
  auto *s = new sl_system();
  s->serial = next_serial++;
  std::string err;
  int rc = wavelet ? parse_wavelet_config(cfg, s->cfg, err) : slh::parse_config(cfg, s->cfg, err);
  if (rc != SL_OK) {
    delete s;
    return fail(rc, err);
  }
  const int64_t npix = s->cfg.npix();
  const bool is3d = s->cfg.ndim == 3;
  const int R = wavelet ? 3 * s->cfg.J + 1 : (int)slh::enumerate_subbands(s->cfg).size();
  std::vector<double> filt64(is3d ? 0 : (size_t)R * npix);
  slh::Bank bank;
  rc = wavelet ? slh::build_wavelet_bank(s->cfg, bank, filt64.data(), err)
               : slh::build_bank(s->cfg, bank, is3d ? nullptr : filt64.data(), err);
  if (rc != SL_OK) {
    delete s;
    return fail(rc, err);
  }
  s->subs = bank.subbands;
  s->R = R;
  s->wavelet = wavelet;
  s->l2 = bank.l2;
  s->l1 = bank.l1;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(SL_EHIP, "no HIP device");
  }
  if (hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount, s->device) !=
          hipSuccess ||
      s->num_cu < 1)
    s->num_cu = 1;
  const char *cap_env = std::getenv("SL_CHUNK_MB");
  // default 2 GiB: on MI355X larger chunks (fewer launches, no repeated
  // accumulator round trips) measured faster than Infinity-Cache-sized ones
  s->chunk_cap = (size_t)(cap_env ? std::max(1, std::atoi(cap_env)) : 2048) << 20;
  // volumes: y and x passes of a z-slice in LDS where the slice fits
  // ($SL_PLANE3D=0 keeps the separate line passes)
  const char *plane_env = std::getenv("SL_PLANE3D");
  s->plane3d = plane_env ? std::atoi(plane_env) != 0 : true;
  std::vector<float> f32(filt64.size());
  for (size_t i = 0; i < f32.size(); ++i) f32[i] = (float)filt64[i];
  std::vector<float> psi32(bank.dual.size());
  for (size_t i = 0; i < psi32.size(); ++i) psi32[i] = (float)bank.dual[i];
  std::vector<float> l2f(R), l1f(R);
  std::vector<int> jof(R);
  for (int i = 0; i < R; ++i) {
    l2f[i] = (float)bank.l2[i];
    // the FP16 scale needs an upper bound: round the l1 norm up
    l1f[i] = std::nextafter((float)bank.l1[i], INFINITY);
    jof[i] = bank.subbands[i].cone == 0 ? -1 : bank.subbands[i].j;
  }
  if ((!is3d && (rc = dev_upload(s, f32, &s->d_filt))) || (rc = dev_upload(s, psi32, &s->d_psi)) ||
      (rc = dev_upload(s, l2f, &s->d_l2)) || (rc = dev_upload(s, l1f, &s->d_l1)) ||
      (rc = dev_upload(s, jof, &s->d_jof))) {
    sl_free_system(s);
    return rc;
  }
  if (is3d) {
    // Per pair of subbands (a, b = a + 1), the filters along the z lines as
    // float2 (value for a, value for b) tables, so that a z line reads both
    // filters of its pair with one load per voxel and factor (Section 3.3.2:
    // every 3D filter is a product of factors along the pyramid's main axis
    // and along each secondary axis).  psi_i(z, y, x) = C_i(y, x) X_i(z, x) Y_i(z, y):
    //   lowpass   C = h(x) h(y),            Y = h(z)   (the same for every y)
    //   main x    C = g(x) Phi_k1(x, y),     X = Phi_k2(x, z)
    //   main y    C = g(y) Phi_k1(y, x),     Y = Phi_k2(y, z)
    //   main z    C = 1,   X = Phi_k1(z, x), Y = g(z) Phi_k2(z, y)
    // A factor a subband lacks is 1; the missing partner of an odd R has C = 0.
    // Every pair has a C block [H][W], and X [D][W] and Y [D][H] blocks when
    // one of its subbands has that factor.  A block interleaves two factors;
    // the same two factors recur in many pairs (consecutive subbands share k1,
    // and a pair's (k2, k2 + 1) recurs for every k1), so each distinct
    // combination is stored once and pairs point to it: neighbouring pairs then
    // find most of their blocks in L2 instead of streaming a fresh block from
    // HBM per pair.  Products are formed in FP64 and rounded once.
    slh::Tables3D t;
    slh::build_tables_3d(s->cfg, t);
    const int D = s->cfg.n(3), H = s->cfg.n(2), W = s->cfg.n(1);
    // factor of one subband in one role: kind 0 = 1, 1 = 0, 2 = lowpass,
    // 3..5 = pyramid with main axis x, y, z; (j, k) pick g and Phi
    struct FKey {
      int kind, j, k;
      bool operator<(const FKey &o) const {
        return kind != o.kind ? kind < o.kind : j != o.j ? j < o.j : k < o.k;
      }
    };
    enum { kOne = 0, kZero = 1, kLow = 2 };
    auto fkey = [&](int i, int role) -> FKey {   // role 0 = C, 1 = X, 2 = Y
      if (i >= R) return FKey{role == 0 ? kZero : kOne, 0, 0};
      const auto &b = bank.subbands[i];
      if (b.cone == 0) return (role == 1) ? FKey{kOne, 0, 0} : FKey{kLow, 0, 0};
      const int kind = 2 + b.cone;   // 3, 4, 5 for main axis x, y, z
      if (role == 0) return b.cone == 3 ? FKey{kOne, 0, 0} : FKey{kind, b.j, b.k1};
      if (role == 1) return b.cone == 2 ? FKey{kOne, 0, 0} : FKey{kind, b.j, b.cone == 3 ? b.k1 : b.k2};
      return b.cone == 1 ? FKey{kOne, 0, 0} : FKey{kind, b.j, b.k2};
    };
    // value of a factor at (v, u): C (y, x), X (z, x), Y (z, y); planes are
    // stored [secondary][main]
    struct Fac {
      int kind, am;
      const double *g, *pl;
    };
    auto resolve = [&](int role, const FKey &f) -> Fac {
      Fac r{f.kind, 0, nullptr, nullptr};
      if (f.kind < 3) return r;
      r.am = f.kind - 2;
      r.g = t.g[(size_t)f.j * 3 + r.am - 1].data();
      // secondary axis of the plane, [role][main axis]: C uses Phi(x, y) or
      // Phi(y, x), X uses Phi(x, z) or Phi(z, x), Y uses Phi(y, z) or Phi(z, y)
      static const int sec[3][4] = {{0, 2, 1, 0}, {0, 3, 0, 1}, {0, 0, 3, 2}};
      const int sa = sec[role][r.am];
      r.pl = t.planes[t.find(f.j, f.k, r.am, sa)].data();
      return r;
    };
    auto fval = [&](int role, const Fac &f, int v, int u) -> double {
      if (f.kind == kOne) return 1.0;
      if (f.kind == kZero) return 0.0;
      if (f.kind == kLow) return role == 0 ? t.low[0][u] * t.low[1][v] : t.low[2][v];
      if (role == 0) {
        if (f.am == 1) return f.g[u] * f.pl[(size_t)v * W + u];
        return f.g[v] * f.pl[(size_t)u * H + v];
      }
      if (role == 1) {
        if (f.am == 1) return f.pl[(size_t)v * W + u];
        return f.pl[(size_t)u * D + v];
      }
      if (f.am == 2) return f.pl[(size_t)v * H + u];
      return f.g[v] * f.pl[(size_t)u * D + v];
    };
    struct Combo {
      int role;
      FKey a, b;
      bool operator<(const Combo &o) const {
        if (role != o.role) return role < o.role;
        if (a < o.a || o.a < a) return a < o.a;
        return b < o.b;
      }
    };
    const size_t rows[3] = {(size_t)H, (size_t)D, (size_t)D};
    const size_t cols[3] = {(size_t)W, (size_t)W, (size_t)H};
    std::map<Combo, long long> combo_off;
    std::vector<Combo> combos;
    size_t total = 0;
    auto place = [&](const Combo &cb) -> long long {
      auto it = combo_off.find(cb);
      if (it != combo_off.end()) return it->second;
      const long long off = (long long)total;
      total += rows[cb.role] * cols[cb.role];
      combo_off.emplace(cb, off);
      combos.push_back(cb);
      return off;
    };
    const int P = (R + 1) / 2;
    std::vector<sl::ZPair> zpairs(P);
    for (int p = 0; p < P; ++p) {
      const int a = 2 * p, b = 2 * p + 1;
      sl::ZPair &z = zpairs[p];
      z.c = place(Combo{0, fkey(a, 0), fkey(b, 0)});
      z.x = z.y = -1;
      for (int role = 1; role <= 2; ++role) {
        const Combo cb{role, fkey(a, role), fkey(b, role)};
        if (cb.a.kind == kOne && cb.b.kind == kOne) continue;   // neither has it
        (role == 1 ? z.x : z.y) = place(cb);
      }
    }
    std::vector<float2> ztab(total);
    slh::parallel_run((int64_t)combos.size(), [&](int64_t q) {
      const Combo &cb = combos[q];
      float2 *dst = ztab.data() + combo_off.at(cb);
      const Fac fa = resolve(cb.role, cb.a), fb = resolve(cb.role, cb.b);
      for (size_t v = 0; v < rows[cb.role]; ++v)
        for (size_t u = 0; u < cols[cb.role]; ++u)
          dst[v * cols[cb.role] + u] = make_float2((float)fval(cb.role, fa, (int)v, (int)u),
                                                   (float)fval(cb.role, fb, (int)v, (int)u));
    });
    if ((rc = dev_upload(s, ztab, &s->d_ztab)) || (rc = dev_upload(s, zpairs, &s->d_zpairs))) {
      sl_free_system(s);
      return rc;
    }
  }
  if (!is3d) {
    // flag that a timed-out cooperative wait sets (host memory the kernel
    // writes directly); without it the cooperative passes stay off
    void *hp = nullptr, *dp = nullptr;
    // off by default: on MI355X the line passes are faster (32 x 512^2 step
    // 2.35 ms against 2.67 ms with the cooperative passes)
    const char *xe = std::getenv("SL_XCD");
    s->xcd = xe ? std::atoi(xe) != 0 : 0;
    if (hipHostMalloc(&hp, 64, hipHostMallocCoherent) == hipSuccess) {
      s->xcd_err_host = (int *)hp;
      *(volatile int *)s->xcd_err_host = 0;
      if (hipHostGetDevicePointer(&dp, hp, 0) == hipSuccess) s->xcd_err_dev = (int *)dp;
    }
    (void)hipGetLastError();
  }
  for (int a = 0; a < s->cfg.ndim; ++a) {
    int N = (int)s->cfg.dims[a];
    if (s->d_tw.count(N)) continue;
    float2 *p = nullptr;
    if ((rc = dev_upload(s, twiddles(N), &p))) {
      sl_free_system(s);
      return rc;
    }
    s->d_tw[N] = p;
  }
  *out = s;
  return SL_OK;
}

}  // namespace

extern "C" {

int sl_build_system(const sl_config *cfg, sl_system **out) {
  return build_system_impl(cfg, false, out);
}

int sl_build_wavelet_system(const sl_config *cfg, sl_system **out) {
  return build_system_impl(cfg, true, out);
}

int sl_build_wavelet_filters_host(const sl_config *cfg, double *filters_host, double *dual_host,
                                  sl_subband *subbands_host) {
  slh::Config c;
  std::string err;
  int rc = parse_wavelet_config(cfg, c, err);
  if (rc != SL_OK) return fail(rc, err);
  slh::Bank bank;
  std::vector<double> tmp;
  double *fo = filters_host;
  if (!fo) {
    tmp.resize((size_t)(3 * c.J + 1) * c.npix());
    fo = tmp.data();
  }
  rc = slh::build_wavelet_bank(c, bank, fo, err);
  if (dual_host) std::copy(bank.dual.begin(), bank.dual.end(), dual_host);
  if (subbands_host)
    for (size_t i = 0; i < bank.subbands.size(); ++i) {
      const auto &b = bank.subbands[i];
      subbands_host[i] = {b.cone, b.j, b.k1, b.k2, bank.l2[i], bank.l1[i]};
    }
  if (rc != SL_OK) return fail(rc, err);
  return SL_OK;
}

void sl_free_system(sl_system *s) {
  if (!s) return;
  for (auto &g : s->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  for (void *p : s->allocs) (void)hipFree(p);
  if (s->xcd_err_host) (void)hipHostFree(s->xcd_err_host);
  delete s;
}

int sl_system_num_subbands(const sl_system *s, int *R_out) {
  if (!s || !R_out) return fail(SL_EINVAL, "NULL argument");
  *R_out = s->R;
  return SL_OK;
}

int sl_system_subband(const sl_system *s, int i, sl_subband *out) {
  if (!s || !out) return fail(SL_EINVAL, "NULL argument");
  if (i < 0 || i >= s->R) return fail(SL_EINVAL, "subband index out of range");
  const auto &b = s->subs[i];
  *out = {b.cone, b.j, b.k1, b.k2, s->l2[i], s->l1[i]};
  return SL_OK;
}

int sl_system_set_line_plan(sl_system *s, int values_factor) {
  if (!s || (values_factor != 1 && values_factor != 2))
    return fail(SL_EINVAL, "values_factor must be 1 or 2");
  s->line_em = values_factor;
  return SL_OK;
}

int sl_system_line_plan(const sl_system *s, int *values_factor) {
  if (!s || !values_factor) return fail(SL_EINVAL, "NULL argument");
  *values_factor = s->line_em;
  return SL_OK;
}

int sl_system_set_xcd(sl_system *s, int enable, int spin_limit) {
  if (!s || (enable != 0 && enable != 1) || spin_limit < 0)
    return fail(SL_EINVAL, "enable must be 0 or 1 and spin_limit >= 0");
  s->xcd = enable;
  s->xcd_spin = spin_limit ? spin_limit : (1 << 20);
  return SL_OK;
}

int sl_system_xcd_active(const sl_system *s, int batch, int *active) {
  if (!s || !active || batch < 1) return fail(SL_EINVAL, "bad arguments");
  *active = use_xcd(s, batch, layout(s, batch)) ? 1 : 0;
  return SL_OK;
}

int sl_workspace_size(const sl_system *s, int batch, size_t *bytes_out) {
  if (!s || !bytes_out) return fail(SL_EINVAL, "NULL argument");
  if (batch < 1) return fail(SL_EINVAL, "batch must be >= 1");
  *bytes_out = layout(s, batch).total;
  return SL_OK;
}

static int forward_impl(const sl_system *s, const float *x_dev, int batch, void *coeffs_dev,
                        float *scales_dev, void *workspace_dev, size_t workspace_bytes,
                        void *stream, bool dual) {
  int rc = check_call(s, batch, x_dev, coeffs_dev, workspace_dev, workspace_bytes);
  if (rc) return rc;
  const bool scaled = s->cfg.dtype != SL_F32;
  if (scaled && !scales_dev) return fail(SL_EINVAL, "scales_dev is required for F16/BF16 storage");
  hipStream_t st = (hipStream_t)stream;
  const Layout L = layout(s, batch);
  char *ws = (char *)workspace_dev;
  float2 *F = (float2 *)(ws + L.off_F);
  float2 *T = (float2 *)(ws + L.off_chunk);
  unsigned *xmax = (unsigned *)(ws + L.off_xmax);
  if (s->cfg.ndim == 3)
    return forward3d(s, x_dev, batch, coeffs_dev, scales_dev, F, T, xmax, dual, st);
  const sl::Sys2D v = view2d(s);
  if (!dual && use_xcd(s, batch, L)) {
    SL_LAUNCH(P_XCD_FWD, st,
              sl::launch_xcd_fwd(v, x_dev, (float *)coeffs_dev, ws + L.off_chunk,
                                 s->xcd_err_dev, batch, s->xcd_spin, st));
    return SL_OK;
  }
  if (scaled) SL_LAUNCH(P_AUX, st, sl::launch_zero_u32(xmax, batch, st));
  SL_LAUNCH(P_ROWS_REAL_FFT, st, sl::launch_rows_real_fft(v, x_dev, F, scaled ? xmax : nullptr, batch, st));
  SL_LAUNCH(P_COLS_FFT, st, sl::launch_cols_fft(v, F, F, batch, false, st));
  if (dual) SL_LAUNCH(P_AUX, st, sl::launch_div_psi(F, s->d_psi, (size_t)s->cfg.npix(), batch, st));
  if (scaled) SL_LAUNCH(P_AUX, st, sl::launch_scales(v, xmax, scales_dev, batch, st));
  int nb, np;
  chunk_plan(s, batch, nb, np);
  const int P = (s->R + 1) / 2;
  for (int b0 = 0; b0 < batch; b0 += nb)
    for (int p0 = 0; p0 < P; p0 += np) {
      sl::Chunk c{b0, std::min(nb, batch - b0), p0, std::min(np, P - p0)};
      SL_LAUNCH(P_COLS_FILTER_IFFT, st, sl::launch_cols_filter_ifft(v, F, T, c, st));
      SL_LAUNCH(P_ROWS_COEF, st, sl::launch_rows_coef(v, T, coeffs_dev, scales_dev, c, st));
    }
  return SL_OK;
}

int sl_forward(const sl_system *s, const float *x_dev, int batch, void *coeffs_dev,
               float *scales_dev, void *workspace_dev, size_t workspace_bytes, void *stream) {
  return forward_impl(s, x_dev, batch, coeffs_dev, scales_dev, workspace_dev, workspace_bytes,
                      stream, false);
}

int sl_inverse_adjoint(const sl_system *s, const float *r_dev, int batch, float *coeffs_dev,
                       void *workspace_dev, size_t workspace_bytes, void *stream) {
  if (s && s->cfg.dtype != SL_F32) return fail(SL_EINVAL, "the adjoint needs SL_F32 storage");
  return forward_impl(s, r_dev, batch, coeffs_dev, nullptr, workspace_dev, workspace_bytes,
                      stream, true);
}

int sl_inverse(const sl_system *s, const void *coeffs_dev, const float *scales_dev, int batch,
               const float *sigma_dev, const float *K_host, float *x_dev, void *workspace_dev,
               size_t workspace_bytes, void *stream) {
  int rc = check_call(s, batch, coeffs_dev, x_dev, workspace_dev, workspace_bytes);
  if (rc) return rc;
  const bool scaled = s->cfg.dtype != SL_F32;
  if (scaled && !scales_dev) return fail(SL_EINVAL, "scales_dev is required for F16/BF16 storage");
  sl::ThrArgs thr{};
  thr.sigma = sigma_dev;
  thr.l2 = s->d_l2;
  thr.jof = s->d_jof;
  if (sigma_dev) {
    if (!K_host) return fail(SL_EINVAL, "K_host is required with sigma_dev");
    if (s->cfg.J > sl::kMaxScales) return fail(SL_EUNSUPPORTED, "too many scales");
    for (int j = 0; j < s->cfg.J; ++j) thr.K[j] = K_host[j];
  }
  hipStream_t st = (hipStream_t)stream;
  const Layout L = layout(s, batch);
  char *ws = (char *)workspace_dev;
  float2 *ACC = (float2 *)(ws + L.off_F);
  float2 *U = (float2 *)(ws + L.off_chunk);
  if (s->cfg.ndim == 3) return inverse3d(s, coeffs_dev, scales_dev, batch, thr, x_dev, ACC, U, st);
  const sl::Sys2D v = view2d(s);
  if (use_xcd(s, batch, L)) {
    SL_LAUNCH(P_XCD_INV, st,
              sl::launch_xcd_inv(v, (const float *)coeffs_dev, thr, x_dev, ws + L.off_chunk,
                                 s->xcd_err_dev, batch, s->xcd_spin, st));
    return SL_OK;
  }
  int nb, np;
  chunk_plan(s, batch, nb, np);
  const int P = (s->R + 1) / 2;
  const int G = inv_groups(s, batch);
  float2 *part = (float2 *)(ws + L.off_part);
  for (int b0 = 0; b0 < batch; b0 += nb)
    for (int p0 = 0; p0 < P; p0 += np) {
      sl::Chunk c{b0, std::min(nb, batch - b0), p0, std::min(np, P - p0)};
      SL_LAUNCH(P_ROWS_COEF_FFT, st, sl::launch_rows_coef_fft(v, coeffs_dev, scales_dev, U, c, thr, st));
      SL_LAUNCH(P_COLS_FFT_ACC, st,
                sl::launch_cols_fft_acc(v, U, ACC, part, G, batch, c, p0 == 0, p0 + c.np == P, st));
    }
  if (G > 1) SL_LAUNCH(P_COLS_FFT_ACC, st, sl::launch_cols_acc_finish(v, ACC, part, G, batch, st));
  SL_LAUNCH(P_ROWS_REAL_IFFT, st, sl::launch_rows_real_ifft(v, ACC, x_dev, batch, st));
  return SL_OK;
}

int sl_denoise_fused(const sl_system *s, const float *x_dev, int batch, const float *sigma_dev,
                     const float *K_host, float *out_dev, void *workspace_dev,
                     size_t workspace_bytes, void *stream) {
  int rc = check_call(s, batch, x_dev, out_dev, workspace_dev, workspace_bytes);
  if (rc) return rc;
  if (!sigma_dev || !K_host) return fail(SL_EINVAL, "sigma_dev and K_host are required");
  if (s->cfg.J > sl::kMaxScales) return fail(SL_EUNSUPPORTED, "too many scales");
  sl::ThrArgs thr{};
  thr.sigma = sigma_dev;
  thr.l2 = s->d_l2;
  thr.jof = s->d_jof;
  for (int j = 0; j < s->cfg.J; ++j) thr.K[j] = K_host[j];
  return denoise_fused_run(s, x_dev, batch, thr, out_dev, (char *)workspace_dev,
                           (hipStream_t)stream);
}

namespace {
size_t al256(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

int sl_denoise_workspace_size(const sl_system *s, int batch, int with_model, size_t *bytes_out) {
  if (!s || !bytes_out) return fail(SL_EINVAL, "NULL argument");
  if (batch < 1) return fail(SL_EINVAL, "batch must be >= 1");
  size_t need = sl::transform_workspace_bytes(s, batch);
  if (with_model) {
    size_t cnn = 0;
    int rc = sl_cnn_workspace_size(s, batch, 0, &cnn);
    if (rc) return rc;
    // the shrunk coefficients, then whatever the CNN and the inverse need (they
    // run one after the other on the stream, so they share the rest)
    need = al256((size_t)batch * s->R * (size_t)s->cfg.npix() * sizeof(float)) +
           std::max(need, cnn);
  }
  *bytes_out = need;
  return SL_OK;
}

int sl_denoise(const sl_system *s, const float *x_dev, int batch, const float *sigma_dev,
               const float *K_host, const sl_shrinkage_model *model, void *coeffs_dev,
               float *scales_dev, float *out_dev, void *workspace_dev, size_t workspace_bytes,
               void *stream) {
  if (!model) {
    if (!sigma_dev || !K_host) return fail(SL_EINVAL, "sigma_dev and K_host are required");
    int rc = sl_forward(s, x_dev, batch, coeffs_dev, scales_dev, workspace_dev, workspace_bytes,
                        stream);
    if (rc) return rc;
    return sl_inverse(s, coeffs_dev, scales_dev, batch, sigma_dev, K_host, out_dev, workspace_dev,
                      workspace_bytes, stream);
  }
  // learned shrinkage: forward, gains from the network, inverse of g .* c
  if (!s) return fail(SL_EINVAL, "system is NULL");
  if (!sigma_dev || !model->params_dev || !model->packed_dev || !workspace_dev)
    return fail(SL_EINVAL, "sigma_dev, the model's buffers and the workspace are required");
  if (batch < 1 || batch > 65535) return fail(SL_EINVAL, "batch must be in 1..65535");
  size_t need = 0;
  int rc = sl_denoise_workspace_size(s, batch, 1, &need);
  if (rc) return rc;
  if (workspace_bytes < need)
    return fail(SL_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if ((uintptr_t)workspace_dev & 15u) return fail(SL_EINVAL, "workspace must be 16-byte aligned");
  const size_t shrunk_bytes = al256((size_t)batch * s->R * (size_t)s->cfg.npix() * sizeof(float));
  float *shrunk = (float *)workspace_dev;
  void *rest = (char *)workspace_dev + shrunk_bytes;
  const size_t rest_bytes = workspace_bytes - shrunk_bytes;
  rc = sl_forward(s, x_dev, batch, coeffs_dev, scales_dev, rest, rest_bytes, stream);
  if (rc) return rc;
  rc = sl_cnn_apply(s, model->params_dev, model->packed_dev, (const float *)coeffs_dev,
                    sigma_dev, batch, shrunk, nullptr, rest, rest_bytes, stream);
  if (rc) return rc;
  return sl_inverse(s, shrunk, nullptr, batch, nullptr, nullptr, out_dev, rest, rest_bytes,
                    stream);
}

int sl_get_filters(const sl_system *s, double *filters_host) {
  if (!s || !filters_host) return fail(SL_EINVAL, "NULL argument");
  slh::Bank bank;
  std::string err;
  int rc = s->wavelet ? slh::build_wavelet_bank(s->cfg, bank, filters_host, err)
                      : slh::build_bank(s->cfg, bank, filters_host, err);
  if (rc != SL_OK) return fail(rc, err);
  return SL_OK;
}

int sl_get_dual_weight(const sl_system *s, double *dual_host) {
  if (!s || !dual_host) return fail(SL_EINVAL, "NULL argument");
  slh::Bank bank;
  std::string err;
  std::vector<double> tmp;
  int rc;
  if (s->wavelet) {
    // the wavelet bank forms Psi_hat from the filters it writes
    tmp.resize((size_t)s->R * s->cfg.npix());
    rc = slh::build_wavelet_bank(s->cfg, bank, tmp.data(), err);
  } else {
    rc = slh::build_bank(s->cfg, bank, nullptr, err);
  }
  if (rc != SL_OK) return fail(rc, err);
  std::copy(bank.dual.begin(), bank.dual.end(), dual_host);
  return SL_OK;
}

int sl_inpaint_workspace_size(const sl_system *s, int batch, size_t *bytes_out) {
  if (!s || !bytes_out) return fail(SL_EINVAL, "NULL argument");
  if (batch < 1) return fail(SL_EINVAL, "batch must be >= 1");
  *bytes_out = inpaint_layout(s, batch).total;
  return SL_OK;
}

int sl_inpaint(const sl_system *s, const float *f_masked_dev, const unsigned char *mask_dev,
               int batch, const float *delta_init_dev, double delta_min, int iterations,
               int t_begin, int t_end, float *f_dev, int use_graph, void *workspace_dev,
               size_t workspace_bytes, void *stream) {
  if (!s) return fail(SL_EINVAL, "system is NULL");
  if (batch < 1 || batch > 65535) return fail(SL_EINVAL, "batch must be in 1..65535");
  if (!f_masked_dev || !mask_dev || !delta_init_dev || !f_dev || !workspace_dev)
    return fail(SL_EINVAL, "NULL buffer");
  if (iterations < 1) return fail(SL_EINVAL, "iterations must be >= 1");
  if (t_begin < 0 || t_end < t_begin || t_end > iterations)
    return fail(SL_EINVAL, "need 0 <= t_begin <= t_end <= iterations");
  if (!(delta_min >= 0.0) || !std::isfinite(delta_min))
    return fail(SL_EINVAL, "delta_min must be finite and >= 0");
  if (((uintptr_t)f_masked_dev | (uintptr_t)f_dev | (uintptr_t)workspace_dev) & 15u)
    return fail(SL_EINVAL, "f_masked, f and the workspace must be 16-byte aligned");
  if ((uintptr_t)mask_dev & 3u) return fail(SL_EINVAL, "mask must be 4-byte aligned");
  if (s->cfg.J > sl::kMaxScales) return fail(SL_EUNSUPPORTED, "too many scales");
  if (s->cfg.npix() % 4) return fail(SL_EUNSUPPORTED, "the sample count must be a multiple of 4");
  const InpaintLayout L = inpaint_layout(s, batch);
  if (workspace_bytes < L.total)
    return fail(SL_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->device)
    return fail(SL_EINVAL, "the current HIP device is not the system's device");
  if (t_begin == t_end) return SL_OK;
  InpaintArgs a{f_masked_dev, mask_dev, batch,   delta_init_dev, delta_min,
                iterations,   t_begin,  t_end,   f_dev,          (char *)workspace_dev};
  std::vector<uint64_t> key = {0x1a, (uint64_t)(uintptr_t)f_masked_dev, (uint64_t)(uintptr_t)mask_dev,
                               (uint64_t)batch, (uint64_t)(uintptr_t)delta_init_dev,
                               bits_of(delta_min), (uint64_t)iterations, (uint64_t)t_begin,
                               (uint64_t)t_end, (uint64_t)(uintptr_t)f_dev,
                               (uint64_t)(uintptr_t)workspace_dev, (uint64_t)s->chunk_cap,
                               (uint64_t)s->inv_images, (uint64_t)s->split_pairs};
  return run_or_replay(s, key, use_graph != 0, (hipStream_t)stream,
                       [&](hipStream_t q) { return inpaint_launches(s, a, q); });
}

int sl_decompose_workspace_size(const sl_system *s0, const sl_system *s1, int batch,
                                size_t *bytes_out) {
  if (!s0 || !s1 || !bytes_out) return fail(SL_EINVAL, "NULL argument");
  if (batch < 1) return fail(SL_EINVAL, "batch must be >= 1");
  if (s0->cfg.ndim != s1->cfg.ndim || s0->cfg.npix() != s1->cfg.npix())
    return fail(SL_EINVAL, "the two systems must have the same dims");
  *bytes_out = decomp_layout(s0, s1, batch).total;
  return SL_OK;
}

int sl_decompose(const sl_system *s0, const sl_system *s1, const float *f_dev, int batch,
                 const float *delta_init_dev, double delta_min, int iterations, int t_begin,
                 int t_end, float *f0_dev, float *f1_dev, int use_graph, void *workspace_dev,
                 size_t workspace_bytes, void *stream) {
  if (!s0 || !s1) return fail(SL_EINVAL, "system is NULL");
  if (s0->cfg.ndim != s1->cfg.ndim)
    return fail(SL_EINVAL, "the two systems must have the same dims");
  for (int a = 0; a < s0->cfg.ndim; ++a)
    if (s0->cfg.dims[a] != s1->cfg.dims[a])
      return fail(SL_EINVAL, "the two systems must have the same dims");
  if (s0->device != s1->device) return fail(SL_EINVAL, "the two systems are on different devices");
  if (batch < 1 || batch > 65535) return fail(SL_EINVAL, "batch must be in 1..65535");
  if (!f_dev || !delta_init_dev || !f0_dev || !f1_dev || !workspace_dev)
    return fail(SL_EINVAL, "NULL buffer");
  if (f0_dev == f1_dev) return fail(SL_EINVAL, "f0 and f1 must be different buffers");
  if (iterations < 1) return fail(SL_EINVAL, "iterations must be >= 1");
  if (t_begin < 0 || t_end < t_begin || t_end > iterations)
    return fail(SL_EINVAL, "need 0 <= t_begin <= t_end <= iterations");
  if (!(delta_min >= 0.0) || !std::isfinite(delta_min))
    return fail(SL_EINVAL, "delta_min must be finite and >= 0");
  if (((uintptr_t)f_dev | (uintptr_t)f0_dev | (uintptr_t)f1_dev | (uintptr_t)workspace_dev) & 15u)
    return fail(SL_EINVAL, "f, f0, f1 and the workspace must be 16-byte aligned");
  if (s0->cfg.J > sl::kMaxScales || s1->cfg.J > sl::kMaxScales)
    return fail(SL_EUNSUPPORTED, "too many scales");
  if (s0->cfg.npix() % 4) return fail(SL_EUNSUPPORTED, "the sample count must be a multiple of 4");
  const DecompLayout L = decomp_layout(s0, s1, batch);
  if (workspace_bytes < L.total)
    return fail(SL_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != s0->device)
    return fail(SL_EINVAL, "the current HIP device is not the systems' device");
  if (t_begin == t_end) return SL_OK;
  char *ws = (char *)workspace_dev;
  float *g0 = (float *)(ws + L.off_g0), *g1 = (float *)(ws + L.off_g1);
  float *sigma = (float *)(ws + L.off_sigma);
  const sl::ThrArgs thr0 = unit_thresholds(s0, sigma), thr1 = unit_thresholds(s1, sigma);
  const size_t n = (size_t)s0->cfg.npix() * batch;
  auto launches = [&](hipStream_t q) -> int {
    for (int t = t_begin; t < t_end; ++t) {
      SL_LAUNCH(P_AUX, q,
                sl::launch_decompose_mix(f_dev, f0_dev, f1_dev, g0, g1, n, t == 0, delta_init_dev,
                                         schedule_factor(delta_min, iterations, t), sigma, batch,
                                         q));
      int rc = denoise_fused_run(s0, g0, batch, thr0, f0_dev, ws, q);
      if (!rc) rc = denoise_fused_run(s1, g1, batch, thr1, f1_dev, ws, q);
      if (rc) return rc;
    }
    return SL_OK;
  };
  // s1 by serial number: a later system at the same address is a new key
  std::vector<uint64_t> key = {0x2b, s1->serial, (uint64_t)(uintptr_t)f_dev,
                               (uint64_t)batch, (uint64_t)(uintptr_t)delta_init_dev,
                               bits_of(delta_min), (uint64_t)iterations, (uint64_t)t_begin,
                               (uint64_t)t_end, (uint64_t)(uintptr_t)f0_dev,
                               (uint64_t)(uintptr_t)f1_dev, (uint64_t)(uintptr_t)workspace_dev,
                               (uint64_t)s0->chunk_cap, (uint64_t)s1->chunk_cap,
                               (uint64_t)s0->inv_images, (uint64_t)s0->split_pairs,
                               (uint64_t)s1->inv_images, (uint64_t)s1->split_pairs};
  return run_or_replay(s0, key, use_graph != 0, (hipStream_t)stream, launches);
}

int sl_timing_enable(int on) {
  g_timing.on = on != 0;
  return SL_OK;
}

int sl_timing_reset(void) {
  g_timing.recycle();
  return SL_OK;
}

int sl_timing_num_passes(void) { return P_COUNT; }

const char *sl_timing_pass_name(int pass) {
  return (pass >= 0 && pass < P_COUNT) ? kPassNames[pass] : nullptr;
}

int sl_timing_query(int pass, double *total_ms_out, int *launches_out) {
  if (pass < 0 || pass >= P_COUNT || !total_ms_out || !launches_out)
    return fail(SL_EINVAL, "bad timing query");
  double tot = 0.0;
  for (auto &p : g_timing.ev[pass]) {
    hipError_t e = hipEventSynchronize(p.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p.first, p.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    tot += ms;
  }
  *total_ms_out = tot;
  *launches_out = (int)g_timing.ev[pass].size();
  return SL_OK;
}

}  // extern "C"
