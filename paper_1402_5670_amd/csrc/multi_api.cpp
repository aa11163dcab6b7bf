// Uneven batches: images of several sizes in one schedule (declared in
// include/shearlet.h).  Each size class runs the batched passes of its own
// system.  Two schedules: per class (the classes are independent, so a
// captured HIP graph forks one branch per class and the GPU runs the
// branches concurrently), or multi-class (one stream; at every step the
// column passes of each class, then one coefficient row launch whose flat
// work list covers the row blocks of all classes, largest first).  An autotuner
// picks each class's schedule by timing the candidates on the caller's
// buffers: the chunk size (the number of subband pairs per pass launch,
// which trades launch count against Infinity Cache residency of the
// intermediate) and, in 2D, the column tile shape of the inverse
// accumulation (one or two images per block) and whether small grids split
// the subband-pair loop over blocks, and for classes with 1024-point lines
// the line plan (values per thread of those lines' FFTs, kernels2d.hip).
// It then times the two schedules.  Results are cached in a small text file,
// one line per class (key, chunk bytes, images per block, split, line plan)
// and one for the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/shearlet.h"
#include "system.hpp"

struct sl_multi {
  std::vector<sl_system *> sys;
  std::vector<int> counts;
  int schedule = 0;   // 0: one multi-class coefficient row launch per step where
                      // supported, else per class; 1: per class (graph branches)
  std::vector<size_t> ws_off;
  size_t ws_total = 0;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t al(size_t v) { return (v + 255) / 256 * 256; }

void layout(sl_multi *m) {
  m->ws_off.assign(m->sys.size(), 0);
  size_t off = 0;
  for (size_t s = 0; s < m->sys.size(); ++s) {
    m->ws_off[s] = off;
    size_t b = 0;
    sl_workspace_size(m->sys[s], m->counts[s], &b);
    off += al(b);
  }
  m->ws_total = off;
}

struct Bufs {
  const float *const *x;
  void *const *coeffs;
  float *const *scales;
  const float *const *sigma;
  const float *K;
  float *const *out;
  char *ws;
};

std::vector<sl::MultiClass2D> classes(sl_multi *m, const Bufs &b) {
  std::vector<sl::MultiClass2D> c(m->sys.size());
  for (size_t s = 0; s < m->sys.size(); ++s) {
    size_t wsb = 0;
    sl_workspace_size(m->sys[s], m->counts[s], &wsb);
    c[s] = {m->sys[s], m->counts[s], b.x ? b.x[s] : nullptr, b.coeffs[s],
            b.scales ? b.scales[s] : nullptr, b.sigma ? b.sigma[s] : nullptr,
            b.out ? b.out[s] : nullptr, b.ws + m->ws_off[s], wsb};
  }
  return c;
}

// the multi-class schedule applies: chosen, and every class supports it
bool use_multi(sl_multi *m) {
  if (m->schedule != 0 || m->sys.size() > (size_t)sl::kMaxMultiClasses) return false;
  Bufs none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<void *> dummy(m->sys.size(), nullptr);
  none.coeffs = dummy.data();
  auto c = classes(m, none);
  return sl::multi2d_supported(c.data(), (int)c.size());
}

int run_all(sl_multi *m, const Bufs &b, int what, hipStream_t st);

int run_class(sl_multi *m, int s, const Bufs &b, int what, hipStream_t st) {
  void *ws = b.ws + m->ws_off[s];
  size_t wsb = 0;
  sl_workspace_size(m->sys[s], m->counts[s], &wsb);
  int rc = SL_OK;
  if (what & 1)
    rc = sl_forward(m->sys[s], b.x[s], m->counts[s], b.coeffs[s], b.scales ? b.scales[s] : nullptr,
                    ws, wsb, st);
  if (rc == SL_OK && (what & 2))
    rc = sl_inverse(m->sys[s], b.coeffs[s], b.scales ? b.scales[s] : nullptr, m->counts[s],
                    b.sigma ? b.sigma[s] : nullptr, b.K, b.out[s], ws, wsb, st);
  return rc;
}

int run_all(sl_multi *m, const Bufs &b, int what, hipStream_t st) {
  if (use_multi(m)) {
    auto c = classes(m, b);
    return sl::run_multi2d(c.data(), (int)c.size(), what, b.K, st);
  }
  for (size_t s = 0; s < m->sys.size(); ++s) {
    int rc = run_class(m, (int)s, b, what, st);
    if (rc) return rc;
  }
  return SL_OK;
}

std::string tune_key(const sl_system *s, int count) {
  std::ostringstream k;
  k << s->cfg.ndim;
  for (int i = 0; i < s->cfg.ndim; ++i) k << "x" << s->cfg.dims[i];
  k << ":R" << s->R << ":B" << count << ":T" << s->cfg.dtype;
  return k.str();
}

struct Sched {
  size_t chunk;
  int inv_images, split, line_em;
};

std::map<std::string, Sched> load_cache(const char *path) {
  std::map<std::string, Sched> c;
  if (!path) return c;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string key;
    Sched v{0, 0, 1, 1};
    if (!(ls >> key >> v.chunk)) continue;
    if (!(ls >> v.inv_images >> v.split)) v.inv_images = 0, v.split = 1;
    if (!(ls >> v.line_em) || (v.line_em != 1 && v.line_em != 2)) v.line_em = 1;
    c[key] = v;
  }
  return c;
}

void save_cache(const char *path, const std::map<std::string, Sched> &c) {
  if (!path) return;
  std::ofstream f(path);
  for (auto &kv : c)
    f << kv.first << " " << kv.second.chunk << " " << kv.second.inv_images << " "
      << kv.second.split << " " << kv.second.line_em << "\n";
}

void apply(sl_system *s, const Sched &v) {
  s->chunk_cap = v.chunk;
  s->inv_images = v.inv_images;
  s->split_pairs = v.split;
  s->line_em = v.line_em;
}

Sched current(const sl_system *s) {
  return {s->chunk_cap, s->inv_images, s->split_pairs, s->line_em};
}

// a class has a second line plan to try when it has 1024-point lines
bool has_em2(const sl_system *s) {
  return s->cfg.ndim == 2 && (s->cfg.dims[0] == 1024 || s->cfg.dims[1] == 1024);
}

#define CK(expr)                                            \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return sl::hip_error(e_, #expr);  \
  } while (0)

}  // namespace

extern "C" {

int sl_system_set_chunk_bytes(sl_system *s, size_t bytes) {
  if (!s || bytes < (1u << 20)) return sl::set_error(SL_EINVAL, "chunk must be >= 1 MiB");
  s->chunk_cap = bytes;
  return SL_OK;
}

size_t sl_system_chunk_bytes(const sl_system *s) { return s ? s->chunk_cap : 0; }

int sl_system_set_block_shape(sl_system *s, int inv_images, int split_pairs) {
  if (!s || inv_images < 0 || inv_images > 2 || (split_pairs != 0 && split_pairs != 1))
    return sl::set_error(SL_EINVAL, "inv_images must be 0, 1 or 2 and split_pairs 0 or 1");
  s->inv_images = inv_images;
  s->split_pairs = split_pairs;
  return SL_OK;
}

int sl_system_block_shape(const sl_system *s, int *inv_images, int *split_pairs) {
  if (!s || !inv_images || !split_pairs) return sl::set_error(SL_EINVAL, "NULL argument");
  *inv_images = s->inv_images;
  *split_pairs = s->split_pairs;
  return SL_OK;
}

int sl_multi_set_schedule(sl_multi *m, int per_class) {
  if (!m || (per_class != 0 && per_class != 1))
    return sl::set_error(SL_EINVAL, "per_class must be 0 or 1");
  m->schedule = per_class;
  return SL_OK;
}

int sl_multi_schedule(sl_multi *m, int *multi_class_rows) {
  if (!m || !multi_class_rows) return sl::set_error(SL_EINVAL, "NULL argument");
  *multi_class_rows = use_multi(m) ? 1 : 0;
  return SL_OK;
}

int sl_multi_create(sl_system *const *systems, const int *counts, int n_classes, sl_multi **out) {
  if (!systems || !counts || !out || n_classes < 1 || n_classes > 64)
    return sl::set_error(SL_EINVAL, "bad arguments to sl_multi_create");
  *out = nullptr;
  auto *m = new sl_multi();
  for (int s = 0; s < n_classes; ++s) {
    if (!systems[s] || counts[s] < 1) {
      delete m;
      return sl::set_error(SL_EINVAL, "every class needs a system and at least one image");
    }
    m->sys.push_back(systems[s]);
    m->counts.push_back(counts[s]);
  }
  layout(m);
  *out = m;
  return SL_OK;
}

void sl_multi_free(sl_multi *m) {
  if (!m) return;
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  for (auto st : m->side) (void)hipStreamDestroy(st);
  for (auto e : m->join) (void)hipEventDestroy(e);
  if (m->fork) (void)hipEventDestroy(m->fork);
  delete m;
}

int sl_multi_workspace_size(sl_multi *m, size_t *bytes_out) {
  if (!m || !bytes_out) return sl::set_error(SL_EINVAL, "NULL argument");
  layout(m);
  *bytes_out = m->ws_total;
  return SL_OK;
}

int sl_multi_run(sl_multi *m, int what, const float *const *x_dev, void *const *coeffs_dev,
                 float *const *scales_dev, const float *const *sigma_dev, const float *K_host,
                 float *const *out_dev, void *workspace_dev, size_t workspace_bytes,
                 void *stream) {
  if (!m || !workspace_dev || (what & ~3) || !what) return sl::set_error(SL_EINVAL, "bad arguments");
  layout(m);
  if (workspace_bytes < m->ws_total) return sl::set_error(SL_ENOMEM, "workspace too small");
  Bufs b{x_dev, coeffs_dev, scales_dev, sigma_dev, K_host, out_dev, (char *)workspace_dev};
  return run_all(m, b, what, (hipStream_t)stream);
}

int sl_multi_autotune(sl_multi *m, const float *const *x_dev, void *const *coeffs_dev,
                      float *const *scales_dev, float *const *out_dev, void *workspace_dev,
                      size_t workspace_bytes, const char *cache_path, void *stream) {
  if (!m || !workspace_dev) return sl::set_error(SL_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  auto cache = load_cache(cache_path);
  static const size_t cand_mb[] = {32, 128, 512, 2048};
  static const int cand_images[] = {1, 2}, cand_split[] = {1, 0};
  Bufs b{x_dev, coeffs_dev, scales_dev, nullptr, nullptr, out_dev, (char *)workspace_dev};
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  // the workspace was sized for the current chunks: only candidates that keep
  // every class within its present slot are admissible
  std::vector<size_t> slot(m->sys.size());
  for (size_t s = 0; s < m->sys.size(); ++s) sl_workspace_size(m->sys[s], m->counts[s], &slot[s]);
  int rc = SL_OK;
  for (size_t s = 0; s < m->sys.size() && rc == SL_OK; ++s) {
    const std::string key = tune_key(m->sys[s], m->counts[s]);
    sl_system *sy = m->sys[s];
    auto it = cache.find(key);
    if (it != cache.end()) {
      const Sched keep = current(sy);
      apply(sy, it->second);
      size_t need = 0;
      sl_workspace_size(sy, m->counts[s], &need);
      if (need > slot[s]) apply(sy, keep);
      continue;
    }
    float best = 1e30f;
    Sched best_s = current(sy);
    // the block shape only applies to 2D systems, the line plan to 1024-point lines
    const int n_images = sy->cfg.ndim == 2 ? 2 : 1, n_split = sy->cfg.ndim == 2 ? 2 : 1;
    const int n_em = has_em2(sy) ? 2 : 1;
    for (size_t mb : cand_mb)
      for (int ii = 0; ii < n_images && rc == SL_OK; ++ii)
        for (int si = 0; si < n_split && rc == SL_OK; ++si)
        for (int em = 1; em <= n_em && rc == SL_OK; ++em) {
          const Sched cand{mb << 20, sy->cfg.ndim == 2 ? cand_images[ii] : sy->inv_images,
                           sy->cfg.ndim == 2 ? cand_split[si] : sy->split_pairs, em};
          apply(sy, cand);
          size_t need = 0;
          sl_workspace_size(sy, m->counts[s], &need);
          if (need > slot[s]) continue;
          rc = run_class(m, (int)s, b, 3, st);                   // warm-up
          if (rc) break;
          (void)hipEventRecord(e0, st);
          for (int r = 0; r < 3 && rc == SL_OK; ++r) rc = run_class(m, (int)s, b, 3, st);
          (void)hipEventRecord(e1, st);
          if (rc) break;
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (ms < best) {
            best = ms;
            best_s = cand;
          }
        }
    apply(sy, best_s);
    cache[key] = best_s;
  }
  // the schedule across classes: per class (graph branches), or one
  // multi-class coefficient row launch per step (1024-point classes then take
  // the line plan that launch needs); cached under the classes' keys
  std::string skey = "schedule";
  for (size_t s = 0; s < m->sys.size(); ++s) skey += ";" + tune_key(m->sys[s], m->counts[s]);
  auto sit = cache.find(skey);
  if (rc == SL_OK && sit != cache.end()) {
    m->schedule = sit->second.split;
    if (m->schedule == 0)
      for (auto *sy : m->sys)
        if (has_em2(sy)) sy->line_em = 2;
  } else if (rc == SL_OK) {
    std::vector<int> em_was;
    for (auto *sy : m->sys) em_was.push_back(sy->line_em);
    auto time_all = [&](float &ms) -> int {
      int r = run_all(m, b, 3, st);   // warm-up
      if (r) return r;
      (void)hipEventRecord(e0, st);
      for (int k = 0; k < 3 && r == SL_OK; ++k) r = run_all(m, b, 3, st);
      (void)hipEventRecord(e1, st);
      if (r) return r;
      (void)hipEventSynchronize(e1);
      return hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? SL_OK : SL_EHIP;
    };
    float t_class = 1e30f, t_multi = 1e30f;
    m->schedule = 1;
    rc = time_all(t_class);
    if (rc == SL_OK) {
      m->schedule = 0;
      for (auto *sy : m->sys)
        if (has_em2(sy)) sy->line_em = 2;
      if (use_multi(m)) rc = time_all(t_multi);
    }
    if (rc == SL_OK && t_multi < t_class) {
      m->schedule = 0;
    } else {
      m->schedule = 1;
      for (size_t s = 0; s < m->sys.size(); ++s) m->sys[s]->line_em = em_was[s];
    }
    Sched sv{0, 0, m->schedule, 0};
    cache[skey] = sv;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  save_cache(cache_path, cache);
  layout(m);
  if (m->ws_total > workspace_bytes) return sl::set_error(SL_ENOMEM, "workspace too small");
  return SL_OK;
}

int sl_multi_graph_build(sl_multi *m, int what, const float *const *x_dev,
                         void *const *coeffs_dev, float *const *scales_dev,
                         const float *const *sigma_dev, const float *K_host,
                         float *const *out_dev, void *workspace_dev, size_t workspace_bytes) {
  if (!m || !workspace_dev || (what & ~3) || !what) return sl::set_error(SL_EINVAL, "bad arguments");
  layout(m);
  if (workspace_bytes < m->ws_total) return sl::set_error(SL_ENOMEM, "workspace too small");
  if (m->exec) {
    (void)hipGraphExecDestroy(m->exec);
    m->exec = nullptr;
  }
  if (m->graph) {
    (void)hipGraphDestroy(m->graph);
    m->graph = nullptr;
  }
  const int n = (int)m->sys.size();
  while ((int)m->side.size() < n) {
    hipStream_t st;
    CK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    m->side.push_back(st);
    hipEvent_t e;
    CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    m->join.push_back(e);
  }
  if (!m->fork) CK(hipEventCreateWithFlags(&m->fork, hipEventDisableTiming));
  Bufs b{x_dev, coeffs_dev, scales_dev, sigma_dev, K_host, out_dev, (char *)workspace_dev};
  hipStream_t cs = m->side[0];
  CK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  // per-pass timing events must not be recorded into the graph
  const bool capturing_was = sl::set_capturing(true);
  int rc = SL_OK;
  hipError_t e = hipSuccess;
  if (use_multi(m)) {
    // one stream: the per-class passes and the multi-class row launches in order
    rc = run_all(m, b, what, cs);
  } else {
    e = hipEventRecord(m->fork, cs);
    for (int s = 1; s < n && e == hipSuccess; ++s) e = hipStreamWaitEvent(m->side[s], m->fork, 0);
    for (int s = 0; s < n && e == hipSuccess && rc == SL_OK; ++s) {
      rc = run_class(m, s, b, what, m->side[s]);
      if (rc == SL_OK && s > 0) {
        e = hipEventRecord(m->join[s], m->side[s]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, m->join[s], 0);
      }
    }
  }
  sl::set_capturing(capturing_was);
  hipGraph_t g = nullptr;
  hipError_t ec = hipStreamEndCapture(cs, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return sl::hip_error(e, "graph capture");
  }
  if (ec != hipSuccess) return sl::hip_error(ec, "hipStreamEndCapture");
  m->graph = g;
  CK(hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0));
  return SL_OK;
}

int sl_multi_graph_launch(sl_multi *m, void *stream) {
  if (!m || !m->exec) return sl::set_error(SL_EINVAL, "no graph: call sl_multi_graph_build");
  CK(hipGraphLaunch(m->exec, (hipStream_t)stream));
  return SL_OK;
}

}  // extern "C"
