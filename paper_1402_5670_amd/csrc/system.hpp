// Library-owned state of a shearlet system (internal to libshearlet).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "dispatch.hpp"
#include "host_filters.hpp"

struct sl_system {
  slh::Config cfg;
  std::vector<slh::Subband> subs;
  std::vector<double> l2, l1;
  int R = 0;
  int device = 0;
  int num_cu = 1;                 // compute units of the device
  uint64_t serial = 0;            // unique per built system (graph cache keys)
  size_t chunk_cap = 0;
  int inv_images = 0;             // images per inverse accumulation block (0 = auto)
  int split_pairs = 1;            // small grids split the pair loop over blocks
  int line_em = 1;                // line plan of 1024-point lines (1 or 2)
  bool plane3d = true;            // volumes: y and x passes of a z-slice in LDS
  bool wavelet = false;           // built by sl_build_wavelet_system
  int xcd = 0;                    // 2D: XCD-cooperative passes where supported
  int xcd_spin = 1 << 20;         // polls before a cooperative wait gives up
  int *xcd_err_host = nullptr;    // host-visible flag a timed-out wait sets
  int *xcd_err_dev = nullptr;     // its device address
  float *d_filt = nullptr;    // 2D: [R][H][W]
  float *d_psi = nullptr;     // Psi_hat on the grid
  float *d_l2 = nullptr, *d_l1 = nullptr;
  int *d_jof = nullptr;
  sl::ZPair *d_zpairs = nullptr;  // 3D: per-pair offsets into d_ztab
  float2 *d_ztab = nullptr;       // 3D: per-pair z-line filter factors
  std::map<int, float2 *> d_tw;
  std::vector<void *> allocs;
  // instantiated inpainting graphs, keyed by every argument they bake in
  // (newest last; a few are kept)
  struct Graph {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> graphs;
  std::mutex graph_mu;
};

#include <string>

namespace sl {
// workspace layout shared by the transforms and the CNN calls
size_t transform_workspace_bytes(const sl_system *s, int batch);
// record an error message for sl_last_error and return code
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
// mark the calling thread as capturing a graph (per-pass timing events are
// then not recorded); returns the previous state
bool set_capturing(bool on);

// One size class of an uneven 2D batch for run_multi2d: its system, image
// count, buffers and its own workspace slot.
struct MultiClass2D {
  const sl_system *s;
  int B;
  const float *x;
  void *coef;
  float *scales;
  const float *sigma;
  float *out;
  void *ws;
  size_t ws_bytes;
};
// Whether run_multi2d can take these classes (2D systems of one storage type
// whose row lengths have a multi-class row pass).
bool multi2d_supported(const MultiClass2D *cls, int n);
// Forward (what & 1) and / or inverse (what & 2, hard threshold with K when
// a class has sigma) of every class on one stream: per class the spectrum
// and column passes, and for each schedule step one coefficient row launch
// across all classes (launch_rows_multi).
int run_multi2d(const MultiClass2D *cls, int n, int what, const float *K, hipStream_t st);
}
