// Host-side FP64 construction of the shearlet filter bank in closed form.
//
// The spatial definition of the paper (digital shear of p_j * W_j,
// Definitions digitSH_alpha and 3DdigitSH_alpha) has the DTFT
//
//   Phi_hat_{j,k}(xi_m, xi_s) = sum_{r=0}^{L-1} h_hat_d((xi_m + r)/L)^2
//        * P(2^{J-j-1} xi_m, 2^{J-j+d} eta_r) * h_hat_{J-j+d}(eta_r),
//   eta_r = xi_s - k (xi_m + r) / L,      L = 2^d,  d = shear_levels[j],
//
// (upsampling by L, the interpolation h_d, the integer shear S_k, h_d again
// and downsampling by L, eqs. dshear1_alpha / dshear2_alpha), and
//   2D cone 1:   psi_hat_{j,k}(xi1, xi2) = g_hat_{J-j}(xi1) Phi_hat_{j,k}(xi1, xi2)
//   3D pyr. 1:   psi_hat_{j,k1,k2}(xi)   = g_hat_{J-j}(xi1) Phi_hat_{j,k1}(xi1, xi2)
//                                                          Phi_hat_{j,k2}(xi1, xi3)
// with the other cones/pyramids obtained by permuting the variables.  The
// cascades follow eq. lowhigh.  Every phase is reduced exactly as an integer
// fraction before the cosine is taken.
#pragma once

#include <cstdint>
#include <string>
#include <functional>
#include <vector>

#include "../../include/shearlet.h"

namespace slh {

struct Config {
  int ndim = 2;
  int64_t dims[3] = {0, 0, 0};       // [H, W] or [D, H, W]
  int J = 1;
  std::vector<int> levels;
  std::vector<double> h;             // h(0), h(1), ... (symmetric half)
  bool default_P = true;
  std::vector<double> P;             // [rows][cols] taps, rows along x2
  int prow = 0, pcol = 0;
  bool full = false;
  int dtype = SL_F32;

  // axis sizes by paper axis: n(1) = N1 (fastest), n(2), n(3)
  int n(int axis) const {
    if (ndim == 2) return (int)(axis == 1 ? dims[1] : dims[0]);
    return (int)(axis == 1 ? dims[2] : axis == 2 ? dims[1] : dims[0]);
  }
  int64_t npix() const {
    int64_t p = 1;
    for (int i = 0; i < ndim; ++i) p *= dims[i];
    return p;
  }
};

struct Subband {
  int cone, j, k1, k2;
};

// Validate and copy a user configuration.  Returns SL_OK or an error code
// with a message in err.
int parse_config(const sl_config *cfg, Config &out, std::string &err);

std::vector<Subband> enumerate_subbands(const Config &c);

bool fft_size_supported(int64_t n);

// Phi_hat_{j,k} sampled on an [Ns][Nm] grid (secondary index slow).
void phi_plane(const Config &c, int j, int k, int Nm, int Ns, double *out);
// g_hat_{J-j} on the N-point grid; h_hat_J on the N-point grid.
void g_line(const Config &c, int j, int N, double *out);
void lowpass_line(const Config &c, int N, double *out);

// Complete bank.  For 2D, filters is [R][H][W]; for 3D [R][D][H][W] (only
// for small volumes).  Either pointer may be null.
struct Bank {
  std::vector<Subband> subbands;
  std::vector<double> l2, l1;
  std::vector<double> dual;          // Psi_hat on the full grid
  double dual_min = 0, dual_max = 0;
};
int build_bank(const Config &c, Bank &bank, double *filters_out, std::string &err);

// Undecimated separable wavelet bank (2D only) from the same QMF cascades
// (eq. lowhigh; the 2D digital wavelet transform of Section 3.4 without its
// subsampling): lowpass h_J (x) h_J, then for j = 0..J-1 cone 1 = g_{J-j}
// along x1 times h_{J-j} along x2, cone 2 = the transpose, cone 3 =
// g_{J-j} along both; k1 = k2 = 0.  R = 3 J + 1.
int build_wavelet_bank(const Config &c, Bank &bank, double *filters_out, std::string &err);

// 3D factor tables used by the device (and by build_bank).
struct Tables3D {
  // per scale j: plane[(j, k, pair)] where pair indexes an ordered
  // (main, secondary) axis combination; g per (j, axis); lowpass per axis.
  struct Key { int j, k, main_axis, sec_axis; };
  std::vector<Key> keys;
  std::vector<std::vector<double>> planes;     // each [Ns][Nm]
  std::vector<std::vector<double>> g;          // index j*3 + (axis-1)
  std::vector<std::vector<double>> low;        // index axis-1
  int find(int j, int k, int main_axis, int sec_axis) const;
};
void build_tables_3d(const Config &c, Tables3D &t);

// fn(0) .. fn(n - 1) on the host's hardware threads (at most 32)
void parallel_run(int64_t n, const std::function<void(int64_t)> &fn);

// Simple FP64 complex FFT for sizes 2^a 3^b (host; used for l1 norms).
void host_dft_inplace(std::vector<double> &re, std::vector<double> &im, int sign);

}  // namespace slh
