// Host FP64 closed-form shearlet filter bank (see host_filters.hpp).
#include "host_filters.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <functional>
#include <thread>

namespace slh {

namespace {

const double kTwoPi = 6.283185307179586476925286766559;

inline int64_t pmod(int64_t a, int64_t m) {
  a %= m;
  return a < 0 ? a + m : a;
}

// cos(2 pi num / den) with the phase reduced exactly in integers.
inline double cos2pi(int64_t num, int64_t den) {
  int64_t r = pmod(num, den);
  if (2 * r > den) r = den - r;
  return std::cos(kTwoPi * (double)r / (double)den);
}

void parallel_for(int64_t n, const std::function<void(int64_t)> &fn) {
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  int nt = (int)std::min<int64_t>(n, std::min(hw, 32u));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= n) break;
        fn(i);
      }
    });
  for (auto &x : th) x.join();
}

// Trigonometric polynomial of a symmetric 1D filter at cos(2 pi xi) = c:
// h(0) + 2 sum_n s^n h(n) T_n(c), s = +1 (lowpass) or -1 (mirror highpass,
// g(n) = (-1)^n h(n)).
inline double qmf_eval(const std::vector<double> &h, double c, bool mirror) {
  double acc = h[0];
  double tm1 = 1.0, t = c;
  for (size_t n = 1; n < h.size(); ++n) {
    double sgn = (mirror && (n & 1)) ? -1.0 : 1.0;
    acc += 2.0 * sgn * h[n] * t;
    double tn = 2.0 * c * t - tm1;
    tm1 = t;
    t = tn;
  }
  return acc;
}

// h_hat_m(num/den) = prod_{k<m} h_hat(2^k num/den)    (eq. lowhigh)
inline double h_casc(const std::vector<double> &h, int m, int64_t num, int64_t den) {
  double v = 1.0;
  int64_t cur = pmod(num, den);
  for (int k = 0; k < m; ++k) {
    v *= qmf_eval(h, cos2pi(cur, den), false);
    cur = pmod(2 * cur, den);
  }
  return v;
}

// g_hat_m(num/den) = g_hat(2^{m-1} num/den) h_hat_{m-1}(num/den)   (eq. lowhigh)
inline double g_casc(const std::vector<double> &h, int m, int64_t num, int64_t den) {
  int64_t cur = pmod(num, den);
  for (int k = 0; k < m - 1; ++k) cur = pmod(2 * cur, den);
  return qmf_eval(h, cos2pi(cur, den), true) * h_casc(h, m - 1, num, den);
}

// Default fan filter: D_2(x) = (1 + x)^2 (2 - x) / 4,
// x = (cos 2 pi eta2 - cos 2 pi eta1) / 2.
inline double fan_default(double cos_eta1, double cos_eta2) {
  double x = 0.5 * (cos_eta2 - cos_eta1);
  return (1.0 + x) * (1.0 + x) * (2.0 - x) * 0.25;
}

// The symmetric 9-tap maximally flat lowpass of Section 5.1, written in
// closed form: H(w) = 1 + (8 sqrt2 - 15) s^3 + (14 - 8 sqrt2) s^4, s = sin^2(w/2).
std::vector<double> default_qmf_half() {
  const double r2 = std::sqrt(2.0);
  return {9.0 / 64.0 + 5.0 * r2 / 16.0, 29.0 / 64.0 - r2 / 8.0, (1.0 - r2) / 8.0,
          -13.0 / 64.0 + r2 / 8.0, 7.0 / 128.0 - r2 / 32.0};
}

}  // namespace

void parallel_run(int64_t n, const std::function<void(int64_t)> &fn) { parallel_for(n, fn); }

bool fft_size_supported(int64_t n) {
  // 2^a 3^b with a >= 2, b <= 1, 8 <= n <= 1024: the lengths the device FFT
  // is instantiated for
  static const int64_t ok[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  for (int64_t v : ok)
    if (v == n) return true;
  return false;
}

int parse_config(const sl_config *cfg, Config &c, std::string &err) {
  if (!cfg) {
    err = "config is NULL";
    return SL_EINVAL;
  }
  if (cfg->ndim != 2 && cfg->ndim != 3) {
    err = "ndim must be 2 or 3";
    return SL_EINVAL;
  }
  c.ndim = cfg->ndim;
  for (int i = 0; i < 3; ++i) c.dims[i] = i < c.ndim ? cfg->dims[i] : 1;
  for (int i = 0; i < c.ndim; ++i) {
    if (cfg->dims[i] <= 0) {
      err = "dims must be positive";
      return SL_EINVAL;
    }
    if (!fft_size_supported(cfg->dims[i])) {
      err = "each dimension must be one of 8, 12, 16, 24, ..., 512, 768, 1024 (2^a or 3*2^a)";
      return SL_EUNSUPPORTED;
    }
  }
  if (cfg->n_scales < 1 || cfg->n_scales > 6) {
    err = "n_scales must be in 1..6";
    return SL_EINVAL;
  }
  c.J = cfg->n_scales;
  if (!cfg->shear_levels) {
    err = "shear_levels is NULL";
    return SL_EINVAL;
  }
  c.levels.assign(cfg->shear_levels, cfg->shear_levels + c.J);
  for (int d : c.levels)
    if (d < 0 || d > 4) {
      err = "shear levels must be in 0..4";
      return SL_EINVAL;
    }
  if (cfg->qmf) {
    int n = cfg->qmf_len;
    if (n < 1 || n % 2 == 0 || n > 65) {
      err = "qmf length must be odd and <= 65";
      return SL_EINVAL;
    }
    int o = n / 2;
    for (int i = 0; i < o; ++i)
      if (std::fabs(cfg->qmf[i] - cfg->qmf[n - 1 - i]) > 1e-12 * (1.0 + std::fabs(cfg->qmf[i]))) {
        err = "qmf must be symmetric about its centre tap";
        return SL_EINVAL;
      }
    c.h.assign(cfg->qmf + o, cfg->qmf + n);
  } else {
    c.h = default_qmf_half();
  }
  if (cfg->dir_filter) {
    int r = cfg->dir_rows, q = cfg->dir_cols;
    if (r < 1 || q < 1 || r % 2 == 0 || q % 2 == 0 || r > 63 || q > 63) {
      err = "directional filter sizes must be odd and <= 63";
      return SL_EINVAL;
    }
    c.default_P = false;
    c.P.assign(cfg->dir_filter, cfg->dir_filter + (size_t)r * q);
    c.prow = r;
    c.pcol = q;
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < q; ++b) {
        double v = c.P[(size_t)a * q + b], w = c.P[(size_t)(r - 1 - a) * q + (q - 1 - b)];
        if (std::fabs(v - w) > 1e-12 * (1.0 + std::fabs(v))) {
          err = "directional filter must be point-symmetric";
          return SL_EINVAL;
        }
      }
  }
  c.full = cfg->full_system != 0;
  if (cfg->coeff_dtype != SL_F32 && cfg->coeff_dtype != SL_F16 && cfg->coeff_dtype != SL_BF16) {
    err = "coeff_dtype must be SL_F32, SL_F16 or SL_BF16";
    return SL_EINVAL;
  }
  c.dtype = cfg->coeff_dtype;
  return SL_OK;
}

std::vector<Subband> enumerate_subbands(const Config &c) {
  std::vector<Subband> out;
  out.push_back({0, -1, 0, 0});
  for (int j = 0; j < c.J; ++j) {
    int L = 1 << c.levels[j];
    if (c.ndim == 2) {
      for (int k = -L; k <= L; ++k) out.push_back({1, j, k, 0});
      int lo = c.full ? -L : -L + 1, hi = c.full ? L : L - 1;
      for (int k = lo; k <= hi; ++k) out.push_back({2, j, k, 0});
    } else {
      for (int p = 1; p <= 3; ++p)
        for (int k1 = -L; k1 <= L; ++k1)
          for (int k2 = -L; k2 <= L; ++k2) {
            bool keep = true;
            if (!c.full) {
              if (p == 2) keep = std::abs(k1) != L;
              if (p == 3) keep = std::abs(k1) != L && std::abs(k2) != L;
            }
            if (keep) out.push_back({p, j, k1, k2});
          }
    }
  }
  return out;
}

void g_line(const Config &c, int j, int N, double *out) {
  for (int m = 0; m < N; ++m) out[m] = g_casc(c.h, c.J - j, m, N);
}

void lowpass_line(const Config &c, int N, double *out) {
  for (int m = 0; m < N; ++m) out[m] = h_casc(c.h, c.J, m, N);
}

void phi_plane(const Config &c, int j, int k, int Nm, int Ns, double *out) {
  const int d = c.levels[j];
  const int64_t L = 1 << d;
  const int64_t a = int64_t(1) << (c.J - j - 1);
  const int64_t b = int64_t(1) << (c.J - j + d);
  const int mh = c.J - j + d;
  const int64_t D = L * Nm * Ns;    // common denominator of eta
  // tables over the eta grid t / D: h_hat_{J-j+d}(t/D) and cos(2 pi b t / D)
  std::vector<double> hcas((size_t)D), cosb;
  parallel_for((D + 4095) / 4096, [&](int64_t blk) {
    int64_t t0 = blk * 4096, t1 = std::min(D, t0 + 4096);
    for (int64_t t = t0; t < t1; ++t) hcas[t] = h_casc(c.h, mh, t, D);
  });
  if (c.default_P) {
    cosb.resize((size_t)D);
    parallel_for((D + 4095) / 4096, [&](int64_t blk) {
      int64_t t0 = blk * 4096, t1 = std::min(D, t0 + 4096);
      for (int64_t t = t0; t < t1; ++t) cosb[t] = cos2pi(b * t, D);
    });
  }
  const int po2 = c.prow / 2, po1 = c.pcol / 2;
  parallel_for(Nm, [&](int64_t mm) {
    std::vector<double> wr((size_t)L);
    for (int64_t r = 0; r < L; ++r) {
      double v = h_casc(c.h, d, mm + r * Nm, L * Nm);   // h_hat_d((xi_m + r)/L)
      wr[r] = v * v;
    }
    const double ca = cos2pi(a * mm, Nm);
    for (int ms = 0; ms < Ns; ++ms) {
      double sum = 0.0;
      for (int64_t r = 0; r < L; ++r) {
        int64_t eta = pmod(L * Nm * ms - (int64_t)k * Ns * (mm + r * Nm), D);
        double Pv;
        if (c.default_P) {
          Pv = fan_default(ca, cosb[eta]);
        } else {
          Pv = 0.0;
          for (int r2 = 0; r2 < c.prow; ++r2)
            for (int r1 = 0; r1 < c.pcol; ++r1) {
              double tap = c.P[(size_t)r2 * c.pcol + r1];
              if (tap == 0.0) continue;
              int64_t n1 = r1 - po1, n2 = r2 - po2;
              int64_t ph = pmod(n1 * a * mm * L * Ns, D) + pmod(n2 * b * eta, D);
              Pv += tap * cos2pi(ph, D);
            }
        }
        sum += wr[r] * Pv * hcas[eta];
      }
      out[(size_t)ms * Nm + mm] = sum;
    }
  });
}

int Tables3D::find(int j, int k, int main_axis, int sec_axis) const {
  for (size_t i = 0; i < keys.size(); ++i)
    if (keys[i].j == j && keys[i].k == k && keys[i].main_axis == main_axis &&
        keys[i].sec_axis == sec_axis)
      return (int)i;
  return -1;
}

void build_tables_3d(const Config &c, Tables3D &t) {
  t.keys.clear();
  t.planes.clear();
  t.g.assign((size_t)c.J * 3, {});
  t.low.assign(3, {});
  for (int ax = 1; ax <= 3; ++ax) {
    t.low[ax - 1].resize(c.n(ax));
    lowpass_line(c, c.n(ax), t.low[ax - 1].data());
  }
  // (main, secondary) combinations used by pyramids 1..3
  const int combos[6][2] = {{1, 2}, {1, 3}, {2, 1}, {2, 3}, {3, 1}, {3, 2}};
  for (int j = 0; j < c.J; ++j) {
    int L = 1 << c.levels[j];
    for (int ax = 1; ax <= 3; ++ax) {
      t.g[(size_t)j * 3 + ax - 1].resize(c.n(ax));
      g_line(c, j, c.n(ax), t.g[(size_t)j * 3 + ax - 1].data());
    }
    for (auto &cb : combos)
      for (int k = -L; k <= L; ++k) {
        t.keys.push_back({j, k, cb[0], cb[1]});
        std::vector<double> pl((size_t)c.n(cb[0]) * c.n(cb[1]));
        phi_plane(c, j, k, c.n(cb[0]), c.n(cb[1]), pl.data());
        t.planes.push_back(std::move(pl));
      }
  }
}

// ---------------------------------------------------------------------------
// host FFT (recursive, radix 2/3) for the spatial l1 norms
// ---------------------------------------------------------------------------

namespace {

void dft_rec(std::complex<double> *a, int n, int N, const std::complex<double> *tab,
             std::complex<double> *scratch) {
  // tab[m] = exp(sign 2 pi i m / N); a sub-transform of length n uses the
  // twiddles with stride N / n
  if (n == 1) return;
  int p = (n % 2 == 0) ? 2 : (n % 3 == 0 ? 3 : n);
  int m = n / p;
  std::complex<double> *tmp = scratch;
  for (int i = 0; i < n; ++i) tmp[(i % p) * m + i / p] = a[i];
  if (m > 1)
    for (int q = 0; q < p; ++q) dft_rec(tmp + (size_t)q * m, m, N, tab, scratch + n);
  const int step = N / n;
  for (int k = 0; k < n; ++k) {
    std::complex<double> s = 0.0;
    for (int q = 0; q < p; ++q) s += tmp[(size_t)q * m + (k % m)] * tab[(size_t)((q * k) % n) * step];
    a[k] = s;
  }
}

}  // namespace

void host_dft_inplace(std::vector<double> &re, std::vector<double> &im, int sign) {
  int n = (int)re.size();
  std::vector<std::complex<double>> a(n), tab(n);
  for (int i = 0; i < n; ++i) a[i] = {re[i], im[i]};
  for (int i = 0; i < n; ++i) {
    double ang = sign * kTwoPi * (double)i / (double)n;
    tab[i] = {std::cos(ang), std::sin(ang)};
  }
  std::vector<std::complex<double>> scratch((size_t)n * 4 + 16);
  dft_rec(a.data(), n, n, tab.data(), scratch.data());
  for (int i = 0; i < n; ++i) {
    re[i] = a[i].real();
    im[i] = a[i].imag();
  }
}

namespace {

// l1 norm of the real spatial filter whose DFT is the real array hat [N2][N1].
double spatial_l1_2d(const double *hat, int N2, int N1) {
  std::vector<double> re(hat, hat + (size_t)N2 * N1), im((size_t)N2 * N1, 0.0);
  std::vector<double> lr(N1), li(N1);
  for (int r = 0; r < N2; ++r) {
    for (int x = 0; x < N1; ++x) {
      lr[x] = re[(size_t)r * N1 + x];
      li[x] = im[(size_t)r * N1 + x];
    }
    host_dft_inplace(lr, li, +1);
    for (int x = 0; x < N1; ++x) {
      re[(size_t)r * N1 + x] = lr[x];
      im[(size_t)r * N1 + x] = li[x];
    }
  }
  std::vector<double> cr(N2), ci(N2);
  double l1 = 0.0;
  for (int x = 0; x < N1; ++x) {
    for (int r = 0; r < N2; ++r) {
      cr[r] = re[(size_t)r * N1 + x];
      ci[r] = im[(size_t)r * N1 + x];
    }
    host_dft_inplace(cr, ci, +1);
    for (int r = 0; r < N2; ++r) l1 += std::fabs(cr[r]);
  }
  return l1 / ((double)N1 * N2);
}

double spatial_l1_1d(const double *hat, int N) {
  std::vector<double> re(hat, hat + N), im(N, 0.0);
  host_dft_inplace(re, im, +1);
  double l1 = 0.0;
  for (int i = 0; i < N; ++i) l1 += std::fabs(re[i]);
  return l1 / N;
}

}  // namespace

int build_wavelet_bank(const Config &c, Bank &bank, double *filters_out, std::string &err) {
  if (c.ndim != 2) {
    err = "the wavelet bank is two-dimensional";
    return SL_EINVAL;
  }
  const int N2 = (int)c.dims[0], N1 = (int)c.dims[1];
  const int64_t npix = c.npix();
  bank.subbands.clear();
  bank.subbands.push_back({0, -1, 0, 0});
  for (int j = 0; j < c.J; ++j)
    for (int cone = 1; cone <= 3; ++cone) bank.subbands.push_back({cone, j, 0, 0});
  const int R = (int)bank.subbands.size();
  bank.l2.assign(R, 0.0);
  bank.l1.assign(R, 0.0);
  bank.dual.assign((size_t)npix, 0.0);
  std::vector<double> a1(N1), a2(N2), b1(N1), b2(N2), plane((size_t)npix);
  for (int i = 0; i < R; ++i) {
    const Subband &sb = bank.subbands[i];
    const int m = sb.cone == 0 ? c.J : c.J - sb.j;
    // factor along x1 (a1) and along x2 (a2)
    for (int x = 0; x < N1; ++x) {
      const double h = h_casc(c.h, m, x, N1);
      const double g = sb.cone == 0 ? 0.0 : g_casc(c.h, m, x, N1);
      a1[x] = (sb.cone == 1 || sb.cone == 3) ? g : h;
      b1[x] = h;
    }
    for (int y = 0; y < N2; ++y) {
      const double h = h_casc(c.h, m, y, N2);
      const double g = sb.cone == 0 ? 0.0 : g_casc(c.h, m, y, N2);
      a2[y] = (sb.cone == 2 || sb.cone == 3) ? g : h;
      b2[y] = h;
    }
    double ss = 0.0;
    for (int y = 0; y < N2; ++y)
      for (int x = 0; x < N1; ++x) {
        const double v = a2[y] * a1[x];
        plane[(size_t)y * N1 + x] = v;
        ss += v * v;
        bank.dual[(size_t)y * N1 + x] += v * v;
      }
    bank.l2[i] = std::sqrt(ss / (double)npix);
    // separable: the l1 norm of the spatial filter is the product of the
    // factors' l1 norms
    bank.l1[i] = spatial_l1_1d(a1.data(), N1) * spatial_l1_1d(a2.data(), N2);
    if (filters_out) std::copy(plane.begin(), plane.end(), filters_out + (size_t)i * npix);
  }
  bank.dual_min = *std::min_element(bank.dual.begin(), bank.dual.end());
  bank.dual_max = *std::max_element(bank.dual.begin(), bank.dual.end());
  if (!(bank.dual_min > 1e-6 * bank.dual_max)) {
    err = "Psi_hat is not bounded away from zero (min/max < 1e-6)";
    return SL_EILLCOND;
  }
  return SL_OK;
}

int build_bank(const Config &c, Bank &bank, double *filters_out, std::string &err) {
  bank.subbands = enumerate_subbands(c);
  const int R = (int)bank.subbands.size();
  const int64_t npix = c.npix();
  bank.l2.assign(R, 0.0);
  bank.l1.assign(R, 0.0);
  bank.dual.assign((size_t)npix, 0.0);
  if (c.ndim == 2) {
    const int N2 = (int)c.dims[0], N1 = (int)c.dims[1];
    std::vector<double> low1(N1), low2(N2);
    lowpass_line(c, N1, low1.data());
    lowpass_line(c, N2, low2.data());
    std::vector<double> plane((size_t)npix), tmp((size_t)npix), g1(N1), g2(N2);
    for (int i = 0; i < R; ++i) {
      const Subband &s = bank.subbands[i];
      if (s.cone == 0) {
        for (int r = 0; r < N2; ++r)
          for (int x = 0; x < N1; ++x) plane[(size_t)r * N1 + x] = low2[r] * low1[x];
      } else if (s.cone == 1) {
        phi_plane(c, s.j, s.k1, N1, N2, tmp.data());          // [xi2][xi1]
        g_line(c, s.j, N1, g1.data());
        for (int r = 0; r < N2; ++r)
          for (int x = 0; x < N1; ++x) plane[(size_t)r * N1 + x] = g1[x] * tmp[(size_t)r * N1 + x];
      } else {
        phi_plane(c, s.j, s.k1, N2, N1, tmp.data());          // [xi1][xi2]
        g_line(c, s.j, N2, g2.data());
        for (int r = 0; r < N2; ++r)
          for (int x = 0; x < N1; ++x) plane[(size_t)r * N1 + x] = g2[r] * tmp[(size_t)x * N2 + r];
      }
      double ss = 0.0;
      for (int64_t p = 0; p < npix; ++p) {
        ss += plane[p] * plane[p];
        bank.dual[p] += plane[p] * plane[p];
      }
      bank.l2[i] = std::sqrt(ss / (double)npix);
      if (filters_out) {
        std::copy(plane.begin(), plane.end(), filters_out + (size_t)i * npix);
      } else {
        bank.l1[i] = spatial_l1_2d(plane.data(), N2, N1);
      }
    }
    if (filters_out)
      parallel_for(R, [&](int64_t i) {
        bank.l1[i] = spatial_l1_2d(filters_out + (size_t)i * npix, N2, N1);
      });
  } else {
    Tables3D t;
    build_tables_3d(c, t);
    const int N3 = c.n(3), N2 = c.n(2), N1 = c.n(1);
    // l1 norms of the factors (1D g / lowpass lines and Phi planes)
    std::vector<double> plane_l1(t.planes.size());
    parallel_for((int64_t)t.planes.size(), [&](int64_t q) {
      const auto &key = t.keys[q];
      plane_l1[q] = spatial_l1_2d(t.planes[q].data(), c.n(key.sec_axis), c.n(key.main_axis));
    });
    for (int i = 0; i < R; ++i) {
      const Subband &s = bank.subbands[i];
      // value(xi3, xi2, xi1) = A(main) * B(main, sec1) * C(main, sec2)
      auto axis_of = [&](int p, int which) {   // which: 0 main, 1 sec1, 2 sec2
        static const int ax[4][3] = {{0, 0, 0}, {1, 2, 3}, {2, 1, 3}, {3, 1, 2}};
        return ax[p][which];
      };
      std::vector<double> vol((size_t)npix);
      if (s.cone == 0) {
        const auto &l1v = t.low[0], &l2v = t.low[1], &l3v = t.low[2];
        for (int z = 0; z < N3; ++z)
          for (int y = 0; y < N2; ++y)
            for (int x = 0; x < N1; ++x)
              vol[((size_t)z * N2 + y) * N1 + x] = l3v[z] * l2v[y] * l1v[x];
        bank.l1[i] = spatial_l1_1d(l1v.data(), N1) * spatial_l1_1d(l2v.data(), N2) *
                     spatial_l1_1d(l3v.data(), N3);
      } else {
        int am = axis_of(s.cone, 0), a1 = axis_of(s.cone, 1), a2 = axis_of(s.cone, 2);
        int q1 = t.find(s.j, s.k1, am, a1), q2 = t.find(s.j, s.k2, am, a2);
        const auto &gv = t.g[(size_t)s.j * 3 + am - 1];
        const auto &P1 = t.planes[q1], &P2 = t.planes[q2];
        const int Nm = c.n(am);
        int idx[4];
        for (int z = 0; z < N3; ++z)
          for (int y = 0; y < N2; ++y)
            for (int x = 0; x < N1; ++x) {
              idx[1] = x;
              idx[2] = y;
              idx[3] = z;
              int im = idx[am], i1 = idx[a1], i2 = idx[a2];
              vol[((size_t)z * N2 + y) * N1 + x] =
                  gv[im] * P1[(size_t)i1 * Nm + im] * P2[(size_t)i2 * Nm + im];
            }
        bank.l1[i] = spatial_l1_1d(gv.data(), Nm) * plane_l1[q1] * plane_l1[q2];
      }
      double ss = 0.0;
      for (int64_t p = 0; p < npix; ++p) {
        ss += vol[p] * vol[p];
        bank.dual[p] += vol[p] * vol[p];
      }
      bank.l2[i] = std::sqrt(ss / (double)npix);
      if (filters_out) std::copy(vol.begin(), vol.end(), filters_out + (size_t)i * npix);
    }
  }
  bank.dual_min = *std::min_element(bank.dual.begin(), bank.dual.end());
  bank.dual_max = *std::max_element(bank.dual.begin(), bank.dual.end());
  if (!(bank.dual_min > 1e-6 * bank.dual_max)) {
    err = "Psi_hat is not bounded away from zero (min/max < 1e-6)";
    return SL_EILLCOND;
  }
  return SL_OK;
}

}  // namespace slh
