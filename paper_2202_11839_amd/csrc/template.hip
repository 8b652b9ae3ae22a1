// The plain window-convolved template path (Sec. III.B, eq.
// window_convolution_X_hankel): for every parameter point the model
// multipoles are taken to configuration space by H^{-1}, multiplied by the
// window mixing Q^X_{l l'}(r) (eq. def_of_Q_llp) and taken back by H_l, each
// transform an FFTLog (Hamilton 2000) of length n_log in FP64 on the device,
// one workgroup per transform.  The output families are the density auto
// spectrum (its quadrupole is the leakage moment of Sec. IV.C), the
// shape-density cross spectrum, and the plus and minus shape spectra
// (eq. all_convolutions and the leakage equations).
//
// FFTLog: with x_n = x_0 e^{n d} and u_n = f(x_n) x_n^{3-q}, c = DFT[u],
// G(y_j) = int f(x) j_l(x y_j) x^2 dx = y_j^{-q} DFT[c_m C_m](j), y_j = 1 / x_{N-1-j},
// C_m = M_l(q + i w_m) (x_0 y_0)^{-i w_m} / N, w_m = 2 pi m' / (N d) (m' the
// signed frequency), M_l(s) = int t^{s-1} j_l(t) dt = sqrt(pi) 2^{s-2}
// Gamma((l+s)/2) / Gamma((3+l-s)/2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <vector>

#include "device_common.h"

namespace lpp {

double window_coefficient(int mX, int l, int lp, int lpp);

namespace {

using cd = std::complex<double>;
using dev::V2;

constexpr int kLog = 4096;          // FFTLog length
constexpr int kLogThreads = kLog / 8;
constexpr int kMaxKOut = 256;
constexpr int kChunk = 2048;        // parameter points per pass (bounds the xi scratch)
constexpr int kMaxRows = 9;         // output multipoles per point (all four families)
constexpr int kMaxQc = 23;          // window-mixing rows Q^X_{l l'} (9 + 4 + 9 + 1)

// ---- host: special functions ----

// log Gamma(z), Re z > 0: recurrence up to Re z >= 12, then Stirling's series
cd lgamma_c(cd z) {
  cd shift = 0.0;
  while (z.real() < 12.0) {
    shift += std::log(z);
    z += 1.0;
  }
  static const double B[] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730, 7.0 / 6};
  cd s = (z - 0.5) * std::log(z) - z + 0.5 * std::log(2.0 * M_PI);
  cd zp = z;
  const cd z2 = z * z;
  for (int k = 1; k <= 7; ++k) {
    s += B[k - 1] / (2.0 * k * (2.0 * k - 1.0) * zp);
    zp *= z2;
  }
  return s - shift;
}

cd mellin_jl(int l, cd s) {
  return std::exp(0.5 * std::log(M_PI) + (s - 2.0) * std::log(2.0) + lgamma_c(0.5 * (l + s.real()) + cd(0, 0.5 * s.imag())) -
                  lgamma_c(cd(0.5 * (3.0 + l - s.real()), -0.5 * s.imag())));
}

long double fact(int n) {
  long double r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// Wigner 3j symbol (Racah's sum), integer arguments
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0 || j3 < std::abs(j1 - j2) || j3 > j1 + j2 || std::abs(m1) > j1 || std::abs(m2) > j2 ||
      std::abs(m3) > j3)
    return 0.0;
  const long double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
  const long double pre = std::sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                                    fact(j3 + m3) * fact(j3 - m3));
  long double sum = 0;
  for (int k = 0; k <= j1 + j2 + j3; ++k) {
    const int a[6] = {k, j3 - j2 + k + m1, j3 - j1 + k - m2, j1 + j2 - j3 - k, j1 - k - m1, j2 - k + m2};
    bool ok = true;
    for (int v : a) ok = ok && v >= 0;
    if (!ok) continue;
    long double den = 1;
    for (int v : a) den *= fact(v);
    sum += ((k % 2) ? -1.0L : 1.0L) / den;
  }
  const int sgn = ((j1 - j2 - m3) % 2 + 2) % 2 ? -1 : 1;
  return static_cast<double>(sgn * pre * sum);
}

// ---- output families ----

enum Family { FAM_DD = 0, FAM_GD = 1, FAM_PLUS = 2, FAM_MINUS = 3 };

// Multipoles of one family (l), the model multipoles it is built from (l'),
// and the m of its window mixing (eq. def_of_Q_llp).
struct FamilyDef {
  int mX, nl, l0;  // l = l0, l0 + 2, ..., and l' over the same list
};
constexpr FamilyDef kFam[4] = {{0, 3, 0}, {2, 2, 2}, {0, 3, 0}, {4, 1, 4}};

// Which transforms a call runs: output row o is multipole rl[o] of family
// rf[o]; its sum over l' uses the inverse transforms xi0[o] .. xi0[o]+nxi[o]-1
// and the mixing rows qc0[o] .. qc0[o]+nxi[o]-1; inverse transform x is the
// model multipole xl[x] of family xf[x].
struct Rows {
  int n_out, n_xi;
  int rf[kMaxRows], rl[kMaxRows], xi0[kMaxRows], nxi[kMaxRows], qc0[kMaxRows];
  int xf[kMaxRows], xl[kMaxRows];
};

Rows make_rows(const int* fams, int nfam) {
  Rows R{};
  int qc = 0;
  for (int i = 0; i < nfam; ++i) {
    const FamilyDef& F = kFam[fams[i]];
    const int x0 = R.n_xi;
    for (int b = 0; b < F.nl; ++b) {
      R.xf[R.n_xi] = fams[i];
      R.xl[R.n_xi] = F.l0 + 2 * b;
      ++R.n_xi;
    }
    for (int a = 0; a < F.nl; ++a) {
      const int o = R.n_out++;
      R.rf[o] = fams[i];
      R.rl[o] = F.l0 + 2 * a;
      R.xi0[o] = x0;
      R.nxi[o] = F.nl;
      R.qc0[o] = qc;
      qc += F.nl;
    }
  }
  return R;
}

// ---- device: one FFTLog per workgroup ----

struct LogTables {
  const double2* tw;     // exp(-2 pi i m / N)
  const double2* cinv;   // [3][N] C_m of H^{-1}_l, l = 0, 2, 4 (bias q_inv)
  const double2* cfwd;   // [3][N] C_m of H_l (bias q_fwd(l))
  const double* pd;      // P_fid(k) exp(-(k/10)^2)
  const double* kpow;    // k^{3 - q_inv}
  const double* rpow;    // r^{-q_inv}
  const double* rpowf;   // [3][N] r^{3 - q_fwd(l)}
  const double* kpowf;   // [3][N] k^{-q_fwd(l)}
  const double* qc;      // [rows][N] Q^X_{l l'}(r), in the order of Rows::qc0
};

// v: this thread's 8 inputs (element t + j N/8).  Returns with v[q] the
// output at row fft_rows(t)[q].
__device__ __forceinline__ void log_fft(double2* sm, const double2* tw, int t, double2* v) {
  dev::fft_column_regs<double, kLog>(tw, sm, 0, t, v);
}

// second half of an FFTLog: c (from log_fft, at rows) times C, then the DFT,
// with the output written to sm[j] (real part times the caller's scale later)
__device__ __forceinline__ void log_second(double2* sm, const double2* tw, const double2* C, int t, double2* v) {
  int row[8];
  dev::fft_rows<kLog>(t, row);
#pragma unroll
  for (int q = 0; q < 8; ++q) sm[row[q]] = dev::cmul(v[q], C[row[q]]);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = sm[t + j * kLogThreads];
  __syncthreads();
  dev::fft_column_regs<double, kLog>(tw, sm, 0, t, v);
#pragma unroll
  for (int q = 0; q < 8; ++q) sm[row[q]] = v[q];
  __syncthreads();
}

// The model multipole l of family fam per unit P_fid (Sec. IV.C model with
// Kaiser density and linear alignment shapes): s = sigma8 / sigma8_fid,
//   dd:    s^2 {b^2 + 2bf/3 + f^2/5, 4bf/3 + 4f^2/7, 8f^2/35}      (l = 0, 2, 4)
//   gd:    A s^2 {-(7b+f)/42, -f/105}                               (L = 2, 4)
//   plus:  A^2 s^2 {2/15, -4/21, 2/35}                              (l = 0, 2, 4)
//   minus: A^2 s^2 / 420                                            (L = 4)
__device__ __forceinline__ double model_amplitude(const double* p, double s8f, int fam, int l) {
  const double A = p[0], b = p[1], f = p[2], s = p[3] / s8f;
  const double s2 = s * s;
  switch (fam) {
    case FAM_DD:
      return s2 * (l == 0 ? b * b + 2.0 * b * f / 3.0 + f * f / 5.0
                          : (l == 2 ? 4.0 * b * f / 3.0 + 4.0 * f * f / 7.0 : 8.0 * f * f / 35.0));
    case FAM_GD:
      return A * s2 * (l == 2 ? -(7.0 * b + f) / 42.0 : -f / 105.0);
    case FAM_PLUS:
      return A * A * s2 * (l == 0 ? 2.0 / 15.0 : (l == 2 ? -4.0 / 21.0 : 2.0 / 35.0));
    default:
      return A * A * s2 / 420.0;
  }
}

// xi[p][x][j]: the inverse transform x of point p (Rows::xf, xl)
__global__ void __launch_bounds__(kLogThreads) fftlog_inverse_kernel(LogTables tb, Rows R,
                                                                     const double* __restrict__ params, double s8f,
                                                                     double* __restrict__ xi) {
  __shared__ double2 sm[kLog];
  const int p = blockIdx.x / R.n_xi, x = blockIdx.x % R.n_xi, t = threadIdx.x;
  const int l = R.xl[x];
  const double amp = model_amplitude(params + 5 * static_cast<int64_t>(p), s8f, R.xf[x], l);
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int n = t + j * kLogThreads;
    v[j] = double2{amp * tb.pd[n] * tb.kpow[n], 0.0};
  }
  log_fft(sm, tb.tw, t, v);
  log_second(sm, tb.tw, tb.cinv + (l / 2) * kLog, t, v);
  const double sign = (l / 2) % 2 ? -1.0 : 1.0;
  double* out = xi + (static_cast<int64_t>(p) * R.n_xi + x) * kLog;
  for (int j = t; j < kLog; j += kLogThreads) out[j] = sign * sm[j].x * tb.rpow[j] / (2.0 * M_PI * M_PI);
}

// out[p][o][i]: output row o (Rows::rf, rl) at kout (linear in ln k); the
// plus monopole carries the shot-noise term
__global__ void __launch_bounds__(kLogThreads) fftlog_forward_kernel(LogTables tb, Rows R,
                                                                     const double* __restrict__ xi,
                                                                     const double* __restrict__ params, double lnk0,
                                                                     double dlnk, const double* __restrict__ lnkout,
                                                                     int nk, double shot, double* __restrict__ out) {
  __shared__ double2 sm[kLog];
  const int p = blockIdx.x / R.n_out, o = blockIdx.x % R.n_out, t = threadIdx.x;
  const int l = R.rl[o];
  const double* xp = xi + (static_cast<int64_t>(p) * R.n_xi + R.xi0[o]) * kLog;
  const double* qp = tb.qc + static_cast<int64_t>(R.qc0[o]) * kLog;
  const int nx = R.nxi[o];
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int n = t + j * kLogThreads;
    double g = 0.0;
    for (int lp = 0; lp < nx; ++lp) g += qp[lp * kLog + n] * xp[lp * kLog + n];
    v[j] = double2{g * tb.rpowf[(l / 2) * kLog + n], 0.0};
  }
  log_fft(sm, tb.tw, t, v);
  log_second(sm, tb.tw, tb.cfwd + (l / 2) * kLog, t, v);
  const double sign = (l / 2) % 2 ? -1.0 : 1.0;
  for (int j = t; j < kLog; j += kLogThreads) sm[j].y = sign * 4.0 * M_PI * sm[j].x * tb.kpowf[(l / 2) * kLog + j];
  __syncthreads();
  const bool noisy = R.rf[o] == FAM_PLUS && l == 0;
  for (int i = t; i < nk; i += kLogThreads) {
    const double u = (lnkout[i] - lnk0) / dlnk;
    int j0 = static_cast<int>(floor(u));
    j0 = j0 < 0 ? 0 : (j0 > kLog - 2 ? kLog - 2 : j0);
    const double w = u - j0;
    double v2 = (1.0 - w) * sm[j0].y + w * sm[j0 + 1].y;
    if (noisy) v2 += shot * params[5 * static_cast<int64_t>(p) + 4];
    out[(static_cast<int64_t>(p) * R.n_out + o) * nk + i] = v2;
  }
}

// ---- host ----

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc(&p, n * sizeof(T)); }
};

// Device memory of one call: the tables (uploaded per call), the xi of up to
// `chunk` points, and (host I/O) staging for their parameters and outputs.
struct TemplateMem {
  double2 *tw, *ci, *cf;
  double *pd, *kp, *rp, *rpf, *kpf, *qc, *lk, *xi, *par, *out;
  int64_t chunk;
};

// doubles of the tables of a call with n_k outputs per multipole
constexpr size_t table_doubles(int n_k) {
  return (2 + 6 + 6 + 3 + 6 + static_cast<size_t>(kMaxQc)) * kLog + static_cast<size_t>(n_k);
}
// doubles per parameter point: its xi, and its staged parameters and outputs
constexpr size_t point_doubles(int n_xi, int n_out, int n_k) {
  return static_cast<size_t>(n_xi) * kLog + 5 + static_cast<size_t>(n_out) * n_k;
}

// Carve the memory of a call out of one device block of `dbl` doubles
// (256-byte aligned pieces); false if it holds no point.
bool carve(double* base, size_t dbl, const Rows& R, int n_k, int64_t want_chunk, TemplateMem& m) {
  auto up = [](size_t v) { return (v + 31) / 32 * 32; };  // 32 doubles = 256 bytes
  const size_t fixed = up(2 * kLog) + 2 * up(6 * kLog) + 3 * up(kLog) + 2 * up(3 * kLog) +
                       up(static_cast<size_t>(kMaxQc) * kLog) + up(n_k);
  if (dbl <= fixed) return false;
  const size_t per = point_doubles(R.n_xi, R.n_out, n_k) + 64;
  int64_t chunk = static_cast<int64_t>((dbl - fixed) / per);
  chunk = std::min<int64_t>(chunk, want_chunk);
  if (chunk < 1) return false;
  size_t o = 0;
  auto take = [&](size_t n) {
    double* q = base + o;
    o += up(n);
    return q;
  };
  m.tw = reinterpret_cast<double2*>(take(2 * kLog));
  m.ci = reinterpret_cast<double2*>(take(6 * kLog));
  m.cf = reinterpret_cast<double2*>(take(6 * kLog));
  m.pd = take(kLog);
  m.kp = take(kLog);
  m.rp = take(kLog);
  m.rpf = take(3 * kLog);
  m.kpf = take(3 * kLog);
  m.qc = take(static_cast<size_t>(kMaxQc) * kLog);
  m.lk = take(n_k);
  m.xi = take(static_cast<size_t>(chunk) * R.n_xi * kLog);
  m.par = take(5 * static_cast<size_t>(chunk));
  m.out = take(static_cast<size_t>(chunk) * R.n_out * n_k);
  m.chunk = chunk;
  return o <= dbl;
}

}  // namespace

// Device scratch of the allocation-free variant (lpp_template_plain_noalloc):
// 24 MiB on every device the library runs on, held until the process ends.
// In host code its name is a host-side stand-in, not a device address: the
// address is looked up per device with hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(24) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

lpp_status scratch_address(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return LPP_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return LPP_E_DEVICE;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return LPP_OK;
}

lpp_status check_args(const double* pfid, double k_min, double k_max, int32_t n_log, const double* r_q,
                      const double* Q, int32_t n_q, const double* params, int64_t n_pts, const double* k_out,
                      int32_t n_k, double nbar, double sigma_gamma, const double* out) {
  if (!pfid || !r_q || !Q || !params || !k_out || !out || n_q < 1 || n_pts < 0 || n_k < 1 || n_k > kMaxKOut)
    return LPP_E_INVALID;
  if (n_log != kLog) return LPP_E_UNSUPPORTED;
  if (!(k_min > 0.0) || !(k_max > k_min) || !(nbar > 0.0) || !std::isfinite(sigma_gamma)) return LPP_E_INVALID;
  for (int i = 1; i < n_q; ++i)
    if (!(r_q[i] > r_q[i - 1])) return LPP_E_INVALID;
  if (!(r_q[0] > 0.0)) return LPP_E_INVALID;
  for (int i = 0; i < n_k; ++i)
    if (!(k_out[i] >= k_min) || !(k_out[i] <= k_max)) return LPP_E_INVALID;
  return LPP_OK;
}

// One call: host tables, upload into m, then the two kernels per chunk of
// points.  `m` is either freshly allocated or the static scratch.
lpp_status run_template(const Rows& R, const TemplateMem& m, const double* pfid, double k_min, double k_max,
                        const double* r_q, const double* Q, int32_t n_q, const double* params, int64_t n_pts,
                        const double* k_out, int32_t n_k, double nbar, double sigma_gamma, double* out,
                        int32_t device_io, hipStream_t st) {
  const int N = kLog;
  const double lnk0 = std::log(k_min), d = (std::log(k_max) - lnk0) / (kLog - 1);
  std::vector<double> k(N), r(N);
  for (int n = 0; n < N; ++n) k[n] = std::exp(lnk0 + n * d);
  for (int j = 0; j < N; ++j) r[j] = 1.0 / k[N - 1 - j];
  // sigma8 of P_fid: trapezoid in ln k of k^3 P W_TH(8k)^2 / (2 pi^2)
  double s8 = 0.0;
  auto integrand = [&](int n) {
    const double x = 8.0 * k[n];
    const double w = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
    return k[n] * k[n] * k[n] * pfid[n] * w * w / (2.0 * M_PI * M_PI);
  };
  for (int n = 0; n + 1 < N; ++n) s8 += 0.5 * (integrand(n) + integrand(n + 1)) * (std::log(k[n + 1]) - std::log(k[n]));
  const double s8f = std::sqrt(s8);
  // host tables
  const double qinv = 1.5;
  auto qfwd = [](int l) { return l == 0 ? 1.0 : 0.5; };
  std::vector<double2> tw(N), cinv(3 * N), cfwd(3 * N);
  for (int m2 = 0; m2 < N; ++m2) {
    const double a = -2.0 * M_PI * m2 / N;
    tw[m2] = double2{std::cos(a), std::sin(a)};
  }
  const double x0y0 = k[0] / k[N - 1];  // (k_0 r_0) = (r_0 k_0) = k_0 / k_{N-1}
  for (int li = 0; li < 3; ++li) {
    const int l = 2 * li;
    for (int m2 = 0; m2 < N; ++m2) {
      const int ms = m2 < N / 2 ? m2 : m2 - N;
      const double w = 2.0 * M_PI * ms / (N * d);
      const cd ph = std::exp(cd(0, -w * std::log(x0y0))) / static_cast<double>(N);
      const cd ci = mellin_jl(l, cd(qinv, w)) * ph, cf = mellin_jl(l, cd(qfwd(l), w)) * ph;
      cinv[li * N + m2] = double2{ci.real(), ci.imag()};
      cfwd[li * N + m2] = double2{cf.real(), cf.imag()};
    }
  }
  std::vector<double> pd(N), kpow(N), rpow(N), rpowf(3 * N), kpowf(3 * N);
  for (int n = 0; n < N; ++n) {
    pd[n] = pfid[n] * std::exp(-(k[n] / 10.0) * (k[n] / 10.0));
    kpow[n] = std::pow(k[n], 3.0 - qinv);
    rpow[n] = std::pow(r[n], -qinv);
    for (int li = 0; li < 3; ++li) {
      rpowf[li * N + n] = std::pow(r[n], 3.0 - qfwd(2 * li));
      kpowf[li * N + n] = std::pow(k[n], -qfwd(2 * li));
    }
  }
  // Q_l on the r grid: linear in r, Q(0) = (1, 0, ...), zero beyond the table
  std::vector<double> qg(5 * static_cast<size_t>(N), 0.0);
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < N; ++j) {
      const double x = r[j];
      double v = 0.0;
      if (x <= r_q[n_q - 1]) {
        if (x < r_q[0]) {
          const double y0 = i == 0 ? 1.0 : 0.0;
          v = y0 + (Q[i * n_q] - y0) * (x / r_q[0]);
        } else {
          const int hi = static_cast<int>(std::upper_bound(r_q, r_q + n_q, x) - r_q);
          const int lo = std::max(0, hi - 1);
          const int h2 = std::min(hi, n_q - 1);
          const double t = h2 > lo ? (x - r_q[lo]) / (r_q[h2] - r_q[lo]) : 0.0;
          v = Q[i * n_q + lo] + t * (Q[i * n_q + h2] - Q[i * n_q + lo]);
        }
      }
      qg[static_cast<size_t>(i) * N + j] = v;
    }
  // Q^X_{l l'}(r) = sum_{l''} c(mX, l, l', l'') Q_{l''}(r), one row per (output, l')
  int n_qc = 0;
  for (int o = 0; o < R.n_out; ++o) n_qc += R.nxi[o];
  std::vector<double> qc(static_cast<size_t>(n_qc) * N, 0.0);
  for (int o = 0; o < R.n_out; ++o) {
    const int mX = kFam[R.rf[o]].mX;
    for (int b = 0; b < R.nxi[o]; ++b) {
      const int slot = R.qc0[o] + b, lp = R.xl[R.xi0[o] + b];
      for (int i = 0; i < 5; ++i) {
        const double c = window_coefficient(mX, R.rl[o], lp, 2 * i);
        if (c == 0.0) continue;
        for (int j = 0; j < N; ++j) qc[static_cast<size_t>(slot) * N + j] += c * qg[static_cast<size_t>(i) * N + j];
      }
    }
  }
  std::vector<double> lnkout(n_k);
  for (int i = 0; i < n_k; ++i) lnkout[i] = std::log(k_out[i]);
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  if (up(m.tw, tw.data(), 16 * N) || up(m.ci, cinv.data(), 16 * 3 * N) || up(m.cf, cfwd.data(), 16 * 3 * N) ||
      up(m.pd, pd.data(), 8 * N) || up(m.kp, kpow.data(), 8 * N) || up(m.rp, rpow.data(), 8 * N) ||
      up(m.rpf, rpowf.data(), 8 * 3 * N) || up(m.kpf, kpowf.data(), 8 * 3 * N) ||
      up(m.qc, qc.data(), 8 * static_cast<size_t>(n_qc) * N) || up(m.lk, lnkout.data(), 8 * n_k))
    return LPP_E_DEVICE;
  LogTables tb{m.tw, m.ci, m.cf, m.pd, m.kp, m.rp, m.rpf, m.kpf, m.qc};
  const double shot = 2.0 * sigma_gamma * sigma_gamma / nbar;
  for (int64_t p0 = 0; p0 < n_pts; p0 += m.chunk) {
    const int np = static_cast<int>(std::min<int64_t>(m.chunk, n_pts - p0));
    const double* par = device_io ? params + 5 * p0 : m.par;
    double* o = device_io ? out + p0 * R.n_out * n_k : m.out;
    if (!device_io && up(m.par, params + 5 * p0, 8 * 5 * static_cast<size_t>(np))) return LPP_E_DEVICE;
    fftlog_inverse_kernel<<<np * R.n_xi, kLogThreads, 0, st>>>(tb, R, par, s8f, m.xi);
    fftlog_forward_kernel<<<np * R.n_out, kLogThreads, 0, st>>>(tb, R, m.xi, par, lnk0, d, m.lk, n_k, shot, o);
    if (hipGetLastError() != hipSuccess) return LPP_E_DEVICE;
    if (!device_io && hipMemcpyAsync(out + p0 * R.n_out * n_k, m.out, 8 * static_cast<size_t>(np) * R.n_out * n_k,
                                     hipMemcpyDeviceToHost, st) != hipSuccess)
      return LPP_E_DEVICE;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return LPP_E_DEVICE;
  return LPP_OK;
}

// The allocating path: one device block per call, released on return.
lpp_status template_alloc(const Rows& R, const double* pfid, double k_min, double k_max, int32_t n_log,
                          const double* r_q, const double* Q, int32_t n_q, const double* params, int64_t n_pts,
                          const double* k_out, int32_t n_k, double nbar, double sigma_gamma, double* out,
                          int32_t device_io, void* stream) {
  const lpp_status s0 =
      check_args(pfid, k_min, k_max, n_log, r_q, Q, n_q, params, n_pts, k_out, n_k, nbar, sigma_gamma, out);
  if (s0 != LPP_OK || n_pts == 0) return s0;
  try {
    const int64_t chunk = std::min<int64_t>(n_pts, kChunk);
    const size_t dbl = table_doubles(n_k) + 64 * 16 + static_cast<size_t>(chunk) * (point_doubles(R.n_xi, R.n_out, n_k) + 64);
    DevBuf<double> block;
    if (block.alloc(dbl) != hipSuccess) {
      (void)hipGetLastError();
      return LPP_E_NOMEM;
    }
    TemplateMem m{};
    if (!carve(block.p, dbl, R, n_k, chunk, m)) return LPP_E_NOMEM;
    return run_template(R, m, pfid, k_min, k_max, r_q, Q, n_q, params, n_pts, k_out, n_k, nbar, sigma_gamma, out,
                        device_io, static_cast<hipStream_t>(stream));
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

const int kFamPlain[2] = {FAM_PLUS, FAM_GD};
const int kFamAll[4] = {FAM_DD, FAM_GD, FAM_PLUS, FAM_MINUS};

}  // namespace

double window_coefficient(int mX, int l, int lp, int lpp) {
  if (l < mX || lp < mX) return 0.0;
  const double f = std::sqrt(static_cast<double>(fact(l - mX) / fact(l + mX) * (fact(lp + mX) / fact(lp - mX))));
  return (2 * l + 1) * f * wigner3j(lpp, l, lp, 0, 0, 0) * wigner3j(lpp, l, lp, 0, mX, -mX);
}

}  // namespace lpp

using namespace lpp;

extern "C" {

lpp_status lpp_window_coefficient(int32_t mX, int32_t l, int32_t lp, int32_t lpp, double* out) {
  if (!out || mX < 0 || l < 0 || lp < 0 || lpp < 0 || l > 16 || lp > 16 || lpp > 16) return LPP_E_INVALID;
  *out = window_coefficient(mX, l, lp, lpp);
  return LPP_OK;
}

lpp_status lpp_template_plain(const double* pfid, double k_min, double k_max, int32_t n_log, const double* r_q,
                              const double* Q, int32_t n_q, const double* params, int64_t n_pts,
                              const double* k_out, int32_t n_k, double nbar, double sigma_gamma, double* out,
                              int32_t device_io, void* stream) {
  return template_alloc(make_rows(kFamPlain, 2), pfid, k_min, k_max, n_log, r_q, Q, n_q, params, n_pts, k_out, n_k,
                        nbar, sigma_gamma, out, device_io, stream);
}

lpp_status lpp_template_multipoles(const double* pfid, double k_min, double k_max, int32_t n_log, const double* r_q,
                                   const double* Q, int32_t n_q, const double* params, int64_t n_pts,
                                   const double* k_out, int32_t n_k, double nbar, double sigma_gamma, double* out,
                                   int32_t device_io, void* stream) {
  return template_alloc(make_rows(kFamAll, 4), pfid, k_min, k_max, n_log, r_q, Q, n_q, params, n_pts, k_out, n_k,
                        nbar, sigma_gamma, out, device_io, stream);
}

lpp_status lpp_template_plain_noalloc(const double* pfid, double k_min, double k_max, int32_t n_log,
                                      const double* r_q, const double* Q, int32_t n_q, const double* params,
                                      int64_t n_pts, const double* k_out, int32_t n_k, double nbar,
                                      double sigma_gamma, double* out, int32_t device_io, void* stream) {
  const lpp_status s0 =
      check_args(pfid, k_min, k_max, n_log, r_q, Q, n_q, params, n_pts, k_out, n_k, nbar, sigma_gamma, out);
  if (s0 != LPP_OK) return s0;
  double* base = nullptr;
  const lpp_status s1 = scratch_address(&base);
  if (s1 != LPP_OK || n_pts == 0) return s1;
  try {
    const Rows R = make_rows(kFamPlain, 2);
    TemplateMem m{};
    if (!carve(base, kScratchBytes / sizeof(double), R, n_k, kChunk, m)) return LPP_E_WORKSPACE;
    return run_template(R, m, pfid, k_min, k_max, r_q, Q, n_q, params, n_pts, k_out, n_k, nbar, sigma_gamma, out,
                        device_io, static_cast<hipStream_t>(stream));
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

}  // extern "C"
