// Window multipoles by pair counting of randoms (Sec. III.B, eq. windowQ_ell):
//
//   Q_l(r_b) / I = (2l+1) alpha^2 sum_{i != j, pair in shell b} w_i w_j L_l(rhat_ij . dhat_ij)
//                  / (V_b I),      V_b = (4 pi / 3) ((b+1)^3 - b^3) dr^3,
//
// over the ordered pairs of a random catalog (the window W = alpha sum_r w_r
// delta_D(x - x_r) of the estimator), with the pair's line of sight dhat
// either the direction of its midpoint (the paper's "direction toward the
// pair") or of its first point (the end point, the line of sight of the LPP
// estimator and of the FFT route of lpp_window_multipoles).  Shell b holds
// (b dr)^2 <= r^2 < ((b+1) dr)^2, decided on r^2 = dx*dx + dy*dy + dz*dz in
// FP64 without fused multiply-adds, so the pair counts are exact; coincident
// points (r = 0) are in no shell.
//
// One workgroup per 256 first points (one per thread); the second points
// stream through LDS 256 at a time, and every pair adds its weight times the
// Legendre polynomials into the workgroup's FP64 shell sums in LDS.  Each
// workgroup writes one partial row per shell; a second kernel adds the rows
// of all workgroups in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lpp_internal.h"

namespace lpp {
namespace {

constexpr int kPT = 256;      // threads per workgroup: first points per workgroup, second points per tile
constexpr int kMaxPairShells = 256;
constexpr int kMaxEll = 5;    // l = 0, 2, 4, 6, 8
constexpr int kW = kMaxEll + 1;  // per shell: sum of r, then sum of w_i w_j L_l for each l

struct PairArgs {
  const double* x;
  const double* y;
  const double* z;
  const double* w;
  int64_t n;
  double ox, oy, oz;
  double rmax2;
  double inv_dr;
  const double* thr;  // (b dr)^2, b = 0 .. nb
  int nb, nl, midpoint;
};

// products and sums rounded one by one (no contraction into FMAs), so that
// host and device decide the same shell for every pair
__device__ __forceinline__ double sep2(double dx, double dy, double dz) {
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

__global__ void __launch_bounds__(kPT) pair_kernel(PairArgs a, double* __restrict__ part,
                                                   unsigned long long* __restrict__ part_cnt) {
  __shared__ double sx[kPT], sy[kPT], sz[kPT], sw[kPT];
  __shared__ double acc[kMaxPairShells * kW];
  __shared__ unsigned long long cnt[kMaxPairShells];
  __shared__ double thr[kMaxPairShells + 1];
  const int t = threadIdx.x;
  for (int i = t; i < a.nb * kW; i += kPT) acc[i] = 0.0;
  for (int i = t; i < a.nb; i += kPT) cnt[i] = 0ull;
  for (int i = t; i <= a.nb; i += kPT) thr[i] = a.thr[i];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kPT + t;
  const bool own = i < a.n;
  double xi = 0.0, yi = 0.0, zi = 0.0, wi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
  if (own) {
    xi = a.x[i];
    yi = a.y[i];
    zi = a.z[i];
    wi = a.w ? a.w[i] : 1.0;
    ex = xi - a.ox;
    ey = yi - a.oy;
    ez = zi - a.oz;
    const double inv = 1.0 / sqrt(ex * ex + ey * ey + ez * ez);
    ex *= inv;
    ey *= inv;
    ez *= inv;
  }
  for (int64_t j0 = 0; j0 < a.n; j0 += kPT) {
    __syncthreads();
    const int64_t jt = j0 + t;
    if (jt < a.n) {
      sx[t] = a.x[jt];
      sy[t] = a.y[jt];
      sz[t] = a.z[jt];
      sw[t] = a.w ? a.w[jt] : 1.0;
    }
    __syncthreads();
    const int m = static_cast<int>(a.n - j0 < kPT ? a.n - j0 : kPT);
    if (!own) continue;
    for (int jj = 0; jj < m; ++jj) {
      if (j0 + jj == i) continue;
      const double dx = sx[jj] - xi, dy = sy[jj] - yi, dz = sz[jj] - zi;
      const double r2 = sep2(dx, dy, dz);
      if (!(r2 < a.rmax2) || !(r2 > 0.0)) continue;
      const double r = sqrt(r2);
      int b = static_cast<int>(r * a.inv_dr);
      b = b < 0 ? 0 : (b > a.nb - 1 ? a.nb - 1 : b);
      while (b + 1 < a.nb && r2 >= thr[b + 1]) ++b;
      while (b > 0 && r2 < thr[b]) --b;
      double mu;
      if (a.midpoint) {
        const double mx = xi + 0.5 * dx - a.ox, my = yi + 0.5 * dy - a.oy, mz = zi + 0.5 * dz - a.oz;
        mu = (dx * mx + dy * my + dz * mz) / (r * sqrt(mx * mx + my * my + mz * mz));
      } else {
        mu = (dx * ex + dy * ey + dz * ez) / r;
      }
      const double ww = wi * sw[jj];
      double* row = acc + b * kW;
      atomicAdd(&row[0], r);
      atomicAdd(&row[1], ww);
      // Legendre polynomials by the three-term recurrence
      // L_{n+1} = ((2n+1) mu L_n - n L_{n-1}) / (n+1); the even orders are kept
      double lp = 1.0, lc = mu;
      for (int nn = 1; nn < 2 * (a.nl - 1); ++nn) {
        const double ln = ((2 * nn + 1) * mu * lc - nn * lp) / (nn + 1);
        lp = lc;
        lc = ln;
        if ((nn & 1) == 1) atomicAdd(&row[1 + (nn + 1) / 2], ww * lc);
      }
      atomicAdd(&cnt[b], 1ull);
    }
  }
  __syncthreads();
  double* out = part + static_cast<size_t>(blockIdx.x) * a.nb * kW;
  for (int k = t; k < a.nb * kW; k += kPT) out[k] = acc[k];
  unsigned long long* oc = part_cnt + static_cast<size_t>(blockIdx.x) * a.nb;
  for (int k = t; k < a.nb; k += kPT) oc[k] = cnt[k];
}

// column c of the partial rows summed over the workgroups in order
__global__ void __launch_bounds__(kPT) pair_reduce_kernel(const double* __restrict__ part,
                                                          const unsigned long long* __restrict__ part_cnt, int blocks,
                                                          int width, int nb, double* __restrict__ out,
                                                          unsigned long long* __restrict__ out_cnt) {
  const int c = blockIdx.x * kPT + threadIdx.x;
  if (c < width) {
    double s = 0.0;
    for (int g = 0; g < blocks; ++g) s += part[static_cast<size_t>(g) * width + c];
    out[c] = s;
  }
  if (c < nb) {
    unsigned long long s = 0;
    for (int g = 0; g < blocks; ++g) s += part_cnt[static_cast<size_t>(g) * nb + c];
    out_cnt[c] = s;
  }
}

template <typename S>
__global__ void to_f64_kernel(const S* __restrict__ in, int64_t n, double* __restrict__ out, int* __restrict__ bad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double v = static_cast<double>(in[i]);
    if (!isfinite(v)) *bad = 1;
    out[i] = v;
  }
}

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace
}  // namespace lpp

using namespace lpp;

extern "C" lpp_status lpp_window_pairs(const lpp_catalog* ran, double alpha, double norm_I, const double* observer,
                                       int32_t los, int32_t lmax, int32_t n_rbins, double rmax, double* Q,
                                       double* r_eff, int64_t* counts, void* stream) {
  if (!ran || !observer || !Q || !r_eff || !counts || ran->n < 2 || ran->n > (int64_t(1) << 26) || !ran->x ||
      !ran->y || !ran->z || (ran->dtype != LPP_F32 && ran->dtype != LPP_F64) || (los != 0 && los != 1) ||
      lmax < 0 || lmax > 8 || (lmax % 2) || n_rbins < 1 || n_rbins > kMaxPairShells || !(rmax > 0.0) ||
      !std::isfinite(rmax) || !(alpha > 0.0) || !std::isfinite(alpha) || !(norm_I > 0.0) || !std::isfinite(norm_I))
    return LPP_E_INVALID;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(observer[k])) return LPP_E_INVALID;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = ran->n;
  const int nb = n_rbins, nl = lmax / 2 + 1, width = nb * kW;
  const int blocks = static_cast<int>((n + kPT - 1) / kPT);
  const double dr = rmax / nb;
  std::vector<double> thr(nb + 1);
  for (int b = 0; b <= nb; ++b) thr[b] = (b * dr) * (b * dr);
  // device memory: four FP64 columns, thresholds, a flag, partial rows and the totals
  const size_t col = static_cast<size_t>(n);
  const size_t dbl = 4 * col + (nb + 1) + 1 + static_cast<size_t>(blocks) * width + width;
  const size_t u64 = static_cast<size_t>(blocks) * nb + nb;
  Buf buf;
  if (hipMalloc(&buf.p, 8 * (dbl + u64)) != hipSuccess) {
    (void)hipGetLastError();
    return LPP_E_NOMEM;
  }
  double* d = static_cast<double*>(buf.p);
  double *X = d, *Y = d + col, *Z = d + 2 * col, *Wt = d + 3 * col, *T = d + 4 * col;
  int* bad = reinterpret_cast<int*>(T + nb + 1);
  double* part = T + nb + 2;
  double* tot = part + static_cast<size_t>(blocks) * width;
  unsigned long long* pc = reinterpret_cast<unsigned long long*>(tot + width);
  unsigned long long* tc = pc + static_cast<size_t>(blocks) * nb;
  hipError_t e = hipMemcpyAsync(T, thr.data(), 8 * (nb + 1), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), st);
  // the columns as FP64 on the device: device columns converted by a kernel,
  // host columns converted on the host and copied
  const void* cols[4] = {ran->x, ran->y, ran->z, ran->w};
  double* dst[4] = {X, Y, Z, Wt};
  std::vector<double> staged[4];
  for (int c = 0; c < 4 && e == hipSuccess; ++c) {
    if (!cols[c]) continue;
    if (ran->on_device) {
      const int g = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
      if (ran->dtype == LPP_F64)
        to_f64_kernel<double><<<g, 256, 0, st>>>(static_cast<const double*>(cols[c]), n, dst[c], bad);
      else
        to_f64_kernel<float><<<g, 256, 0, st>>>(static_cast<const float*>(cols[c]), n, dst[c], bad);
      e = hipGetLastError();
    } else {
      staged[c].resize(col);
      for (size_t k = 0; k < col; ++k) {
        const double v = ran->dtype == LPP_F64 ? static_cast<const double*>(cols[c])[k]
                                               : static_cast<double>(static_cast<const float*>(cols[c])[k]);
        if (!std::isfinite(v)) return LPP_E_NONFINITE;
        staged[c][k] = v;
      }
      e = hipMemcpyAsync(dst[c], staged[c].data(), 8 * col, hipMemcpyHostToDevice, st);
    }
  }
  int bad_h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return LPP_E_DEVICE;
  if (bad_h) return LPP_E_NONFINITE;
  PairArgs a{X, Y, Z, ran->w ? Wt : nullptr, n, observer[0], observer[1], observer[2], rmax * rmax, 1.0 / dr, T,
             nb, nl, los};
  pair_kernel<<<blocks, kPT, 0, st>>>(a, part, pc);
  e = hipGetLastError();
  if (e == hipSuccess) {
    pair_reduce_kernel<<<(width + kPT - 1) / kPT, kPT, 0, st>>>(part, pc, blocks, width, nb, tot, tc);
    e = hipGetLastError();
  }
  std::vector<double> h(width);
  std::vector<unsigned long long> hc(nb);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), tot, 8 * width, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), tc, 8 * nb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return LPP_E_DEVICE;
  for (int b = 0; b < nb; ++b) {
    const double vb = 4.0 * M_PI / 3.0 * (static_cast<double>(b + 1) * (b + 1) * (b + 1) -
                                          static_cast<double>(b) * b * b) * dr * dr * dr;
    counts[b] = static_cast<int64_t>(hc[b]);
    r_eff[b] = hc[b] ? h[b * kW] / static_cast<double>(hc[b]) : 0.0;
    for (int il = 0; il < nl; ++il)
      Q[il * nb + b] = (4 * il + 1) * alpha * alpha * h[b * kW + 1 + il] / (vb * norm_I);
  }
  return LPP_OK;
}
