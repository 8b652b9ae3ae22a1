// Multipoles of the window's auto-correlation, Q_l(r) (Sec. III.B, eqs.
// windowQ and windowQ_ell, end-point line of sight), on z-blocked meshes.
//
// With the real harmonics h_a of degree l (the same ones the estimator
// uses), L_l(rhat . xhat) = sum_a kappa_a h_a(rhat) h_a(xhat), so
//   int_x W(x) W(x+r) L_l(rhat . xhat) = sum_a h_a(rhat) X_a(r),
//   X_a(r) = int_x [kappa_a h_a(xhat) W(x)] W(x+r) = IFT[conj(F_a) F_0](r),
// where F_a is the transform of the window weighted by kappa_a h_a(xhat)
// (deposited, interlaced and compensated like a density field) and F_0 the
// transform of the window itself.  The X_a are real, so two of them share
// one inverse transform: with Z = Y_a + i Y_b (Y = conj(F_a) F_0),
// IFT[Z] = X_a + i X_b, and IFT[Z] = conj(DFT[conj Z]) / N^3, so the kernels
// build conj(Z), run the forward transform and read X_a = Re / N^3,
// X_b = -Im / N^3 (the 1/N^3 is applied on the host).
#include "device_common.h"

namespace lpp {

namespace {

using dev::cmul;
using dev::combine;
using dev::harmonic;
using dev::KSpec;
using dev::kspec_of;
using dev::sgn_mode;
using dev::V2;

constexpr int kWinThreads = 256;
constexpr int kWinWaves = kWinThreads / 64;

// mode (x, y, z) at position i of a z-blocked mesh
__device__ __forceinline__ void zb_coords(int64_t i, int N, int& x, int& y, int& z) {
  const int64_t g = i >> 3;
  x = static_cast<int>(g % N);
  y = static_cast<int>((g / N) % N);
  z = static_cast<int>(g / (static_cast<int64_t>(N) * N)) * kZb + static_cast<int>(i & 7);
}

// the transform of field a at mode (ix, iy, iz) from its packed interlaced copies
template <typename T>
__device__ __forceinline__ typename V2<T>::type field_at(const typename V2<T>::type* __restrict__ P, int N,
                                                         int64_t idx, int64_t midx, int interlace,
                                                         typename V2<T>::type ph, T invw) {
  using T2 = typename V2<T>::type;
  const T2 p = P[idx], pm = P[midx];
  const T2 f1{static_cast<T>(0.5) * (p.x + pm.x), static_cast<T>(0.5) * (p.y - pm.y)};
  const T2 f2{static_cast<T>(0.5) * (p.y + pm.y), static_cast<T>(-0.5) * (p.x - pm.x)};
  return combine<T, T2>(f1, f2, interlace, ph, invw);
}

// slot < 0: B0 = F_0 (the window itself) at every mode;
// slot 0:  Zc = conj(conj(F_a) B0);  slot 1:  Zc += -i conj(conj(F_b) B0)
template <typename T>
__global__ void __launch_bounds__(kWinThreads) window_product_kernel(WinArgs a, const typename V2<T>::type* __restrict__ P,
                                                                    typename V2<T>::type* __restrict__ B0,
                                                                    typename V2<T>::type* __restrict__ Zc, int slot) {
  using T2 = typename V2<T>::type;
  const int N = a.N, mask = N - 1;
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n3;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int ix, iy, iz;
    zb_coords(i, N, ix, iy, iz);
    const int64_t m = zb_index((N - ix) & mask, (N - iy) & mask, (N - iz) & mask, N);
    const int nsum = sgn_mode(ix, N) + sgn_mode(iy, N) + sgn_mode(iz, N);
    const T2 ph = a.interlace ? phase[nsum + 3 * N / 2] : T2{1, 0};
    const T2 F = field_at<T>(P, N, i, m, a.interlace, ph, invw[ix] * invw[iy] * invw[iz]);
    if (slot < 0) {
      B0[i] = F;
      continue;
    }
    // Y = conj(F_a) B0, made Hermitian, Y_h(k) = [Y(k) + conj(Y(-k))]/2, so
    // that its inverse transform is exactly the real part of IFT[Y]: the two
    // terms differ only on the Nyquist planes, where -k is k's own index but
    // the interlacing phase is not conjugated.
    const int mx = (N - ix) & mask, my = (N - iy) & mask, mz = (N - iz) & mask;
    const int msum = sgn_mode(mx, N) + sgn_mode(my, N) + sgn_mode(mz, N);
    const T2 phm = a.interlace ? phase[msum + 3 * N / 2] : T2{1, 0};
    const T2 Fm = field_at<T>(P, N, m, i, a.interlace, phm, invw[mx] * invw[my] * invw[mz]);
    const T2 b = B0[i], bm = B0[m];
    // conj(Y(k)) = F conj(b);  Y(-k) = conj(Fm) bm
    const T2 c1{F.x * b.x + F.y * b.y, F.y * b.x - F.x * b.y};
    const T2 y2{Fm.x * bm.x + Fm.y * bm.y, Fm.x * bm.y - Fm.y * bm.x};
    const T2 yc{static_cast<T>(0.5) * (c1.x + y2.x), static_cast<T>(0.5) * (c1.y + y2.y)};  // conj(Y_h(k))
    if (slot == 0) {
      Zc[i] = yc;
    } else {  // -i conj(Y) = (yc.y, -yc.x)
      const T2 z = Zc[i];
      Zc[i] = T2{z.x + yc.y, z.y - yc.x};
    }
  }
}

// Shell sums over the separations r (minimum image, in cells) of the
// transform D = DFT[conj Z]: row_a += h_a(rhat) Re D, row_b -= h_b(rhat) Im D,
// and (with_counts) the number of separations and the sum of |n| per shell.
// Rows: [n_ell][nb] of field rows, then counts[nb], then |n| sums[nb].
template <typename T>
__global__ void __launch_bounds__(kWinThreads) window_bin_kernel(WinArgs a, const typename V2<T>::type* __restrict__ D,
                                                                KSpec<T> ha, KSpec<T> hb, int row_a, int row_b,
                                                                int with_counts, double* __restrict__ partial) {
  using T2 = typename V2<T>::type;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb, nrow = a.n_rows;
  // one row set per wavefront, added in a fixed order at the end (bitwise
  // reproducible sums)
  int* thr = reinterpret_cast<int*>(dyn);
  double* rows = reinterpret_cast<double*>(dyn + 16 * ((4 * (nb + 1) + 15) / 16));
  const int width = nrow * nb;
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) thr[i] = static_cast<int>(a.thr[i]);
  for (int i = threadIdx.x; i < kWinWaves * width; i += blockDim.x) rows[i] = 0.0;
  __syncthreads();
  double* acc = rows + (threadIdx.x >> 6) * width;
  const int qmax = thr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  const int hasb = row_b >= 0;
  double* ra = acc + static_cast<int64_t>(row_a) * nb;
  double* rb = acc + static_cast<int64_t>(hasb ? row_b : row_a) * nb;
  double* rc = acc + static_cast<int64_t>(nrow - 2) * nb;
  double* rs = acc + static_cast<int64_t>(nrow - 1) * nb;
  int cur = -1;
  double sa = 0, sb = 0, sc = 0, ss = 0;
  auto flush = [&]() {
    if (cur >= 0) {
      atomicAdd(&ra[cur], sa);
      if (hasb) atomicAdd(&rb[cur], sb);
      if (with_counts) {
        atomicAdd(&rc[cur], sc);
        atomicAdd(&rs[cur], ss);
      }
    }
    sa = sb = sc = ss = 0.0;
  };
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n3;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int ix, iy, iz;
    zb_coords(i, N, ix, iy, iz);
    const int nx = sgn_mode(ix, N), ny = sgn_mode(iy, N), nz = sgn_mode(iz, N);
    const int q = nx * nx + ny * ny + nz * nz;
    const int b = dev::shell_of(q, thr, nb, inv_dn);
    if (b < 0) continue;
    if (b != cur) {
      flush();
      cur = b;
    }
    const T2 d = D[i];
    const T rq = static_cast<T>(1) / sqrt(static_cast<T>(q));
    const T ux = nx * rq, uy = ny * rq, uz = nz * rq;
    sa += static_cast<double>(harmonic(ha, ux, uy, uz) * d.x);
    if (hasb) sb -= static_cast<double>(harmonic(hb, ux, uy, uz) * d.y);
    sc += 1.0;
    ss += sqrt(static_cast<double>(q));
  }
  flush();
  __syncthreads();
  for (int i = threadIdx.x; i < width; i += blockDim.x) {
    double v = rows[i];
#pragma unroll
    for (int w = 1; w < kWinWaves; ++w) v += rows[w * width + i];
    partial[static_cast<int64_t>(i) * gridDim.x + blockIdx.x] = v;
  }
}

int grid_for(int64_t n3) {
  const int64_t want = (n3 + kWinThreads - 1) / kWinThreads;
  return static_cast<int>(want < 4096 ? want : 4096);
}

}  // namespace

int window_bin_blocks(int N) { return grid_for(static_cast<int64_t>(N) * N * N); }

template <typename T>
hipError_t launch_window_product(const WinArgs& a, const void* packed, void* B0, void* Zc, int slot, hipStream_t st) {
  using T2 = typename V2<T>::type;
  const int64_t n3 = static_cast<int64_t>(a.N) * a.N * a.N;
  window_product_kernel<T><<<grid_for(n3), kWinThreads, 0, st>>>(a, static_cast<const T2*>(packed),
                                                                  static_cast<T2*>(B0), static_cast<T2*>(Zc), slot);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_window_bin(const WinArgs& a, const void* D, const FieldSpec* fa, const FieldSpec* fb, int row_a,
                             int row_b, int with_counts, double* partial, hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb < 1 || a.nb > kMaxShells || a.n_rows > kWinMaxRows) return hipErrorInvalidValue;
  const size_t lds = 16 * ((4 * (a.nb + 1) + 15) / 16) + 8 * static_cast<size_t>(kWinWaves) * a.n_rows * a.nb;
  KSpec<T> ha = kspec_of<T>(*fa), hb = fb ? kspec_of<T>(*fb) : KSpec<T>{};
  window_bin_kernel<T><<<window_bin_blocks(a.N), kWinThreads, lds, st>>>(a, static_cast<const T2*>(D), ha, hb, row_a,
                                                                          fb ? row_b : -1, with_counts, partial);
  return hipGetLastError();
}

template hipError_t launch_window_product<float>(const WinArgs&, const void*, void*, void*, int, hipStream_t);
template hipError_t launch_window_product<double>(const WinArgs&, const void*, void*, void*, int, hipStream_t);
template hipError_t launch_window_bin<float>(const WinArgs&, const void*, const FieldSpec*, const FieldSpec*, int, int,
                                             int, double*, hipStream_t);
template hipError_t launch_window_bin<double>(const WinArgs&, const void*, const FieldSpec*, const FieldSpec*, int, int,
                                              int, double*, hipStream_t);

}  // namespace lpp
