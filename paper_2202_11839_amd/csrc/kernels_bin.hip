// k-shell binning of the transformed fields.
//
// For every mode n the kernels form the compensated, interlaced transform
//   F(k) = [F1(k) + exp(-i k.s) F2(k)] / (2 W_p(k))      (F1 alone without interlacing)
// multiply it by the degree-L real harmonic h_a(khat) of the field and by the
// base field (conj(B(k)) for delta-delta, plus and cross; B(-k) for minus),
// and accumulate the real and imaginary parts per shell in FP64 (Sec. III.A,
// eqs. lpp_dens_app, lpp_estimator_cross_Xiij, lpp_estimator_auto_+/-).
//
// The meshes are z-blocked (lpp_internal.h).  Each thread walks runs of the 8
// z-modes of one (x, y) group (one contiguous 64-byte load per mesh for
// float2; consecutive threads take consecutive x), keeps a running FP64 sum
// while the shell index stays the same and flushes it to an LDS accumulator
// on change; the block's accumulators go to a per-block partial row that a
// second kernel reduces in block order.
//
// Density fields are real: their two interlaced copies are packed as the real
// and imaginary parts of one complex mesh, P = D1 + i D2, and are separated
// with F1(k) = [P(k) + P*(-k)]/2, F2(k) = [P(k) - P*(-k)]/(2i).  Those kernels
// walk half of k-space (z-index < N/2 with the usual tie-breaks on the
// z = 0 and y = 0 planes) and count each mode pair (k, -k) twice.
#include "device_common.h"

namespace lpp {

namespace {

using dev::cmul;
using dev::cmulc;
using dev::combine;
using dev::harmonic;
using dev::KSpec;
using dev::kspec_of;
using dev::sgn_mode;
using dev::shell_of;
using dev::V2;

constexpr int kBinThreads = 256;
constexpr int kRun = 8;
constexpr int kMaxBins = 512;

struct Acc {
  int cur;
  double re, im, cnt, ks;
};

template <bool COUNTS>
__device__ __forceinline__ void acc_add(Acc& a, int b, double re, double im, double cnt, double ks, double* sre,
                                        double* sim, double* scnt, double* sks) {
  if (b != a.cur) {
    if (a.cur >= 0) {
      atomicAdd(&sre[a.cur], a.re);
      atomicAdd(&sim[a.cur], a.im);
      if (COUNTS) {
        atomicAdd(&scnt[a.cur], a.cnt);
        atomicAdd(&sks[a.cur], a.ks);
      }
    }
    a.cur = b;
    a.re = a.im = a.cnt = a.ks = 0.0;
  }
  a.re += re;
  a.im += im;
  if (COUNTS) {
    a.cnt += cnt;
    a.ks += ks;
  }
}

template <bool COUNTS>
__device__ __forceinline__ void acc_flush(Acc& a, double* sre, double* sim, double* scnt, double* sks) {
  if (a.cur >= 0) {
    atomicAdd(&sre[a.cur], a.re);
    atomicAdd(&sim[a.cur], a.im);
    if (COUNTS) {
      atomicAdd(&scnt[a.cur], a.cnt);
      atomicAdd(&sks[a.cur], a.ks);
    }
  }
  a.cur = -1;
}

// Does the run of kRun z-modes starting at z0 reach inside the last shell,
// given qxy = nx^2 + ny^2?  (N/2 is a multiple of kRun, so a run is all
// non-negative or all negative modes.)
static_assert(kRun == kZb, "a run is one z-group");
__device__ __forceinline__ bool run_live(int z0, int N, int qxy, int qmax) {
  const int mz = z0 < N / 2 ? z0 : N - z0 - (kRun - 1);  // smallest |nz| of the run
  return mz * mz + qxy < qmax;
}

// shared-memory layout: thr[kMaxBins+1] ints, then 4*nb doubles
struct Smem {
  int thr[kMaxBins + 1];
  double v[4 * kMaxBins];
};

// Per-axis tables staged in dynamic LDS (bytes: tables_bytes<T>(N)): the
// interlacing phase factor along one axis, exp(-i pi n/N) at n + N/2, and
// 1/W(n).  The full phase is the z factor times the run's exp(-i pi (nx+ny)/N).
template <typename T>
constexpr size_t tables_bytes(int N) {
  return static_cast<size_t>(N) * (sizeof(typename V2<T>::type) + sizeof(T));
}
template <typename T>
__device__ __forceinline__ void tables_init(const BinArgs& a, typename V2<T>::type* px, T* iw) {
  using T2 = typename V2<T>::type;
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  for (int i = threadIdx.x; i < a.N; i += blockDim.x) {
    px[i] = phase[i + a.N];  // nx = i - N/2 sits at nx + 3N/2 of the phase table
    iw[i] = invw[i];
  }
}

__device__ __forceinline__ void smem_init(Smem& s, const int64_t* thr, int nb) {
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) s.thr[i] = static_cast<int>(thr[i]);
  for (int i = threadIdx.x; i < 4 * nb; i += blockDim.x) s.v[i] = 0.0;
  __syncthreads();
}

// partial rows are stored column-major, [width][gridDim.x], for a coalesced reduction
__device__ __forceinline__ void smem_store(const Smem& s, double* partial, int width) {
  __syncthreads();
  for (int i = threadIdx.x; i < width; i += blockDim.x) partial[static_cast<int64_t>(i) * gridDim.x + blockIdx.x] = s.v[i];
}

// ---- density fields (packed pair of real copies), half k-space ----
template <typename T, bool BASE>
__global__ void __launch_bounds__(kBinThreads) bin_dd_kernel(BinArgs a, KSpec<T> h,
                                                             const typename V2<T>::type* __restrict__ P,
                                                             typename V2<T>::type* __restrict__ B) {
  using T2 = typename V2<T>::type;
  __shared__ Smem s;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb;
  T2* px = reinterpret_cast<T2*>(dyn);
  T* iw = reinterpret_cast<T*>(px + N);
  tables_init<T>(a, px, iw);
  smem_init(s, a.thr, nb);  // (ends with a barrier)
  double *sre = s.v, *sim = s.v + nb, *scnt = s.v + 2 * nb, *sks = s.v + 3 * nb;
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = s.thr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
  const int mask = N - 1;
  const int64_t NN = static_cast<int64_t>(N) * N;
  const int64_t nruns = NN * (N / 2 / kRun);  // runs (x, y, z-group) with z < N/2
  Acc acc{-1, 0, 0, 0, 0};
  for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < nruns;
       r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int ix = static_cast<int>(r % N);
    const int iy = static_cast<int>((r / N) % N);
    const int z0 = static_cast<int>(r / NN) * kRun;
    const int nx = sgn_mode(ix, N), ny = sgn_mode(iy, N);
    if (!run_live(z0, N, nx * nx + ny * ny, qmax)) continue;
    const int64_t run = r * kRun;  // = zb_index(ix, iy, z0, N)
    const int mx = (N - ix) & mask, my = (N - iy) & mask;
    const T wxy = invw[ix] * invw[iy];
    const T2 pxy = phase[nx + ny + 3 * N / 2];
    T2 pv[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) pv[j] = P[run + j];
    T2 bv[kRun];
    if (!BASE) {
#pragma unroll
      for (int j = 0; j < kRun; ++j) bv[j] = B[run + j];
    }
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int iz = z0 + j, nz = iz;  // iz < N/2
      if (iz == 0 && !(iy < N / 2)) continue;                            // z=0 plane: y in [0, N/2)
      if (iz == 0 && iy == 0 && !(ix > 0 && ix < N / 2)) continue;  // y=0 line: x in (0, N/2)
      const int q = nx * nx + ny * ny + nz * nz;
      const int b = shell_of(q, s.thr, nb, inv_dn);
      if (b < 0) continue;
      const int64_t midx = zb_index(mx, my, (N - iz) & mask, N);
      const T2 pm = P[midx];
      // unpack the two real copies
      const T2 f1{static_cast<T>(0.5) * (pv[j].x + pm.x), static_cast<T>(0.5) * (pv[j].y - pm.y)};
      const T2 f2{static_cast<T>(0.5) * (pv[j].y + pm.y), static_cast<T>(-0.5) * (pv[j].x - pm.x)};
      const T2 F = combine<T, T2>(f1, f2, a.interlace, cmul(pxy, px[nz + N / 2]), wxy * iw[iz]);
      if (BASE) {
        B[run + j] = F;
        B[midx] = T2{F.x, -F.y};
        acc_add<true>(acc, b, 2.0 * (static_cast<double>(F.x) * F.x + static_cast<double>(F.y) * F.y), 0.0, 2.0,
                      2.0 * sqrt(static_cast<double>(q)), sre, sim, scnt, sks);
      } else {
        const T rq = static_cast<T>(1) / sqrt(static_cast<T>(q));
        const T hk = harmonic(h, nx * rq, ny * rq, nz * rq);
        // 2 Re[h F conj(B)]
        const double v = 2.0 * static_cast<double>(hk * (F.x * bv[j].x + F.y * bv[j].y));
        acc_add<false>(acc, b, v, 0.0, 0.0, 0.0, sre, sim, scnt, sks);
      }
    }
  }
  if (BASE)
    acc_flush<true>(acc, sre, sim, scnt, sks);
  else
    acc_flush<false>(acc, sre, sim, scnt, sks);
  smem_store(s, a.partial, (BASE ? 4 : 2) * nb);
}

// ---- complex (shape) fields, full k-space ----
// KIND 0: h G conj(B(k)); KIND 1: h G B(-k); KIND 2: base construction (B = G, |G|^2)
template <typename T, int KIND>
__global__ void __launch_bounds__(kBinThreads) bin_gg_kernel(BinArgs a, KSpec<T> h,
                                                             const typename V2<T>::type* __restrict__ G1,
                                                             const typename V2<T>::type* __restrict__ G2,
                                                             typename V2<T>::type* __restrict__ B) {
  using T2 = typename V2<T>::type;
  __shared__ Smem s;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb;
  T2* px = reinterpret_cast<T2*>(dyn);
  T* iw = reinterpret_cast<T*>(px + N);
  tables_init<T>(a, px, iw);
  smem_init(s, a.thr, nb);  // (ends with a barrier)
  double *sre = s.v, *sim = s.v + nb, *scnt = s.v + 2 * nb, *sks = s.v + 3 * nb;
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = s.thr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
  const int mask = N - 1;
  const int64_t NN = static_cast<int64_t>(N) * N;
  const int64_t nruns = NN * (N / kRun);  // runs (x, y, z-group)
  Acc acc{-1, 0, 0, 0, 0};
  for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < nruns;
       r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int ix = static_cast<int>(r % N);
    const int iy = static_cast<int>((r / N) % N);
    const int z0 = static_cast<int>(r / NN) * kRun;
    const int nx = sgn_mode(ix, N), ny = sgn_mode(iy, N);
    if (!run_live(z0, N, nx * nx + ny * ny, qmax)) continue;
    const int64_t run = r * kRun;  // = zb_index(ix, iy, z0, N)
    const int mx = (N - ix) & mask, my = (N - iy) & mask;
    const T wxy = invw[ix] * invw[iy];
    const T2 pxy = phase[nx + ny + 3 * N / 2];
    T2 g1[kRun], g2[kRun], bv[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) g1[j] = G1[run + j];
    if (a.interlace) {
#pragma unroll
      for (int j = 0; j < kRun; ++j) g2[j] = G2[run + j];
    }
    if (KIND == 0) {
#pragma unroll
      for (int j = 0; j < kRun; ++j) bv[j] = B[run + j];
    }
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int iz = z0 + j;
      const int nz = sgn_mode(iz, N);
      const int q = nx * nx + ny * ny + nz * nz;
      const int b = shell_of(q, s.thr, nb, inv_dn);
      if (b < 0) continue;
      const T2 F = combine<T, T2>(g1[j], a.interlace ? g2[j] : g1[j], a.interlace, cmul(pxy, px[nz + N / 2]),
                                  wxy * iw[iz]);
      if (KIND == 2) {
        B[run + j] = F;
        acc_add<true>(acc, b, static_cast<double>(F.x) * F.x + static_cast<double>(F.y) * F.y, 0.0, 1.0,
                      sqrt(static_cast<double>(q)), sre, sim, scnt, sks);
        continue;
      }
      const T rq = static_cast<T>(1) / sqrt(static_cast<T>(q));
      const T hk = harmonic(h, nx * rq, ny * rq, nz * rq);
      T2 p;
      if (KIND == 0) {
        p = cmulc(F, bv[j]);
      } else {
        const T2 bm = B[zb_index(mx, my, (N - iz) & mask, N)];
        p = cmul(F, bm);
      }
      acc_add<false>(acc, b, static_cast<double>(hk * p.x), static_cast<double>(hk * p.y), 0.0, 0.0, sre, sim, scnt,
                     sks);
    }
  }
  if (KIND == 2)
    acc_flush<true>(acc, sre, sim, scnt, sks);
  else
    acc_flush<false>(acc, sre, sim, scnt, sks);
  smem_store(s, a.partial, (KIND == 2 ? 4 : 2) * nb);
}

// one block per column: strided partial sums, then a fixed-shape tree (deterministic)
constexpr int kRedThreads = 256;
__global__ void __launch_bounds__(kRedThreads) reduce_partials_kernel(const double* __restrict__ partial, int nblocks,
                                                                      double* __restrict__ acc) {
  __shared__ double sh[kRedThreads];
  const int w = blockIdx.x;
  const double* col = partial + static_cast<int64_t>(w) * nblocks;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kRedThreads) s += col[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[w] += sh[0];
}

}  // namespace

int bin_blocks(int N) {
  const int64_t runs = static_cast<int64_t>(N) * N * N / kRun;
  int64_t want = (runs + kBinThreads - 1) / kBinThreads;
  if (want > 4096) want = 4096;
  if (want < 1) want = 1;
  return static_cast<int>(want);
}

template <typename T>
hipError_t launch_base_dd(const BinArgs& a, const void* packed, void* base, hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb > kMaxBins) return hipErrorInvalidValue;
  KSpec<T> h{};
  bin_dd_kernel<T, true><<<a.nblocks, kBinThreads, tables_bytes<T>(a.N), st>>>(a, h, static_cast<const T2*>(packed),
                                                              static_cast<T2*>(base));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_base_gg(const BinArgs& a, const void* g1, const void* g2, void* base, hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb > kMaxBins) return hipErrorInvalidValue;
  KSpec<T> h{};
  bin_gg_kernel<T, 2><<<a.nblocks, kBinThreads, tables_bytes<T>(a.N), st>>>(a, h, static_cast<const T2*>(g1),
                                                          static_cast<const T2*>(g2), static_cast<T2*>(base));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bin_dd(const BinArgs& a, const FieldSpec& f, const void* packed, const void* base,
                         hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb > kMaxBins) return hipErrorInvalidValue;
  bin_dd_kernel<T, false><<<a.nblocks, kBinThreads, tables_bytes<T>(a.N), st>>>(a, kspec_of<T>(f), static_cast<const T2*>(packed),
                                                               const_cast<T2*>(static_cast<const T2*>(base)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bin_gg(const BinArgs& a, const FieldSpec& f, const void* g1, const void* g2, const void* base,
                         int kind, hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb > kMaxBins) return hipErrorInvalidValue;
  T2* b = const_cast<T2*>(static_cast<const T2*>(base));
  if (kind == 0)
    bin_gg_kernel<T, 0><<<a.nblocks, kBinThreads, tables_bytes<T>(a.N), st>>>(a, kspec_of<T>(f), static_cast<const T2*>(g1),
                                                            static_cast<const T2*>(g2), b);
  else
    bin_gg_kernel<T, 1><<<a.nblocks, kBinThreads, tables_bytes<T>(a.N), st>>>(a, kspec_of<T>(f), static_cast<const T2*>(g1),
                                                            static_cast<const T2*>(g2), b);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int nblocks, int width, double* acc, hipStream_t st) {
  reduce_partials_kernel<<<width, kRedThreads, 0, st>>>(partial, nblocks, acc);
  return hipGetLastError();
}

template hipError_t launch_base_dd<float>(const BinArgs&, const void*, void*, hipStream_t);
template hipError_t launch_base_dd<double>(const BinArgs&, const void*, void*, hipStream_t);
template hipError_t launch_base_gg<float>(const BinArgs&, const void*, const void*, void*, hipStream_t);
template hipError_t launch_base_gg<double>(const BinArgs&, const void*, const void*, void*, hipStream_t);
template hipError_t launch_bin_gg<float>(const BinArgs&, const FieldSpec&, const void*, const void*, const void*, int,
                                         hipStream_t);
template hipError_t launch_bin_gg<double>(const BinArgs&, const FieldSpec&, const void*, const void*, const void*,
                                          int, hipStream_t);
template hipError_t launch_bin_dd<float>(const BinArgs&, const FieldSpec&, const void*, const void*, hipStream_t);
template hipError_t launch_bin_dd<double>(const BinArgs&, const FieldSpec&, const void*, const void*, hipStream_t);

}  // namespace lpp
