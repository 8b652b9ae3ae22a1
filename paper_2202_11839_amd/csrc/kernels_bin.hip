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
// second kernel reduces in block order.  The fields of one gather pass that
// share the base and the kind of product are summed by one launch, which
// reads the base once for all of them.
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

// 1/sqrt(q) for the unit vector of a mode: the hardware reciprocal square
// root in FP32 (1 ulp; the harmonic weights then carry a few ulp, far below
// the FP32 path's rounding of the fields), the correctly rounded quotient in
// FP64
template <typename T>
__device__ __forceinline__ T inv_sqrt(int q) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_rsqf(static_cast<float>(q));
  else
    return 1.0 / sqrt(static_cast<double>(q));
}

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

// Shell sums go to one LDS row set per wavefront (its flushes come in program
// order, and one instruction's lanes in a fixed order), and the rows of the
// four wavefronts are added in a fixed order when the block stores its
// partial row: two runs give bitwise the same sums.
constexpr int kBinWaves = kBinThreads / 64;

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

// dynamic LDS: the per-axis tables, then kBinWaves rows of `width` FP64 sums
template <typename T>
constexpr size_t rows_offset(int N) {
  return (tables_bytes<T>(N) + 15) / 16 * 16;
}
template <typename T>
size_t bin_lds_bytes(int N, int width) {
  return rows_offset<T>(N) + 8 * static_cast<size_t>(kBinWaves) * width;
}

// thresholds to LDS, every row to zero; returns this wavefront's row
__device__ __forceinline__ double* rows_init(unsigned char* dyn, size_t off, int width, const int64_t* thr, int* sthr,
                                             int nb) {
  double* rows = reinterpret_cast<double*>(dyn + off);
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) sthr[i] = static_cast<int>(thr[i]);
  for (int i = threadIdx.x; i < kBinWaves * width; i += blockDim.x) rows[i] = 0.0;
  __syncthreads();
  return rows + (threadIdx.x >> 6) * width;
}

// the block's partial row (the wavefront rows added in order), stored
// column-major, [width][gridDim.x], for a coalesced reduction
__device__ __forceinline__ void rows_store(const unsigned char* dyn, size_t off, int width, double* partial) {
  const double* rows = reinterpret_cast<const double*>(dyn + off);
  __syncthreads();
  for (int i = threadIdx.x; i < width; i += blockDim.x) {
    double v = rows[i];
#pragma unroll
    for (int w = 1; w < kBinWaves; ++w) v += rows[w * width + i];
    partial[static_cast<int64_t>(i) * gridDim.x + blockIdx.x] = v;
  }
}

// ---- the bases: B = F at every mode inside the last shell, with |F|^2, the
// mode count and the sum of |n| per shell (rows [re, im, counts, sum |n|]) ----

// density base from the packed pair of real copies, half k-space, B also
// written at -k as conj(F)
template <typename T>
__global__ void __launch_bounds__(kBinThreads) base_dd_kernel(BinArgs a, const typename V2<T>::type* __restrict__ P,
                                                              typename V2<T>::type* __restrict__ B) {
  using T2 = typename V2<T>::type;
  __shared__ int sthr[kMaxBins + 1];
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb;
  T2* px = reinterpret_cast<T2*>(dyn);
  T* iw = reinterpret_cast<T*>(px + N);
  tables_init<T>(a, px, iw);
  double* v = rows_init(dyn, rows_offset<T>(N), 4 * nb, a.thr, sthr, nb);  // (ends with a barrier)
  double *sre = v, *sim = v + nb, *scnt = v + 2 * nb, *sks = v + 3 * nb;
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = sthr[nb];
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
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int iz = z0 + j, nz = iz;  // iz < N/2
      if (iz == 0 && !(iy < N / 2)) continue;                            // z=0 plane: y in [0, N/2)
      if (iz == 0 && iy == 0 && !(ix > 0 && ix < N / 2)) continue;  // y=0 line: x in (0, N/2)
      const int q = nx * nx + ny * ny + nz * nz;
      const int b = shell_of(q, sthr, nb, inv_dn);
      if (b < 0) continue;
      const int64_t midx = zb_index(mx, my, (N - iz) & mask, N);
      const T2 pm = P[midx];
      // unpack the two real copies
      const T2 f1{static_cast<T>(0.5) * (pv[j].x + pm.x), static_cast<T>(0.5) * (pv[j].y - pm.y)};
      const T2 f2{static_cast<T>(0.5) * (pv[j].y + pm.y), static_cast<T>(-0.5) * (pv[j].x - pm.x)};
      const T2 F = combine<T, T2>(f1, f2, a.interlace, cmul(pxy, px[nz + N / 2]), wxy * iw[iz]);
      B[run + j] = F;
      B[midx] = T2{F.x, -F.y};
      acc_add<true>(acc, b, 2.0 * (static_cast<double>(F.x) * F.x + static_cast<double>(F.y) * F.y), 0.0, 2.0,
                    2.0 * sqrt(static_cast<double>(q)), sre, sim, scnt, sks);
    }
  }
  acc_flush<true>(acc, sre, sim, scnt, sks);
  rows_store(dyn, rows_offset<T>(N), 4 * nb, a.partial);
}

// shape base from the two interlaced copies, full k-space
template <typename T>
__global__ void __launch_bounds__(kBinThreads) base_gg_kernel(BinArgs a, const typename V2<T>::type* __restrict__ G1,
                                                              const typename V2<T>::type* __restrict__ G2,
                                                              typename V2<T>::type* __restrict__ B) {
  using T2 = typename V2<T>::type;
  __shared__ int sthr[kMaxBins + 1];
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb;
  T2* px = reinterpret_cast<T2*>(dyn);
  T* iw = reinterpret_cast<T*>(px + N);
  tables_init<T>(a, px, iw);
  double* v = rows_init(dyn, rows_offset<T>(N), 4 * nb, a.thr, sthr, nb);  // (ends with a barrier)
  double *sre = v, *sim = v + nb, *scnt = v + 2 * nb, *sks = v + 3 * nb;
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = sthr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
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
    const T wxy = invw[ix] * invw[iy];
    const T2 pxy = phase[nx + ny + 3 * N / 2];
    T2 g1[kRun], g2[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) g1[j] = G1[run + j];
    if (a.interlace) {
#pragma unroll
      for (int j = 0; j < kRun; ++j) g2[j] = G2[run + j];
    }
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int iz = z0 + j;
      const int nz = sgn_mode(iz, N);
      const int q = nx * nx + ny * ny + nz * nz;
      const int b = shell_of(q, sthr, nb, inv_dn);
      if (b < 0) continue;
      const T2 F = combine<T, T2>(g1[j], a.interlace ? g2[j] : g1[j], a.interlace, cmul(pxy, px[nz + N / 2]),
                                  wxy * iw[iz]);
      B[run + j] = F;
      acc_add<true>(acc, b, static_cast<double>(F.x) * F.x + static_cast<double>(F.y) * F.y, 0.0, 1.0,
                    sqrt(static_cast<double>(q)), sre, sim, scnt, sks);
    }
  }
  acc_flush<true>(acc, sre, sim, scnt, sks);
  rows_store(dyn, rows_offset<T>(N), 4 * nb, a.partial);
}

// ---- several fields of one gather pass against the same base ----
// The fields of a group share the base (read once per run) and the shell
// index of every mode; each field keeps its own running sum.  Rows: field f
// at [2f nb, 2f nb + nb) (real part) and [(2f + 1) nb, ...) (imaginary part).
template <typename T, int NFB>
struct DdGroup {
  KSpec<T> h[NFB];
  const typename V2<T>::type* P[NFB];  // packed pairs of real copies
};
template <typename T, int NFB>
struct GgGroup {
  KSpec<T> h[NFB];
  const typename V2<T>::type* g1[NFB];  // grid copy
  const typename V2<T>::type* g2[NFB];  // interlaced copy (unused without interlacing)
};

template <typename T, int NFB>
__global__ void __launch_bounds__(kBinThreads) bin_dd_group_kernel(BinArgs a, DdGroup<T, NFB> g,
                                                                   const typename V2<T>::type* __restrict__ B) {
  using T2 = typename V2<T>::type;
  __shared__ int sthr[kMaxBins + 1];
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb;
  T2* px = reinterpret_cast<T2*>(dyn);
  T* iw = reinterpret_cast<T*>(px + N);
  tables_init<T>(a, px, iw);
  double* v = rows_init(dyn, rows_offset<T>(N), 2 * NFB * nb, a.thr, sthr, nb);  // (ends with a barrier)
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = sthr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
  const int mask = N - 1;
  const int64_t NN = static_cast<int64_t>(N) * N;
  const int64_t nruns = NN * (N / 2 / kRun);  // runs (x, y, z-group) with z < N/2
  int cur[NFB];
  double sr[NFB];
#pragma unroll
  for (int f = 0; f < NFB; ++f) {
    cur[f] = -1;
    sr[f] = 0.0;
  }
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
    T2 bv[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) bv[j] = B[run + j];
    int bq[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int iz = z0 + j;  // iz < N/2
      const bool keep = !(iz == 0 && !(iy < N / 2)) && !(iz == 0 && iy == 0 && !(ix > 0 && ix < N / 2));
      bq[j] = keep ? shell_of(nx * nx + ny * ny + iz * iz, sthr, nb, inv_dn) : -1;
    }
#pragma unroll
    for (int f = 0; f < NFB; ++f) {
      const T2* __restrict__ P = g.P[f];
      T2 pv[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) pv[j] = P[run + j];
#pragma unroll
      for (int j = 0; j < kRun; ++j) {
        const int b = bq[j];
        if (b < 0) continue;
        const int iz = z0 + j, nz = iz;
        const T2 pm = P[zb_index(mx, my, (N - iz) & mask, N)];
        const T2 f1{static_cast<T>(0.5) * (pv[j].x + pm.x), static_cast<T>(0.5) * (pv[j].y - pm.y)};
        const T2 f2{static_cast<T>(0.5) * (pv[j].y + pm.y), static_cast<T>(-0.5) * (pv[j].x - pm.x)};
        const T2 F = combine<T, T2>(f1, f2, a.interlace, cmul(pxy, px[nz + N / 2]), wxy * iw[iz]);
        const int q = nx * nx + ny * ny + nz * nz;
        const T rq = inv_sqrt<T>(q);
        const T hk = harmonic(g.h[f], nx * rq, ny * rq, nz * rq);
        if (b != cur[f]) {
          if (cur[f] >= 0) atomicAdd(&v[2 * f * nb + cur[f]], sr[f]);
          cur[f] = b;
          sr[f] = 0.0;
        }
        // 2 Re[h F conj(B)]
        sr[f] += 2.0 * static_cast<double>(hk * (F.x * bv[j].x + F.y * bv[j].y));
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NFB; ++f)
    if (cur[f] >= 0) atomicAdd(&v[2 * f * nb + cur[f]], sr[f]);
  rows_store(dyn, rows_offset<T>(N), 2 * NFB * nb, a.partial);
}

// KIND 0: h G conj(B(k)); KIND 1: h G B(-k)
template <typename T, int KIND, int NFB>
__global__ void __launch_bounds__(kBinThreads) bin_gg_group_kernel(BinArgs a, GgGroup<T, NFB> g,
                                                                   const typename V2<T>::type* __restrict__ B) {
  using T2 = typename V2<T>::type;
  __shared__ int sthr[kMaxBins + 1];
  extern __shared__ __align__(16) unsigned char dyn[];
  const int N = a.N, nb = a.nb;
  T2* px = reinterpret_cast<T2*>(dyn);
  T* iw = reinterpret_cast<T*>(px + N);
  tables_init<T>(a, px, iw);
  double* v = rows_init(dyn, rows_offset<T>(N), 2 * NFB * nb, a.thr, sthr, nb);  // (ends with a barrier)
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = sthr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
  const int mask = N - 1;
  const int64_t NN = static_cast<int64_t>(N) * N;
  const int64_t nruns = NN * (N / kRun);  // runs (x, y, z-group)
  int cur[NFB];
  double sre[NFB], sim[NFB];
#pragma unroll
  for (int f = 0; f < NFB; ++f) {
    cur[f] = -1;
    sre[f] = sim[f] = 0.0;
  }
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
    int bq[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int nz = sgn_mode(z0 + j, N);
      bq[j] = shell_of(nx * nx + ny * ny + nz * nz, sthr, nb, inv_dn);
    }
    // the base at k (plus, cross) or at -k (minus), once for all fields
    T2 bv[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      bv[j] = T2{0, 0};
      if (KIND == 0) bv[j] = B[run + j];
      else if (bq[j] >= 0) bv[j] = B[zb_index(mx, my, (N - z0 - j) & mask, N)];
    }
#pragma unroll
    for (int f = 0; f < NFB; ++f) {
      T2 g1[kRun], g2[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) g1[j] = g.g1[f][run + j];
      if (a.interlace) {
#pragma unroll
        for (int j = 0; j < kRun; ++j) g2[j] = g.g2[f][run + j];
      }
#pragma unroll
      for (int j = 0; j < kRun; ++j) {
        const int b = bq[j];
        if (b < 0) continue;
        const int iz = z0 + j, nz = sgn_mode(iz, N);
        const T2 F = combine<T, T2>(g1[j], a.interlace ? g2[j] : g1[j], a.interlace, cmul(pxy, px[nz + N / 2]),
                                    wxy * iw[iz]);
        const int q = nx * nx + ny * ny + nz * nz;
        const T rq = inv_sqrt<T>(q);
        const T hk = harmonic(g.h[f], nx * rq, ny * rq, nz * rq);
        const T2 p = KIND == 0 ? cmulc(F, bv[j]) : cmul(F, bv[j]);
        if (b != cur[f]) {
          if (cur[f] >= 0) {
            atomicAdd(&v[2 * f * nb + cur[f]], sre[f]);
            atomicAdd(&v[(2 * f + 1) * nb + cur[f]], sim[f]);
          }
          cur[f] = b;
          sre[f] = sim[f] = 0.0;
        }
        sre[f] += static_cast<double>(hk * p.x);
        sim[f] += static_cast<double>(hk * p.y);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NFB; ++f)
    if (cur[f] >= 0) {
      atomicAdd(&v[2 * f * nb + cur[f]], sre[f]);
      atomicAdd(&v[(2 * f + 1) * nb + cur[f]], sim[f]);
    }
  rows_store(dyn, rows_offset<T>(N), 2 * NFB * nb, a.partial);
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
  if (want > 8192) want = 8192;
  if (want < 1) want = 1;
  return static_cast<int>(want);
}

template <typename T>
hipError_t launch_base_dd(const BinArgs& a, const void* packed, void* base, hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb > kMaxBins) return hipErrorInvalidValue;
  base_dd_kernel<T><<<a.nblocks, kBinThreads, bin_lds_bytes<T>(a.N, 4 * a.nb), st>>>(a, static_cast<const T2*>(packed),
                                                                          static_cast<T2*>(base));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_base_gg(const BinArgs& a, const void* g1, const void* g2, void* base, hipStream_t st) {
  using T2 = typename V2<T>::type;
  if (a.nb > kMaxBins) return hipErrorInvalidValue;
  base_gg_kernel<T><<<a.nblocks, kBinThreads, bin_lds_bytes<T>(a.N, 4 * a.nb), st>>>(a, static_cast<const T2*>(g1),
                                                                          static_cast<const T2*>(g2),
                                                                          static_cast<T2*>(base));
  return hipGetLastError();
}

template <typename T, int NFB>
hipError_t bin_dd_group_n(const BinArgs& a, const FieldSpec* const* f, const void* const* packed, const void* base,
                          hipStream_t st) {
  using T2 = typename V2<T>::type;
  DdGroup<T, NFB> g{};
  for (int i = 0; i < NFB; ++i) {
    g.h[i] = kspec_of<T>(*f[i]);
    g.P[i] = static_cast<const T2*>(packed[i]);
  }
  bin_dd_group_kernel<T, NFB><<<a.nblocks, kBinThreads, bin_lds_bytes<T>(a.N, 2 * NFB * a.nb), st>>>(a, g, static_cast<const T2*>(base));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bin_dd(const BinArgs& a, const FieldSpec* const* f, const void* const* packed, int n,
                         const void* base, hipStream_t st) {
  if (a.nb > kMaxBins || 2 * n * a.nb > 4 * kMaxBins) return hipErrorInvalidValue;
  switch (n) {
    case 1: return bin_dd_group_n<T, 1>(a, f, packed, base, st);
    case 2: return bin_dd_group_n<T, 2>(a, f, packed, base, st);
    case 3: return bin_dd_group_n<T, 3>(a, f, packed, base, st);
    case 4: return bin_dd_group_n<T, 4>(a, f, packed, base, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int KIND, int NFB>
hipError_t bin_gg_group_n(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2,
                          const void* base, hipStream_t st) {
  using T2 = typename V2<T>::type;
  GgGroup<T, NFB> g{};
  for (int i = 0; i < NFB; ++i) {
    g.h[i] = kspec_of<T>(*f[i]);
    g.g1[i] = static_cast<const T2*>(g1[i]);
    g.g2[i] = static_cast<const T2*>(g2 ? g2[i] : g1[i]);
  }
  bin_gg_group_kernel<T, KIND, NFB><<<a.nblocks, kBinThreads, bin_lds_bytes<T>(a.N, 2 * NFB * a.nb), st>>>(a, g,
                                                                                      static_cast<const T2*>(base));
  return hipGetLastError();
}

template <typename T, int KIND>
hipError_t bin_gg_kind(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2, int n,
                       const void* base, hipStream_t st) {
  switch (n) {
    case 1: return bin_gg_group_n<T, KIND, 1>(a, f, g1, g2, base, st);
    case 2: return bin_gg_group_n<T, KIND, 2>(a, f, g1, g2, base, st);
    case 3: return bin_gg_group_n<T, KIND, 3>(a, f, g1, g2, base, st);
    case 4: return bin_gg_group_n<T, KIND, 4>(a, f, g1, g2, base, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_bin_gg(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2,
                         int n, const void* base, int kind, hipStream_t st) {
  if (a.nb > kMaxBins || 2 * n * a.nb > 4 * kMaxBins) return hipErrorInvalidValue;
  return kind == 0 ? bin_gg_kind<T, 0>(a, f, g1, g2, n, base, st) : bin_gg_kind<T, 1>(a, f, g1, g2, n, base, st);
}

hipError_t launch_reduce_partials(const double* partial, int nblocks, int width, double* acc, hipStream_t st) {
  reduce_partials_kernel<<<width, kRedThreads, 0, st>>>(partial, nblocks, acc);
  return hipGetLastError();
}

template hipError_t launch_base_dd<float>(const BinArgs&, const void*, void*, hipStream_t);
template hipError_t launch_base_dd<double>(const BinArgs&, const void*, void*, hipStream_t);
template hipError_t launch_base_gg<float>(const BinArgs&, const void*, const void*, void*, hipStream_t);
template hipError_t launch_base_gg<double>(const BinArgs&, const void*, const void*, void*, hipStream_t);
template hipError_t launch_bin_gg<float>(const BinArgs&, const FieldSpec* const*, const void* const*,
                                         const void* const*, int, const void*, int, hipStream_t);
template hipError_t launch_bin_gg<double>(const BinArgs&, const FieldSpec* const*, const void* const*,
                                          const void* const*, int, const void*, int, hipStream_t);
template hipError_t launch_bin_dd<float>(const BinArgs&, const FieldSpec* const*, const void* const*, int, const void*,
                                         hipStream_t);
template hipError_t launch_bin_dd<double>(const BinArgs&, const FieldSpec* const*, const void* const*, int,
                                          const void*, hipStream_t);

}  // namespace lpp
