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
// reads the base once for all of them.  For complex (shape) fields the z pass
// of the transform is fused into that launch (zbin_gg_kernel below), so the
// transformed fields never go to HBM; bin_gg_group_kernel reads them back
// from HBM when the plan's tuning asks for the unfused path.
//
// Density fields are real: their two interlaced copies are packed as the real
// and imaginary parts of one complex mesh, P = D1 + i D2, and are separated
// with F1(k) = [P(k) + P*(-k)]/2, F2(k) = [P(k) - P*(-k)]/(2i).  Those kernels
// walk column pairs: a column A = (x, y) of the half plane 0 <= y < N/2 (on
// y = 0, x < N/2) together with its mirror column M = (-x, -y), whose z-groups
// are read whole.  Group g of A holds z = 8g .. 8g+7, whose mirrors N - z are
// elements 7 .. 1 of group N/8 - 1 - g of M, plus element 0 of the group read
// one step earlier (carried in registers), so every HBM access is an aligned
// 64-byte run read once.  The z-groups of A are walked in the order
// c = (g + N/16) mod N/8, which puts nz = 0 in the middle and the groups
// inside the last shell on one range of c; a thread takes one chunk of that
// range (the chunk's first carried element is one extra 8-byte load).  Each
// mode pair (k, -k) is counted twice from its mode in A (once from both
// modes in the self-mirrored column (0, 0)).
#include "device_common.h"

namespace lpp {

namespace {

using dev::cmul;
using dev::cmulc;
using dev::combine;
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

// The real harmonic h_{L,M,cs}(khat) = Q(khat_z) Re|Im (khat_x + i khat_y)^M
// of a mode n, written as Q(nz/|n|) az / |n|^M with the azimuthal factor
// az = Re|Im (nx + i ny)^M of the mode's (x, y) column, which every mode of a
// z-run shares: per mode a polynomial in nz/|n| and M products.
template <typename T>
__device__ __forceinline__ T column_azimuth(const KSpec<T>& h, int nx, int ny) {
  T er = 1, ei = 0;
  for (int m = 0; m < h.M; ++m) {
    const T tr = er * static_cast<T>(nx) - ei * static_cast<T>(ny);
    ei = er * static_cast<T>(ny) + ei * static_cast<T>(nx);
    er = tr;
  }
  return h.cs ? ei : er;
}
// (The polynomial takes a fixed number of terms, five up to degree 4, else
// nine: the coefficients past nq are zero, so the leading steps give exact
// zeros, and no per-mode loop reads the count and the coefficients again.)
template <typename T>
__device__ __forceinline__ T harmonic_of_column(const KSpec<T>& h, T az, int nz, T rq) {
  const T u = static_cast<T>(nz) * rq;
  T Q;
  if (h.nq <= 5) {
    Q = h.q[4];
#pragma unroll
    for (int i = 3; i >= 0; --i) Q = Q * u + h.q[i];
  } else {
    Q = h.q[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) Q = Q * u + h.q[i];
  }
  T sc = az;
  for (int m = 0; m < h.M; ++m) sc *= rq;
  return Q * sc;
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

// Column pairs (density kernels).  A unit is one chunk of kPairChunk (or
// fewer) consecutive c of one column A: unit u = column + (N * N/2) * chunk,
// the column x + N y, so that the lanes of a wavefront take consecutive x of
// the same z-groups (contiguous 64-byte runs in A, and in reverse order in M).
__host__ __device__ inline int pair_chunk(int N) { return N / kRun < (N >= 512 ? 16 : 4) ? N / kRun : (N >= 512 ? 16 : 4); }
__host__ __device__ inline int64_t pair_units(int N) {
  return static_cast<int64_t>(N) * (N / 2) * (N / kRun / pair_chunk(N));
}

struct PairUnit {
  int ix, iy, mx, my, nx, ny, qxy;
  int c0, c1;  // this unit's c range (inclusive), inside the live range of the column
  int clo;     // the column's first live c
  bool self;   // A is its own mirror (the column (0, 0))
};

// largest s with s * s <= v (v >= 0)
__device__ __forceinline__ int isqrt_floor(int v) {
  int s = static_cast<int>(sqrtf(static_cast<float>(v)));
  while (s * s > v) --s;
  while ((s + 1) * (s + 1) <= v) ++s;
  return s;
}

// the unit's column pair and chunk; false if nothing of it lies inside the
// last shell (qmax <= (N/2)^2, so the live range of c stays in [0, N/8))
__device__ __forceinline__ bool pair_unit(int64_t u, int N, int qmax, int C, PairUnit& p) {
  const int64_t half = static_cast<int64_t>(N) * (N / 2);
  const int k = static_cast<int>(u / half);
  const int r = static_cast<int>(u - k * half);
  p.ix = r % N;
  p.iy = r / N;  // < N/2
  if (p.iy == 0 && p.ix >= N / 2) return false;  // mirrors of (x, 0), 0 < x < N/2; (N/2, 0) is never inside
  p.nx = sgn_mode(p.ix, N);
  p.ny = p.iy;
  p.qxy = p.nx * p.nx + p.ny * p.ny;
  if (p.qxy >= qmax) return false;
  const int zl = isqrt_floor(qmax - 1 - p.qxy);  // largest |nz| inside
  const int H = N / (2 * kRun);
  p.clo = H - (zl + kRun - 1) / kRun;
  const int chi = H + zl / kRun;
  p.c0 = max(k * C, p.clo);
  p.c1 = min(k * C + C - 1, chi);
  if (p.c0 > p.c1) return false;
  p.mx = (N - p.ix) & (N - 1);
  p.my = (N - p.iy) & (N - 1);
  p.self = p.ix == 0 && p.iy == 0;
  return true;
}

// z-group of A at position c of the walk, and the start of a z-group's run
__device__ __forceinline__ int pair_group(int c, int N) { return (c + N / (2 * kRun)) % (N / kRun); }
__device__ __forceinline__ int64_t group_run(int x, int y, int g, int N) {
  return ((static_cast<int64_t>(g) * N + y) * N + x) * kRun;
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

// thresholds to LDS, every row to zero (NW wavefronts); returns this wavefront's row
template <int NW = kBinWaves>
__device__ __forceinline__ double* rows_init(unsigned char* dyn, size_t off, int width, const int64_t* thr, int* sthr,
                                             int nb) {
  double* rows = reinterpret_cast<double*>(dyn + off);
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) sthr[i] = static_cast<int>(thr[i]);
  for (int i = threadIdx.x; i < NW * width; i += blockDim.x) rows[i] = 0.0;
  __syncthreads();
  return rows + (threadIdx.x >> 6) * width;
}

// the block's partial row (the wavefront rows added in order), stored
// column-major, [width][gridDim.x], for a coalesced reduction
template <int NW = kBinWaves>
__device__ __forceinline__ void rows_store(const unsigned char* dyn, size_t off, int width, double* partial) {
  const double* rows = reinterpret_cast<const double*>(dyn + off);
  __syncthreads();
  for (int i = threadIdx.x; i < width; i += blockDim.x) {
    double v = rows[i];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += rows[w * width + i];
    partial[static_cast<int64_t>(i) * gridDim.x + blockIdx.x] = v;
  }
}

// ---- the bases: B = F at every mode inside the last shell, with |F|^2, the
// mode count and the sum of |n| per shell (rows [re, im, counts, sum |n|]) ----

// density base from the packed pair of real copies over column pairs: B is
// written at every mode of A and, as conj(F), at the mirrors in M (whole
// runs: group N/8 - 1 - g of M once the next step has its element 0; the
// unit's last one with an extra element of A)
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
  const int G8 = N / kRun, C = pair_chunk(N);
  const int64_t units = pair_units(N);
  Acc acc{-1, 0, 0, 0, 0};
  for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < units;
       u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    PairUnit pu;
    if (!pair_unit(u, N, qmax, C, pu)) continue;
    const T wxy = invw[pu.ix] * invw[pu.iy];
    const T2 pxy = phase[pu.nx + pu.ny + 3 * N / 2];
    const double wt = pu.self ? 1.0 : 2.0;
    // F at z-index iz of A from P there and at its mirror
    auto unpack = [&](T2 pa, T2 pm, int iz) -> T2 {
      const T2 f1{static_cast<T>(0.5) * (pa.x + pm.x), static_cast<T>(0.5) * (pa.y - pm.y)};
      const T2 f2{static_cast<T>(0.5) * (pa.y + pm.y), static_cast<T>(-0.5) * (pa.x - pm.x)};
      return combine<T, T2>(f1, f2, a.interlace, cmul(pxy, px[sgn_mode(iz, N) + N / 2]), wxy * iw[iz]);
    };
    int g = pair_group(pu.c0, N);
    // element 0 of the mirror group of the step before the first: the mirror of A's z = 8g
    T2 carry = P[group_run(pu.mx, pu.my, (G8 - g) % G8, N)];
    T2 bm[kRun];  // B of the previous step's mirror group (element 0 pending)
    for (int c = pu.c0; c <= pu.c1; ++c, g = pair_group(c, N)) {
      const int gm = G8 - 1 - g;
      const int64_t run = group_run(pu.ix, pu.iy, g, N), mrun = group_run(pu.mx, pu.my, gm, N);
      T2 pa[kRun], pm[kRun], fa[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) pa[j] = P[run + j];
#pragma unroll
      for (int j = 0; j < kRun; ++j) pm[j] = P[mrun + j];
#pragma unroll
      for (int j = 0; j < kRun; ++j) fa[j] = unpack(pa[j], j ? pm[kRun - j] : carry, kRun * g + j);
#pragma unroll
      for (int j = 0; j < kRun; ++j) B[run + j] = fa[j];
      if (!pu.self) {
        const int64_t prev = group_run(pu.mx, pu.my, (gm + 1) % G8, N);
        if (c > pu.c0) {
          bm[0] = T2{fa[0].x, -fa[0].y};
#pragma unroll
          for (int j = 0; j < kRun; ++j) B[prev + j] = bm[j];
        } else if (c == pu.clo) {
          // the column's first live group: its element 0's mirror has no earlier step
          const int nz = sgn_mode(kRun * g, N);
          if (pu.qxy + nz * nz < qmax) B[prev] = T2{fa[0].x, -fa[0].y};
        }
#pragma unroll
        for (int j = 1; j < kRun; ++j) bm[j] = T2{fa[kRun - j].x, -fa[kRun - j].y};
      }
#pragma unroll
      for (int j = 0; j < kRun; ++j) {
        const int nz = sgn_mode(kRun * g + j, N);
        const int q = pu.qxy + nz * nz;
        const int b = shell_of(q, sthr, nb, inv_dn);
        if (b < 0) continue;
        acc_add<true>(acc, b, wt * (static_cast<double>(fa[j].x) * fa[j].x + static_cast<double>(fa[j].y) * fa[j].y),
                      0.0, wt, wt * sqrt(static_cast<double>(q)), sre, sim, scnt, sks);
      }
      carry = pm[0];
    }
    if (!pu.self) {
      // the last mirror group's element 0 is the mirror of element 0 of A's next group
      const int gn = (pair_group(pu.c1, N) + 1) % G8;
      const T2 f = unpack(P[group_run(pu.ix, pu.iy, gn, N)], carry, kRun * gn);
      bm[0] = T2{f.x, -f.y};
      const int64_t last = group_run(pu.mx, pu.my, G8 - 1 - pair_group(pu.c1, N), N);
#pragma unroll
      for (int j = 0; j < kRun; ++j) B[last + j] = bm[j];
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
  const int G8 = N / kRun, C = pair_chunk(N);
  const int64_t units = pair_units(N);
  int cur[NFB];
  double sr[NFB];
#pragma unroll
  for (int f = 0; f < NFB; ++f) {
    cur[f] = -1;
    sr[f] = 0.0;
  }
  for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < units;
       u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    PairUnit pu;
    if (!pair_unit(u, N, qmax, C, pu)) continue;
    const T wxy = invw[pu.ix] * invw[pu.iy];
    const T2 pxy = phase[pu.nx + pu.ny + 3 * N / 2];
    const double wt = pu.self ? 1.0 : 2.0;
    int gA = pair_group(pu.c0, N);
    T2 carry[NFB];  // element 0 of the previous step's mirror group, per field
    {
      const int64_t prev = group_run(pu.mx, pu.my, (G8 - gA) % G8, N);
#pragma unroll
      for (int f = 0; f < NFB; ++f) carry[f] = g.P[f][prev];
    }
    for (int c = pu.c0; c <= pu.c1; ++c, gA = pair_group(c, N)) {
      const int64_t run = group_run(pu.ix, pu.iy, gA, N), mrun = group_run(pu.mx, pu.my, G8 - 1 - gA, N);
      T2 bv[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) bv[j] = B[run + j];
      int bq[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) {
        const int nz = sgn_mode(kRun * gA + j, N);
        bq[j] = shell_of(pu.qxy + nz * nz, sthr, nb, inv_dn);
      }
#pragma unroll
      for (int f = 0; f < NFB; ++f) {
        const T2* __restrict__ P = g.P[f];
        const T az = column_azimuth(g.h[f], pu.nx, pu.ny);
        T2 pa[kRun], pm[kRun];
#pragma unroll
        for (int j = 0; j < kRun; ++j) pa[j] = P[run + j];
#pragma unroll
        for (int j = 0; j < kRun; ++j) pm[j] = P[mrun + j];
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
          const int b = bq[j];
          if (b < 0) continue;
          const int iz = kRun * gA + j, nz = sgn_mode(iz, N);
          const T2 m = j ? pm[kRun - j] : carry[f];
          const T2 f1{static_cast<T>(0.5) * (pa[j].x + m.x), static_cast<T>(0.5) * (pa[j].y - m.y)};
          const T2 f2{static_cast<T>(0.5) * (pa[j].y + m.y), static_cast<T>(-0.5) * (pa[j].x - m.x)};
          const T2 F = combine<T, T2>(f1, f2, a.interlace, cmul(pxy, px[nz + N / 2]), wxy * iw[iz]);
          const T hk = harmonic_of_column(g.h[f], az, nz, inv_sqrt<T>(pu.qxy + nz * nz));
          if (b != cur[f]) {
            if (cur[f] >= 0) atomicAdd(&v[2 * f * nb + cur[f]], sr[f]);
            cur[f] = b;
            sr[f] = 0.0;
          }
          // Re[h F conj(B)] for both modes of the pair (once each in the self-mirrored column)
          sr[f] += wt * static_cast<double>(hk * (F.x * bv[j].x + F.y * bv[j].y));
        }
        carry[f] = pm[0];
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
      const T az = column_azimuth(g.h[f], nx, ny);
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
        const T hk = harmonic_of_column(g.h[f], az, nz, inv_sqrt<T>(nx * nx + ny * ny + nz * nz));
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

// ---- the z pass of complex fields fused with their shell sums ----
//
// The last transform pass (along z) of a group's fields is followed at once
// by the shell sums, so that the transformed fields are never written to HBM
// and read back.  A workgroup takes NL adjacent columns x of one row y (the
// z pass's lines: N/8 threads per column, the same pruning as in
// fft_zb_kernel) and, field by field, transforms the grid copy and the
// interlaced copy of every column, combines the two in registers and passes
// the combined modes through LDS, after which each thread holds one z-group
// run of one column: the run's shells are found once for all fields of the
// group (its base values are read per field, from the L2 after the first),
// and the sums go, as in bin_gg_group_kernel, to the thread's wavefront's LDS
// row (fields in order, so two runs are bitwise equal).  Workgroups walk the
// (column block, y) items in a stride of the grid; a block outside the last
// shell is skipped whole.
template <typename T>
struct ZbGroup {
  KSpec<T> h[kBinGroupMax];
  const typename V2<T>::type* g1[kBinGroupMax];  // grid copies after the x and y passes
  const typename V2<T>::type* g2[kBinGroupMax];  // interlaced copies (unused without interlacing)
  int n;
};

template <typename T, int N, int NL>
constexpr int zbin_waves() {
  return (NL * (N / 8) + 63) / 64;
}

// Waves per SIMD the kernel keeps registers for (its launch bound): four in
// FP32 (at most 128 VGPRs), three in FP64 (168); the fields per launch are then
// chosen so that the LDS of a workgroup (lines, tables, shell rows) lets that
// many waves reside (zbin_group_max).
template <typename T>
constexpr int zbin_waves_per_simd() {
  return sizeof(T) == 4 ? 4 : 3;
}
// the per-axis tables in LDS in FP32; FP64 reads them from the global tables
// (cached), which leaves the LDS for a third workgroup per CU
template <typename T, int N>
constexpr size_t zbin_tables_lds() {
  return sizeof(T) == 4 ? rows_offset<T>(N) : 0;
}
template <typename T, int N, int NL>
constexpr int zbin_min_waves() {
  constexpr int own = (NL * (N / 8) + 255) / 256;  // one workgroup's waves per SIMD
  return own > zbin_waves_per_simd<T>() ? own : zbin_waves_per_simd<T>();
}

// KIND 0: h F conj(B(k)); KIND 1: h F B(-k)
template <typename T, int N, int NL, int KIND>
__global__ void __launch_bounds__(NL* N / 8, (zbin_min_waves<T, N, NL>())) zbin_gg_kernel(BinArgs a, ZbGroup<T> g,
                                                             const typename V2<T>::type* __restrict__ B,
                                                             const typename V2<T>::type* __restrict__ tw,
                                                             const uint8_t* __restrict__ plane) {
  using T2 = typename V2<T>::type;
  constexpr int TL = N / 8;
  constexpr int NT = NL * TL;
  constexpr int NW = zbin_waves<T, N, NL>();
  static_assert(NL <= N / 2 && (N / 2) % NL == 0, "column blocks inside one half of the kx range");
  __shared__ T2 sm[NL * N];
  __shared__ T2 stw[N];
  __shared__ int sthr[kMaxBins + 1];
  extern __shared__ __align__(16) unsigned char dyn[];
  const int nb = a.nb, n = g.n;
  constexpr size_t roff = zbin_tables_lds<T, N>();
  const T2* px;
  const T* iw;
  if constexpr (roff > 0) {
    T2* lpx = reinterpret_cast<T2*>(dyn);
    T* liw = reinterpret_cast<T*>(lpx + N);
    tables_init<T>(a, lpx, liw);
    px = lpx;
    iw = liw;
  } else {
    px = static_cast<const T2*>(a.phase) + N;  // (as tables_init: nx = i - N/2 at i + N)
    iw = static_cast<const T*>(a.invw);
  }
  for (int i = threadIdx.x; i < N; i += NT) stw[i] = tw[i];
  const int width = 2 * n * nb;
  double* v = rows_init<NW>(dyn, roff, width, a.thr, sthr, nb);  // (ends with a barrier)
  const T2* phase = static_cast<const T2*>(a.phase);
  const T* invw = static_cast<const T*>(a.invw);
  const int qmax = sthr[nb];
  const float inv_dn = static_cast<float>(nb) / sqrtf(static_cast<float>(qmax));
  constexpr int mask = N - 1;
  constexpr int64_t hi = static_cast<int64_t>(N) * N * kZb;  // z-group stride
  const int tid = threadIdx.x;
  // the thread's transform line (as the z pass) ...
  int col, t, swz;
  if constexpr (TL >= 8) {
    col = (tid >> 3) % NL;
    t = (tid & 7) | ((tid / (8 * NL)) << 3);
    swz = dev::swizzle_rows8<N>(col);
  } else {
    col = tid % NL;
    t = tid / NL;
    swz = col & 15;
  }
  // ... and its run for the sums: column rc, z-group rg (one run per thread)
  const int rc = tid % NL, rg = tid / NL;
  const int rswz = TL >= 8 ? dev::swizzle_rows8<N>(rc) : (rc & 15);
  const int z0 = rg * kRun;
  constexpr int nitems = (N / NL) * N;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int xc = item % (N / NL), y = item / (N / NL);
    const int c0 = xc * NL;
    const int mxb = c0 < N / 2 ? c0 : N - c0 - (NL - 1);  // the block's smallest |nx|
    const int ny = sgn_mode(y, N);
    if (mxb * mxb + ny * ny >= qmax) continue;  // (uniform over the block)
    const int x = c0 + col, nx = sgn_mode(x, N);
    const bool live = nx * nx + ny * ny < qmax;
    const int64_t lbase = zb_index(x, y, 0, N);
    bool rd[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) rd[j] = live && (plane == nullptr || plane[t + j * TL] != 0);
    const T wxy = invw[x] * invw[y];
    const T2 pxy = phase[nx + ny + 3 * N / 2];
    const int rx = c0 + rc, rnx = sgn_mode(rx, N);
    const int qxy = rnx * rnx + ny * ny;
    const bool rlive = run_live(z0, N, qxy, qmax);
    int bq[kRun];  // the run's shells (-1: outside the last shell)
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      const int nz = sgn_mode(z0 + j, N);
      bq[j] = rlive ? shell_of(qxy + nz * nz, sthr, nb, inv_dn) : -1;
    }
#pragma unroll 1
    for (int f = 0; f < n; ++f) {
      // Opaque copies of the line position and the run start: what depends
      // on them only (load offsets, LDS addresses of the transform's
      // exchanges, output rows, the modes' unit vectors) is then recomputed
      // where it is used instead of being held in registers across the field
      // loop and the transforms, which would halve the occupancy.
      // (The masks restore the ranges the asm hides, no-ops on the values:
      // with t < N/8 and the swizzle below 64 the exchanges' row addresses
      // t + j N/8 become one base plus immediate offsets.)
      int tq = t, cq = col, sq = swz, zq = z0;
      asm volatile("" : "+v"(tq), "+v"(cq), "+v"(sq), "+v"(zq));
      tq &= TL - 1;
      cq &= NL - 1;
      sq &= (TL >= 8 ? 63 : 15);
      // both copies' loads in flight before the first transform (element e
      // = t + j N/8 of a line sits at (e >> 3) hi + (e & 7): with N/8 a
      // multiple of 8 that is the thread's first element plus j (N/64) hi)
      T2 v1[8], w[8];
      {
        int64_t off0;
        constexpr int64_t jstep = TL >= 8 ? (TL / 8) * hi : 0;
        if constexpr (TL >= 8) off0 = lbase + (tq >> 3) * hi + (tq & 7);
        else off0 = lbase;
        auto off = [&](int j) -> int64_t {
          if constexpr (TL >= 8) return off0 + j * jstep;
          const int e = tq + j * TL;
          return off0 + (e >> 3) * hi + (e & 7);
        };
        const T2* __restrict__ s1 = g.g1[f];
#pragma unroll
        for (int j = 0; j < 8; ++j) v1[j] = rd[j] ? dev::nt_load(s1 + off(j)) : T2{0, 0};
        if (a.interlace) {
          const T2* __restrict__ s2 = g.g2[f];
#pragma unroll
          for (int j = 0; j < 8; ++j) w[j] = rd[j] ? dev::nt_load(s2 + off(j)) : T2{0, 0};
        }
      }
      dev::fft_column_regs<T, N>(stw, sm, cq, tq, v1, sq);
      if (a.interlace) {
        asm volatile("" : "+v"(tq), "+v"(cq), "+v"(sq));
        tq &= TL - 1;
        cq &= NL - 1;
        sq &= (TL >= 8 ? 63 : 15);
        dev::fft_column_regs<T, N>(stw, sm, cq, tq, w, sq);
      }
      asm volatile("" : "+v"(tq), "+v"(cq), "+v"(sq));
      tq &= TL - 1;
      cq &= NL - 1;
      sq &= (TL >= 8 ? 63 : 15);
      // combined, compensated modes of the lines to LDS, runs back
      int row[8];
      dev::fft_rows<N>(tq, row);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int iz = row[q];  // (signed mode nz at nz + N/2 = iz ^ N/2 of the phase table)
        sm[dev::sidx<N>(cq, iz, sq)] =
            combine<T, T2>(v1[q], w[q], a.interlace, cmul(pxy, px[iz ^ (N / 2)]), wxy * iw[iz]);
      }
      __syncthreads();
      T2 F[kRun];
#pragma unroll
      for (int j = 0; j < kRun; ++j) F[j] = sm[dev::sidx<N>(rc, zq + j, rswz)];
      __syncthreads();  // (sm is the next transform's exchange buffer)
      if (rlive) {
        // the run's base values (again for every field, from the L2 after
        // the first: held across the transforms they would cost registers
        // and with them occupancy)
        T2 bv[kRun];
        const int64_t run = zb_index(rx, y, zq, N);
        const int mx = (N - rx) & mask, my = (N - y) & mask;
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
          bv[j] = T2{0, 0};
          if (KIND == 0) bv[j] = B[run + j];
          else if (bq[j] >= 0) bv[j] = B[zb_index(mx, my, (N - zq - j) & mask, N)];
        }
        const KSpec<T> h = g.h[f];  // (a copy: the field's coefficients read once)
        const T az = column_azimuth(h, rnx, ny);
        int cur = -1;
        double sre = 0.0, sim = 0.0;
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
          const int b = bq[j];
          if (b < 0) continue;
          const int nz = sgn_mode(zq + j, N);
          const T hk = harmonic_of_column(h, az, nz, inv_sqrt<T>(qxy + nz * nz));
          const T2 p = KIND == 0 ? cmulc(F[j], bv[j]) : cmul(F[j], bv[j]);
          if (b != cur) {
            if (cur >= 0) {
              atomicAdd(&v[2 * f * nb + cur], sre);
              atomicAdd(&v[(2 * f + 1) * nb + cur], sim);
            }
            cur = b;
            sre = sim = 0.0;
          }
          sre += static_cast<double>(hk * p.x);
          sim += static_cast<double>(hk * p.y);
        }
        if (cur >= 0) {
          atomicAdd(&v[2 * f * nb + cur], sre);
          atomicAdd(&v[(2 * f + 1) * nb + cur], sim);
        }
      }
    }
  }
  rows_store<NW>(dyn, roff, width, a.partial);
}

// one block per column c: strided partial sums, then a fixed-shape tree
// (deterministic).  With n fields, column c of field i (partial column
// i width + c) is added to dst.d[i][c], field by field in order: fields of
// one launch that feed the same series (the 2L + 1 harmonics of one
// multipole) add to the same row, as one launch per field would.
constexpr int kRedThreads = 256;
struct RowDst {
  double* d[kBinGroupMax];
};
__global__ void __launch_bounds__(kRedThreads) reduce_partials_kernel(const double* __restrict__ partial, int nblocks,
                                                                      int width, int n, RowDst dst) {
  __shared__ double sh[kRedThreads];
  const int c = blockIdx.x;
  for (int i = 0; i < n; ++i) {
    const double* col = partial + (static_cast<int64_t>(i) * width + c) * nblocks;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) s += col[b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) dst.d[i][c] += sh[0];
    __syncthreads();  // sh is reused by the next field
  }
}

}  // namespace

int pair_bin_blocks(int N, int nblocks) {
  const int64_t want = (pair_units(N) + kBinThreads - 1) / kBinThreads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, nblocks)));
}

int bin_group_max(bool complex_fields, bool fp64, int nb) {
  const int by_regs = (complex_fields && !fp64) ? kBinGroupMax : kBinGroup;
  const int by_lds = (4 * kMaxBins) / (2 * std::max(1, nb));  // LDS rows of 2 n nb sums per wavefront
  return std::max(1, std::min(by_regs, by_lds));
}

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
  if (a.nb > kMaxBins || a.qmax > a.N * a.N / 4) return hipErrorInvalidValue;
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
  if (a.nb > kMaxBins || 2 * n * a.nb > 4 * kMaxBins || a.qmax > a.N * a.N / 4) return hipErrorInvalidValue;
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
    case 5:  // FP32 only: five fields keep three waves per SIMD (155 VGPRs)
      if constexpr (sizeof(T) == 4) return bin_gg_group_n<T, KIND, 5>(a, f, g1, g2, base, st);
      else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_bin_gg(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2,
                         int n, const void* base, int kind, hipStream_t st) {
  if (a.nb > kMaxBins || 2 * n * a.nb > 4 * kMaxBins) return hipErrorInvalidValue;
  return kind == 0 ? bin_gg_kind<T, 0>(a, f, g1, g2, n, base, st) : bin_gg_kind<T, 1>(a, f, g1, g2, n, base, st);
}

namespace {

// columns per workgroup of the fused kernel: 4 (runs of 256 contiguous bytes
// in FP32, 512 in FP64).  Small workgroups keep the LDS per wave low: at 512^3
// in FP32 four workgroups of 256 threads with three fields' shell rows reside
// per CU (16 waves), against two of 512 threads with eight columns (the
// shape shell sums 27.2 -> 25.1 ms per estimate).
constexpr int zbin_lines(bool /*fp64*/) { return 4; }

}  // namespace

// workgroups of the fused kernel for a budget of nblocks: at most one per
// item, and an odd count when fewer: a workgroup's items lie a grid stride
// apart, and with an even stride (a multiple of the N/4 column blocks of a
// row) they would all be the same column block, so that the workgroups of
// the outer blocks, with few items inside the last shell, finished early
// while the inner ones ran on (shape shell sums 25.1 -> 24.6 ms at 512^3)
int zbin_blocks(int N, bool fp64, int nblocks) {
  const int items = (N / zbin_lines(fp64)) * N;
  const int g = std::max(1, std::min(items, nblocks));
  return g < items && g % 2 == 0 ? g - 1 : g;
}

namespace {

// dynamic LDS (the per-axis tables and a row of 2 n nb sums per wavefront),
// and all of it with the static arrays (lines, twiddles, thresholds)
template <typename T, int N>
size_t zbin_dyn_lds(int n, int nb) {
  constexpr int NW = zbin_waves<T, N, zbin_lines(sizeof(T) == 8)>();
  return zbin_tables_lds<T, N>() + 8 * static_cast<size_t>(NW) * 2 * n * nb;
}
template <typename T, int N>
size_t zbin_lds(int n, int nb) {
  constexpr int NL = zbin_lines(sizeof(T) == 8);
  return static_cast<size_t>(NL + 1) * N * sizeof(typename V2<T>::type) + 4 * (kMaxBins + 1) + zbin_dyn_lds<T, N>(n, nb);
}

template <typename T, int N>
int zbin_group_max_n(int nb) {
  // the most fields per launch that keep the workgroups per CU of one field:
  // as many as the launch bound's waves allow, if the LDS holds them
  constexpr int threads = zbin_lines(sizeof(T) == 8) * (N / 8);
  constexpr int block_waves = (threads + 63) / 64;
  constexpr int by_waves = 4 * zbin_waves_per_simd<T>() / block_waves > 0 ? 4 * zbin_waves_per_simd<T>() / block_waves : 1;
  auto blocks = [&](int n) { return std::min<size_t>(by_waves, (160 * 1024) / zbin_lds<T, N>(n, nb)); };
  if (blocks(1) < 1) return 0;
  const int cap = sizeof(T) == 4 ? kBinGroupMax : kBinGroup;
  int n = 1;
  while (n < cap && blocks(n + 1) >= blocks(1)) ++n;
  return n;
}

template <typename T, int N, int KIND>
hipError_t zbin_launch(const BinArgs& a, const ZbGroup<T>& g, const void* base, const void* tw, const uint8_t* plane,
                       hipStream_t st) {
  using T2 = typename V2<T>::type;
  constexpr int NL = zbin_lines(sizeof(T) == 8);
  const int grid = zbin_blocks(N, sizeof(T) == 8, a.nblocks);
  zbin_gg_kernel<T, N, NL, KIND><<<grid, NL * (N / 8), zbin_dyn_lds<T, N>(g.n, a.nb), st>>>(
      a, g, static_cast<const T2*>(base), static_cast<const T2*>(tw), plane);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t zbin_n(const BinArgs& a, const ZbGroup<T>& g, const void* base, int kind, const void* tw,
                  const uint8_t* plane, hipStream_t st) {
  if (g.n < 1 || g.n > zbin_group_max_n<T, N>(a.nb)) return hipErrorInvalidValue;
  return kind == 0 ? zbin_launch<T, N, 0>(a, g, base, tw, plane, st) : zbin_launch<T, N, 1>(a, g, base, tw, plane, st);
}

}  // namespace

int zbin_group_max(int N, bool fp64, int nb) {
  if (nb < 1 || nb > kMaxBins) return 0;
  switch (N) {
    case 16: return fp64 ? zbin_group_max_n<double, 16>(nb) : zbin_group_max_n<float, 16>(nb);
    case 32: return fp64 ? zbin_group_max_n<double, 32>(nb) : zbin_group_max_n<float, 32>(nb);
    case 64: return fp64 ? zbin_group_max_n<double, 64>(nb) : zbin_group_max_n<float, 64>(nb);
    case 128: return fp64 ? zbin_group_max_n<double, 128>(nb) : zbin_group_max_n<float, 128>(nb);
    case 256: return fp64 ? zbin_group_max_n<double, 256>(nb) : zbin_group_max_n<float, 256>(nb);
    case 512: return fp64 ? zbin_group_max_n<double, 512>(nb) : zbin_group_max_n<float, 512>(nb);
    case 1024: return fp64 ? zbin_group_max_n<double, 1024>(nb) : zbin_group_max_n<float, 1024>(nb);
    default: return 0;
  }
}

template <typename T>
hipError_t launch_zbin_gg(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2,
                          int n, const void* base, int kind, const void* tw, const uint8_t* plane, hipStream_t st) {
  using T2 = typename V2<T>::type;
  // (the partial rows hold 2 kBinGroupMax nb sums per workgroup; the LDS
  // bound on n is checked per N)
  if (a.nb < 1 || a.nb > kMaxBins || n < 1 || n > kBinGroupMax) return hipErrorInvalidValue;
  ZbGroup<T> g{};
  g.n = n;
  for (int i = 0; i < n; ++i) {
    g.h[i] = kspec_of<T>(*f[i]);
    g.g1[i] = static_cast<const T2*>(g1[i]);
    g.g2[i] = static_cast<const T2*>(g2 ? g2[i] : g1[i]);
  }
  switch (a.N) {
    case 16: return zbin_n<T, 16>(a, g, base, kind, tw, plane, st);
    case 32: return zbin_n<T, 32>(a, g, base, kind, tw, plane, st);
    case 64: return zbin_n<T, 64>(a, g, base, kind, tw, plane, st);
    case 128: return zbin_n<T, 128>(a, g, base, kind, tw, plane, st);
    case 256: return zbin_n<T, 256>(a, g, base, kind, tw, plane, st);
    case 512: return zbin_n<T, 512>(a, g, base, kind, tw, plane, st);
    case 1024: return zbin_n<T, 1024>(a, g, base, kind, tw, plane, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_partials(const double* partial, int nblocks, int width, double* acc, hipStream_t st) {
  RowDst dst{};
  dst.d[0] = acc;
  reduce_partials_kernel<<<width, kRedThreads, 0, st>>>(partial, nblocks, width, 1, dst);
  return hipGetLastError();
}

hipError_t launch_reduce_partials_group(const double* partial, int nblocks, int width, int n, double* const* acc,
                                        hipStream_t st) {
  if (n < 1 || n > kBinGroupMax) return hipErrorInvalidValue;
  RowDst dst{};
  for (int i = 0; i < n; ++i) dst.d[i] = acc[i];
  reduce_partials_kernel<<<width, kRedThreads, 0, st>>>(partial, nblocks, width, n, dst);
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
template hipError_t launch_zbin_gg<float>(const BinArgs&, const FieldSpec* const*, const void* const*,
                                          const void* const*, int, const void*, int, const void*, const uint8_t*,
                                          hipStream_t);
template hipError_t launch_zbin_gg<double>(const BinArgs&, const FieldSpec* const*, const void* const*,
                                           const void* const*, int, const void*, int, const void*, const uint8_t*,
                                           hipStream_t);
template hipError_t launch_bin_dd<float>(const BinArgs&, const FieldSpec* const*, const void* const*, int, const void*,
                                         hipStream_t);
template hipError_t launch_bin_dd<double>(const BinArgs&, const FieldSpec* const*, const void* const*, int,
                                          const void*, hipStream_t);

}  // namespace lpp
