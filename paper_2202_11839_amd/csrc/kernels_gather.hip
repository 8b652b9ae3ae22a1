// Mass assignment as a gather over cell-sorted objects.
//
// Objects are counting-sorted by mesh cell (cell_start[c] .. cell_start[c+1]
// are the objects whose position lies in cell c).  One workgroup owns a tile
// of TT^3 mesh nodes; the nodes of the tile can only receive weight from
// objects in the (TT+3)^3 cells [t0-2, t0+TT] on each axis (the TSC stencil
// of the grid reaches nodes c-1..c+2 of an object in cell c, the interlaced
// grid nodes c-1..c+1).  The workgroup stages those objects in LDS (in
// chunks of CAP objects), computing each object's line-of-sight weighted
// value once, and every thread then sums the contributions to one x-row of TT
// nodes in registers, in a fixed order.  Every node of the mesh is written
// exactly once with a plain store: no atomics, no separate clearing pass, and
// the result is bitwise reproducible.
#include "lpp_internal.h"

namespace lpp {

namespace {

template <typename T>
struct V2;
template <>
struct V2<float> {
  using type = float2;
};
template <>
struct V2<double> {
  using type = double2;
};

template <typename T>
struct SpecT {
  int s, L, M, cs;
  int nq[5];
  T q[5][9];
  T binom[5];
  T scale;
};

template <typename T>
SpecT<T> to_spec(const FieldSpec& f) {
  SpecT<T> o{};
  o.s = f.s;
  o.L = f.L;
  o.M = f.M;
  o.cs = f.cs;
  for (int j = 0; j < 5; ++j) {
    o.nq[j] = f.nq[j];
    o.binom[j] = static_cast<T>(f.binom[j]);
    for (int i = 0; i < 9; ++i) o.q[j][i] = static_cast<T>(f.q[j][i]);
  }
  o.scale = static_cast<T>(f.scale);
  return o;
}

template <typename T>
__device__ __forceinline__ T ipow(T b, int e) {
  T r = static_cast<T>(1);
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// s! [t^s] h_{L,M,cs}(xhat + t m) * kappa_{LM}, with m = e_theta - i e_phi (see FieldSpec).
template <typename T>
__device__ __forceinline__ void los_weight(const SpecT<T>& f, T ct, T st, T cp, T sp, T& gr, T& gi) {
  T er = 1, ei = 0;
  for (int m = 0; m < f.M; ++m) {
    const T t = er * cp - ei * sp;
    ei = er * sp + ei * cp;
    er = t;
  }
  T accr = 0, acci = 0;
  T stj = 1;
  for (int j = 0; j <= f.s; ++j) {
    const int jj = f.s - j;
    if (jj <= f.M) {
      T Q = 0;
      for (int i = f.nq[j] - 1; i >= 0; --i) Q = Q * ct + f.q[j][i];
      Q *= stj;
      const T base = f.binom[j] * ipow(st, f.M - jj);
      const T A = base * ipow(static_cast<T>(1) + ct, jj);
      const T B = base * ipow(ct - static_cast<T>(1), jj);
      if (f.cs == 0) {
        accr += static_cast<T>(0.5) * Q * (A + B) * er;
        acci += static_cast<T>(0.5) * Q * (A - B) * ei;
      } else {
        accr += static_cast<T>(0.5) * Q * (A + B) * ei;
        acci -= static_cast<T>(0.5) * Q * (A - B) * er;
      }
    }
    stj *= st;
  }
  gr = f.scale * accr;
  gi = f.scale * acci;
}

// 1D assignment window W_p(x), x = (object - node) in cells.
template <typename T, int P>
__device__ __forceinline__ T window(T x) {
  if (P == 1) return (x >= static_cast<T>(-0.5) && x < static_cast<T>(0.5)) ? static_cast<T>(1) : static_cast<T>(0);
  const T ax = x < 0 ? -x : x;
  if (P == 2) return ax < 1 ? 1 - ax : static_cast<T>(0);
  if (ax < static_cast<T>(0.5)) return static_cast<T>(0.75) - ax * ax;
  if (ax < static_cast<T>(1.5)) {
    const T d = static_cast<T>(1.5) - ax;
    return static_cast<T>(0.5) * d * d;
  }
  return static_cast<T>(0);
}

constexpr int TT = 8;          // tile edge (nodes)
constexpr int R = TT + 3;      // region edge (cells t0-2 .. t0+TT)
constexpr int R3 = R * R * R;
constexpr int kRows = TT * TT;          // x-rows of the tile
constexpr int kParts = 4;               // threads sharing one row's objects
constexpr int kThreads = kRows * kParts;

template <typename T>
constexpr int cap_of() {
  return sizeof(T) == 4 ? 1024 : 832;
}

// inclusive scan of one value per lane across a 64-wide wavefront
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

constexpr int R2 = R * R;  // region rows (y, z)

// MODE 0: packed real field (grid -> .x, interlaced grid -> .y); 1: complex on the
// grid; 2: complex on the interlaced grid.
template <typename T, int P, int MODE>
__global__ void __launch_bounds__(kThreads) gather_kernel(GObjSet<T> o, const uint32_t* __restrict__ cell_start,
                                                          int N, int lgN, int interlace, T H, T relx, T rely, T relz,
                                                          SpecT<T> f, typename V2<T>::type* __restrict__ mesh) {
  using T2 = typename V2<T>::type;
  constexpr int CAP = cap_of<T>();
  // each region row (cells x in [t0x-2, t0x+TT] at fixed y, z) is at most two
  // contiguous ranges of the cell-sorted objects (two when the row wraps)
  __shared__ uint32_t seg_beg[R2][2];
  __shared__ uint32_t seg_cnt[R2];   // objects in the first range
  __shared__ uint32_t roff[R2 + 1];  // offsets of the rows in staging order
  __shared__ T su[5][CAP];           // [0..2] region-local positions, [3..4] values (re, im)
  static_assert(5 * CAP >= 2 * TT * kRows * (kParts - 1), "row reduction reuses the staging buffers");
  static_assert(R2 <= 2 * 64, "row scan uses two values per lane of one wavefront");

  const int nt = N / TT;
  const int tile = blockIdx.x;
  const int tx = tile % nt, ty = (tile / nt) % nt, tz = tile / (nt * nt);
  const int t0x = tx * TT, t0y = ty * TT, t0z = tz * TT;
  const int mask = N - 1;
  const int tid = threadIdx.x;

  if (tid < 64) {
    uint32_t cnt[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = tid * 2 + h;
      cnt[h] = 0;
      if (r < R2) {
        const int ly = r % R, lz = r / R;
        const int gy = (t0y - 2 + ly) & mask, gz = (t0z - 2 + lz) & mask;
        const int64_t rowbase = static_cast<int64_t>(N) * (gy + static_cast<int64_t>(N) * gz);
        const int xa = t0x - 2, xb = t0x + TT;  // inclusive cell range
        int a0, a1, b0, b1;                       // [a0, a1) and [b0, b1) in x
        if (xa < 0) {
          a0 = N + xa; a1 = N; b0 = 0; b1 = xb + 1;
        } else if (xb >= N) {
          a0 = xa; a1 = N; b0 = 0; b1 = xb - N + 1;
        } else {
          a0 = xa; a1 = xb + 1; b0 = 0; b1 = 0;
        }
        const uint32_t sa = cell_start[rowbase + a0], ea = cell_start[rowbase + a1];
        uint32_t sb = 0, eb = 0;
        if (b1 > b0) {
          sb = cell_start[rowbase + b0];
          eb = cell_start[rowbase + b1];
        }
        seg_beg[r][0] = sa;
        seg_beg[r][1] = sb;
        seg_cnt[r] = ea - sa;
        cnt[h] = (ea - sa) + (eb - sb);
      }
    }
    const uint32_t inc = wave_inclusive_scan(cnt[0] + cnt[1]);
    const uint32_t exc = inc - cnt[0] - cnt[1];
    if (tid * 2 < R2) roff[tid * 2] = exc;
    if (tid * 2 + 1 < R2) roff[tid * 2 + 1] = exc + cnt[0];
    if (tid == 63) roff[R2] = inc;
  }
  __syncthreads();
  const uint32_t total = roff[R2];

  // this thread's row: nodes (t0x + k, t0y + ny, t0z + nz), k = 0..TT-1; `part` strides the objects
  const int rowid = tid % kRows, part = tid / kRows;
  const int ny = rowid % TT, nz = rowid / TT;
  T a1[TT], a2[TT];
#pragma unroll
  for (int k = 0; k < TT; ++k) a1[k] = a2[k] = 0;

  for (uint32_t c0 = 0; c0 < total; c0 += CAP) {
    const uint32_t c1 = min(total, c0 + static_cast<uint32_t>(CAP));
    // stage the chunk [c0, c1): each thread takes objects k, finds its row by bisection
    for (uint32_t k = c0 + tid; k < c1; k += kThreads) {
      int lo = 0, hi = R2;  // roff[lo] <= k < roff[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (roff[mid] <= k) lo = mid; else hi = mid;
      }
      const int r = lo;
      const uint32_t j = k - roff[r];
      const uint32_t src = j < seg_cnt[r] ? seg_beg[r][0] + j : seg_beg[r][1] + (j - seg_cnt[r]);
      const uint32_t key = o.key[src];
      const int cx = static_cast<int>(key & mask);
      const int cy = static_cast<int>((key >> lgN) & mask);
      const int cz = static_cast<int>(key >> (2 * lgN));
      const int lx = (cx - t0x + 2) & mask, ly = r % R, lz = r / R;
      const T fx = o.fx[src], fy = o.fy[src], fz = o.fz[src];
      T gr = 1, gi = 0;
      if (f.L > 0 || f.s > 0) {
        const T px = relx + (static_cast<T>(cx) + fx) * H;
        const T py = rely + (static_cast<T>(cy) + fy) * H;
        const T pz = relz + (static_cast<T>(cz) + fz) * H;
        const T rinv = static_cast<T>(1) / sqrt(px * px + py * py + pz * pz);
        const T xx = px * rinv, xy = py * rinv, xz = pz * rinv;
        const T st = sqrt(xx * xx + xy * xy);
        const T cp = st > 0 ? xx / st : static_cast<T>(1);
        const T sp = st > 0 ? xy / st : static_cast<T>(0);
        los_weight(f, xz, st, cp, sp, gr, gi);
      }
      const uint32_t d = k - c0;
      su[0][d] = static_cast<T>(lx) + fx;
      su[1][d] = static_cast<T>(ly) + fy;
      su[2][d] = static_cast<T>(lz) + fz;
      if (MODE == 0) {
        su[3][d] = o.wr[src] * gr;
      } else {
        const T ar = o.wr[src], ai = o.wi[src];
        su[3][d] = ar * gr - ai * gi;
        su[4][d] = ar * gi + ai * gr;
      }
    }
    __syncthreads();
    // gather: rows that can reach this node row are y in [ny, ny+3], z in [nz, nz+3] (region coordinates)
    const T nyc = static_cast<T>(ny + 2), nzc = static_cast<T>(nz + 2);
    for (int dz = 0; dz < 4; ++dz) {
      for (int dy = 0; dy < 4; ++dy) {
        const int row = (ny + dy) + (nz + dz) * R;
        const uint32_t lo = max(roff[row], c0), hi = min(roff[row + 1], c1);
        for (uint32_t k = lo + part; k < hi; k += kParts) {
          const uint32_t d = k - c0;
          const T ux = su[0][d], uy = su[1][d], uz = su[2][d];
          if (MODE == 0) {
            const T v = su[3][d];
            const T w1 = v * window<T, P>(uy - nyc) * window<T, P>(uz - nzc);
            const T w2 = interlace ? v * window<T, P>(uy - nyc - static_cast<T>(0.5)) *
                                         window<T, P>(uz - nzc - static_cast<T>(0.5))
                                   : static_cast<T>(0);
#pragma unroll
            for (int kx = 0; kx < TT; ++kx) {
              const T xk = ux - static_cast<T>(kx + 2);
              a1[kx] += w1 * window<T, P>(xk);
              a2[kx] += w2 * window<T, P>(xk - static_cast<T>(0.5));
            }
          } else {
            const T sh = (MODE == 2) ? static_cast<T>(0.5) : static_cast<T>(0);
            const T wyz = window<T, P>(uy - nyc - sh) * window<T, P>(uz - nzc - sh);
            const T vr = su[3][d] * wyz, vi = su[4][d] * wyz;
#pragma unroll
            for (int kx = 0; kx < TT; ++kx) {
              const T wx = window<T, P>(ux - static_cast<T>(kx + 2) - sh);
              a1[kx] += vr * wx;
              a2[kx] += vi * wx;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // combine the kParts partial rows in a fixed order (the staging buffers are free now)
  T* red = &su[0][0];
  if (part > 0) {
#pragma unroll
    for (int kx = 0; kx < TT; ++kx) {
      red[((part - 1) * kRows + rowid) * 2 * TT + kx] = a1[kx];
      red[((part - 1) * kRows + rowid) * 2 * TT + TT + kx] = a2[kx];
    }
  }
  __syncthreads();
  T2* out = reinterpret_cast<T2*>(&su[0][0]) + (kParts - 1) * kRows * TT;  // after the partial rows
  static_assert(5 * CAP >= 2 * TT * kRows * kParts, "output staging fits after the partial rows");
  if (part == 0) {
#pragma unroll
    for (int q = 1; q < kParts; ++q)
#pragma unroll
      for (int kx = 0; kx < TT; ++kx) {
        a1[kx] += red[((q - 1) * kRows + rowid) * 2 * TT + kx];
        a2[kx] += red[((q - 1) * kRows + rowid) * 2 * TT + TT + kx];
      }
#pragma unroll
    for (int kx = 0; kx < TT; ++kx) out[rowid * TT + kx] = T2{a1[kx], a2[kx]};
  }
  __syncthreads();
  // coalesced store of the tile: each lane writes two adjacent nodes of one x-row
  for (int i = tid; i < kRows * TT / 2; i += kThreads) {
    const int r = i / (TT / 2), kx = 2 * (i % (TT / 2));
    const int yy = r % TT, zz = r / TT;
    const int64_t base = t0x + kx + static_cast<int64_t>(N) * ((t0y + yy) + static_cast<int64_t>(N) * (t0z + zz));
    mesh[base] = out[r * TT + kx];
    mesh[base + 1] = out[r * TT + kx + 1];
  }
}

// ---- counting sort of objects by cell ----

__device__ __forceinline__ int cell_of(double u, int N) {
  int c = static_cast<int>(floor(u));
  return c < 0 ? 0 : (c >= N ? N - 1 : c);
}

__device__ __forceinline__ double ldc(const void* p, int64_t i, int dtype) {
  return dtype == LPP_F64 ? static_cast<const double*>(p)[i] : static_cast<double>(static_cast<const float*>(p)[i]);
}

__global__ void cell_count_kernel(RawCat c, Geometry g, uint32_t* counts, uint32_t* rank, uint32_t* cell_of_obj) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= c.n) return;
  const int N = g.N;
  const int cx = cell_of((ldc(c.x, i, c.dtype) - g.origin[0]) / g.H, N);
  const int cy = cell_of((ldc(c.y, i, c.dtype) - g.origin[1]) / g.H, N);
  const int cz = cell_of((ldc(c.z, i, c.dtype) - g.origin[2]) / g.H, N);
  const uint32_t cell = static_cast<uint32_t>(cx + N * (cy + static_cast<int64_t>(N) * cz));
  cell_of_obj[i] = cell;
  rank[i] = atomicAdd(&counts[cell], 1u);
}

template <typename T>
__global__ void cell_scatter_kernel(RawCat c, Geometry g, double wscale, int shape, const uint32_t* starts,
                                    const uint32_t* rank, const uint32_t* cell_of_obj, GObjSet<T> out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= c.n) return;
  const int N = g.N;
  const double ux = (ldc(c.x, i, c.dtype) - g.origin[0]) / g.H;
  const double uy = (ldc(c.y, i, c.dtype) - g.origin[1]) / g.H;
  const double uz = (ldc(c.z, i, c.dtype) - g.origin[2]) / g.H;
  const int cx = cell_of(ux, N), cy = cell_of(uy, N), cz = cell_of(uz, N);
  const uint32_t cell = cell_of_obj[i];
  const int64_t d = static_cast<int64_t>(starts[cell]) + rank[i];
  out.key[d] = cell;
  out.fx[d] = static_cast<T>(ux - cx);
  out.fy[d] = static_cast<T>(uy - cy);
  out.fz[d] = static_cast<T>(uz - cz);
  const double w = c.w ? ldc(c.w, i, c.dtype) : 1.0;
  if (shape) {
    out.wr[d] = static_cast<T>(w * ldc(c.g1, i, c.dtype));
    out.wi[d] = static_cast<T>(w * ldc(c.g2, i, c.dtype));
  } else {
    out.wr[d] = static_cast<T>(wscale * w);
  }
}

// exclusive scan of n counts into starts[0..n] (starts[n] = total), three phases
constexpr int kScanT = 1024;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanT * kScanPer;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kScanT; o <<= 1) {
    const uint32_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  total = sh[kScanT - 1];
  const uint32_t r = sh[threadIdx.x] - v;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kScanT) scan_reduce_kernel(const uint32_t* in, int64_t n, uint32_t* bsum) {
  __shared__ uint32_t sh[kScanT];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + static_cast<int64_t>(threadIdx.x) * kScanPer;
  uint32_t s = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t tot;
  block_exclusive_scan(s, sh, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanT) scan_blocks_kernel(uint32_t* bsum, int nb) {
  // single block: exclusive scan of nb block sums in place; bsum[nb] = grand total
  __shared__ uint32_t sh[kScanT];
  const int per = (nb + kScanT - 1) / kScanT;
  const int lo = threadIdx.x * per, hi = min(nb, lo + per);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += bsum[i];
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, sh, tot);
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = bsum[i];
    bsum[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) bsum[nb] = tot;
}

__global__ void __launch_bounds__(kScanT) scan_apply_kernel(const uint32_t* in, int64_t n, const uint32_t* bsum,
                                                            int nb, uint32_t* out) {
  __shared__ uint32_t sh[kScanT];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + static_cast<int64_t>(threadIdx.x) * kScanPer;
  uint32_t v[kScanPer];
  uint32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, sh, tot) + bsum[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

template <typename T, int MODE>
hipError_t dispatch(int p, dim3 grid, const GObjSet<T>& o, const uint32_t* starts, const Geometry& g,
                    const SpecT<T>& f, void* mesh, hipStream_t st) {
  using T2 = typename V2<T>::type;
  const T H = static_cast<T>(g.H), rx = static_cast<T>(g.rel[0]), ry = static_cast<T>(g.rel[1]),
          rz = static_cast<T>(g.rel[2]);
  T2* m = static_cast<T2*>(mesh);
  int lg = 0;
  while ((1 << lg) < g.N) ++lg;
  switch (p) {
    case 1:
      gather_kernel<T, 1, MODE><<<grid, kThreads, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz, f, m);
      break;
    case 2:
      gather_kernel<T, 2, MODE><<<grid, kThreads, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz, f, m);
      break;
    default:
      gather_kernel<T, 3, MODE><<<grid, kThreads, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz, f, m);
      break;
  }
  return hipGetLastError();
}

}  // namespace

int64_t scan_block_count(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

hipError_t launch_cell_count(const RawCat& c, const Geometry& g, uint32_t* counts, uint32_t* rank,
                             uint32_t* cell_of_obj, hipStream_t st) {
  if (c.n == 0) return hipSuccess;
  cell_count_kernel<<<static_cast<unsigned>((c.n + 255) / 256), 256, 0, st>>>(c, g, counts, rank, cell_of_obj);
  return hipGetLastError();
}

hipError_t launch_big_scan(const uint32_t* counts, int64_t n, uint32_t* bsum, uint32_t* starts, hipStream_t st) {
  const int64_t nb = scan_block_count(n);
  scan_reduce_kernel<<<static_cast<unsigned>(nb), kScanT, 0, st>>>(counts, n, bsum);
  scan_blocks_kernel<<<1, kScanT, 0, st>>>(bsum, static_cast<int>(nb));
  scan_apply_kernel<<<static_cast<unsigned>(nb), kScanT, 0, st>>>(counts, n, bsum, static_cast<int>(nb), starts);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cell_scatter(const RawCat& c, const Geometry& g, double wscale, int shape, const uint32_t* starts,
                               const uint32_t* rank, const uint32_t* cell_of_obj, GObjSet<T> out, hipStream_t st) {
  if (c.n == 0) return hipSuccess;
  cell_scatter_kernel<T><<<static_cast<unsigned>((c.n + 255) / 256), 256, 0, st>>>(c, g, wscale, shape, starts, rank,
                                                                                    cell_of_obj, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const GObjSet<T>& o, const uint32_t* cell_start, const Geometry& g, const FieldSpec& f,
                         int mode, void* mesh, hipStream_t st) {
  if (g.N % TT != 0) return hipErrorInvalidValue;
  const int nt = g.N / TT;
  dim3 grid(static_cast<unsigned>(nt) * nt * nt);
  const SpecT<T> sp = to_spec<T>(f);
  switch (mode) {
    case 0:
      return dispatch<T, 0>(g.p, grid, o, cell_start, g, sp, mesh, st);
    case 1:
      return dispatch<T, 1>(g.p, grid, o, cell_start, g, sp, mesh, st);
    default:
      return dispatch<T, 2>(g.p, grid, o, cell_start, g, sp, mesh, st);
  }
}

template hipError_t launch_cell_scatter<float>(const RawCat&, const Geometry&, double, int, const uint32_t*,
                                               const uint32_t*, const uint32_t*, GObjSet<float>, hipStream_t);
template hipError_t launch_cell_scatter<double>(const RawCat&, const Geometry&, double, int, const uint32_t*,
                                                const uint32_t*, const uint32_t*, GObjSet<double>, hipStream_t);
template hipError_t launch_gather<float>(const GObjSet<float>&, const uint32_t*, const Geometry&, const FieldSpec&,
                                         int, void*, hipStream_t);
template hipError_t launch_gather<double>(const GObjSet<double>&, const uint32_t*, const Geometry&,
                                          const FieldSpec&, int, void*, hipStream_t);

}  // namespace lpp
