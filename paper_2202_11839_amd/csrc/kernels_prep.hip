// Catalog preparation: FP64 normalisation sums and input checks, the
// counting sort of objects by mesh tile, and the compact per-object records
// (packed cell, fractional offset, weight) that the deposit kernels read.
#include "lpp_internal.h"

namespace lpp {

namespace {

__device__ __forceinline__ double ld(const void* p, int64_t i, int dtype) {
  return dtype == LPP_F64 ? static_cast<const double*>(p)[i] : static_cast<double>(static_cast<const float*>(p)[i]);
}

constexpr int kSumThreads = 256;
constexpr int kSumBlocks = 1024;
constexpr int kSumWidth = 8;

__global__ void __launch_bounds__(kSumThreads) catalog_sums_kernel(RawCat c, Geometry g, double nbar_default,
                                                                    double* partial) {
  double acc[kSumWidth] = {0, 0, 0, 0, 0, 0, 0, 0};
  const double minr2 = (1e-6 * g.box) * (1e-6 * g.box);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < c.n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double x = ld(c.x, i, c.dtype), y = ld(c.y, i, c.dtype), z = ld(c.z, i, c.dtype);
    const double w = c.w ? ld(c.w, i, c.dtype) : 1.0;
    const double nb = c.nbar ? ld(c.nbar, i, c.dtype) : nbar_default;
    double g2 = 0.0;
    bool finite = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(w) && isfinite(nb);
    if (c.g1) {
      const double a = ld(c.g1, i, c.dtype), b = ld(c.g2, i, c.dtype);
      finite = finite && isfinite(a) && isfinite(b);
      g2 = a * a + b * b;
    }
    if (!finite) {
      acc[4] += 1.0;
      continue;
    }
    const double ux = (x - g.origin[0]) / g.H, uy = (y - g.origin[1]) / g.H, uz = (z - g.origin[2]) / g.H;
    if (!(ux >= 0.0 && ux < g.N && uy >= 0.0 && uy < g.N && uz >= 0.0 && uz < g.N)) acc[5] += 1.0;
    const double rx = x - g.origin[0] + g.rel[0], ry = y - g.origin[1] + g.rel[1], rz = z - g.origin[2] + g.rel[2];
    if (rx * rx + ry * ry + rz * rz < minr2) acc[6] += 1.0;
    acc[0] += w;
    acc[1] += w * w;
    acc[2] += w * w * nb;
    acc[3] += w * w * g2;
  }
  __shared__ double sh[kSumThreads];
  for (int k = 0; k < kSumWidth; ++k) {
    sh[threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kSumThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x * kSumWidth + k] = sh[0];
    __syncthreads();
  }
}

// out[k] = sum over blocks, in block order (deterministic)
__global__ void __launch_bounds__(kSumWidth) sum_partials_kernel(const double* partial, int nblocks, double* out) {
  const int k = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * kSumWidth + k];
  out[k] = s;
}

__device__ __forceinline__ int cell_of(double u, int N) {
  int c = static_cast<int>(floor(u));
  return c < 0 ? 0 : (c >= N ? N - 1 : c);
}

template <typename T>
__global__ void tile_count_kernel(RawCat c, Geometry g, int tshift, uint32_t* counts, uint32_t* rank,
                                  uint32_t* tile_of) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= c.n) return;
  const int N = g.N;
  const int cx = cell_of((ld(c.x, i, c.dtype) - g.origin[0]) / g.H, N);
  const int cy = cell_of((ld(c.y, i, c.dtype) - g.origin[1]) / g.H, N);
  const int cz = cell_of((ld(c.z, i, c.dtype) - g.origin[2]) / g.H, N);
  const int nt = N >> tshift;
  const uint32_t t = static_cast<uint32_t>((cx >> tshift) + nt * ((cy >> tshift) + nt * (cz >> tshift)));
  tile_of[i] = t;
  rank[i] = atomicAdd(&counts[t], 1u);
}

// single-block exclusive scan of n counts into starts[0..n]
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads) scan_kernel(const uint32_t* counts, uint32_t* starts, int n) {
  __shared__ uint32_t sh[kScanThreads];
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int lo = threadIdx.x * per;
  const int hi = min(n, lo + per);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    uint32_t v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = sh[threadIdx.x] - s;  // exclusive prefix of this chunk
  for (int i = lo; i < hi; ++i) {
    starts[i] = run;
    run += counts[i];
  }
  if (threadIdx.x == kScanThreads - 1) starts[n] = sh[kScanThreads - 1];
}

template <typename T>
__global__ void scatter_kernel(RawCat c, Geometry g, double wscale, int shape, const uint32_t* starts,
                               const uint32_t* rank, const uint32_t* tile_of, ObjSet<T> out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= c.n) return;
  const int N = g.N;
  const double ux = (ld(c.x, i, c.dtype) - g.origin[0]) / g.H;
  const double uy = (ld(c.y, i, c.dtype) - g.origin[1]) / g.H;
  const double uz = (ld(c.z, i, c.dtype) - g.origin[2]) / g.H;
  const int cx = cell_of(ux, N), cy = cell_of(uy, N), cz = cell_of(uz, N);
  const int64_t d = static_cast<int64_t>(starts[tile_of[i]]) + rank[i];
  out.key[d] = static_cast<uint32_t>(cx) | (static_cast<uint32_t>(cy) << 10) | (static_cast<uint32_t>(cz) << 20);
  out.fx[d] = static_cast<T>(ux - cx);
  out.fy[d] = static_cast<T>(uy - cy);
  out.fz[d] = static_cast<T>(uz - cz);
  const double w = c.w ? ld(c.w, i, c.dtype) : 1.0;
  if (shape) {
    out.wr[d] = static_cast<T>(w * ld(c.g1, i, c.dtype));
    out.wi[d] = static_cast<T>(w * ld(c.g2, i, c.dtype));
  } else {
    out.wr[d] = static_cast<T>(wscale * w);
  }
}

__global__ void fill_zero_kernel(uint4* p, size_t n16) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n16;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void fill_zero_bytes_kernel(unsigned char* p, size_t n) {
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i < n) p[i] = 0;
}

int log2i(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return s;
}

}  // namespace

int catalog_sum_blocks() { return kSumBlocks; }

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  if (n16) {
    const size_t want = (n16 + 255) / 256;
    const unsigned blocks = static_cast<unsigned>(want < 8192 ? want : 8192);
    fill_zero_kernel<<<blocks, 256, 0, st>>>(static_cast<uint4*>(p), n16);
  }
  const size_t rem = bytes - n16 * 16;
  if (rem) fill_zero_bytes_kernel<<<1, 256, 0, st>>>(static_cast<unsigned char*>(p) + n16 * 16, rem);
  return hipGetLastError();
}

hipError_t launch_catalog_sums(const RawCat& c, const Geometry& g, double nbar_default, double* partial,
                               int nblocks, double* out, hipStream_t st) {
  catalog_sums_kernel<<<nblocks, kSumThreads, 0, st>>>(c, g, nbar_default, partial);
  sum_partials_kernel<<<1, kSumWidth, 0, st>>>(partial, nblocks, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tile_count(const RawCat& c, const Geometry& g, int tile, uint32_t* counts, uint32_t* rank,
                             uint32_t* tile_of, hipStream_t st) {
  if (c.n == 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((c.n + 255) / 256);
  tile_count_kernel<T><<<blocks, 256, 0, st>>>(c, g, log2i(tile), counts, rank, tile_of);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* counts, uint32_t* starts, int n, hipStream_t st) {
  scan_kernel<<<1, kScanThreads, 0, st>>>(counts, starts, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter(const RawCat& c, const Geometry& g, double wscale, int shape, const uint32_t* starts,
                          const uint32_t* rank, const uint32_t* tile_of, ObjSet<T> out, int64_t offset,
                          hipStream_t st) {
  (void)offset;
  if (c.n == 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((c.n + 255) / 256);
  scatter_kernel<T><<<blocks, 256, 0, st>>>(c, g, wscale, shape, starts, rank, tile_of, out);
  return hipGetLastError();
}

template hipError_t launch_tile_count<float>(const RawCat&, const Geometry&, int, uint32_t*, uint32_t*, uint32_t*,
                                             hipStream_t);
template hipError_t launch_tile_count<double>(const RawCat&, const Geometry&, int, uint32_t*, uint32_t*,
                                              uint32_t*, hipStream_t);
template hipError_t launch_scatter<float>(const RawCat&, const Geometry&, double, int, const uint32_t*,
                                          const uint32_t*, const uint32_t*, ObjSet<float>, int64_t, hipStream_t);
template hipError_t launch_scatter<double>(const RawCat&, const Geometry&, double, int, const uint32_t*,
                                           const uint32_t*, const uint32_t*, ObjSet<double>, int64_t, hipStream_t);

}  // namespace lpp
