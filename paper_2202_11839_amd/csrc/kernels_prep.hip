// Catalog preparation: FP64 normalisation sums and input checks, and the
// mesh clearing kernel.
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
    if (!g.global_los && rx * rx + ry * ry + rz * rz < minr2) acc[6] += 1.0;
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
    if (threadIdx.x == 0) partial[k * gridDim.x + blockIdx.x] = sh[0];
    __syncthreads();
  }
}

// out[k] = sum over blocks (partials stored [k][block]); one block per k, fixed-shape tree
__global__ void __launch_bounds__(kSumThreads) sum_partials_kernel(const double* partial, int nblocks, double* out) {
  __shared__ double sh[kSumThreads];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kSumThreads) s += partial[k * nblocks + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kSumThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = sh[0];
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
  sum_partials_kernel<<<kSumWidth, kSumThreads, 0, st>>>(partial, nblocks, out);
  return hipGetLastError();
}

}  // namespace lpp
