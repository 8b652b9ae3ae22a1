// A fully connected emulator network for the window-convolved templates:
// widths w_0 -> w_1 -> ... -> w_L, SiLU between layers, linear output,
// mean-squared-error loss and Adam.  Every matrix product runs on the
// matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation); parameters, gradients and Adam moments are FP32, with a
// BF16 copy of the weights refreshed by every update.  In the forward pass
// each layer input a is carried as two BF16 values, hi = bf16(a) and
// lo = bf16(a - hi), and multiplied by the BF16 weights with two MFMAs
// (hi, then lo, into the same FP32 accumulator): the inputs keep about 16
// significant bits instead of 8, which is what the emulator's output
// precision is limited by.  The backward products use the hi halves.
//
// Layouts: activations row-major [batch][width]; weights W_l [w_{l+1}][w_l]
// (y = x W^T + b).  One 256-thread workgroup computes a 32 x 32 tile of the
// product, each 64-wide wavefront a 16 x 16 block; the K loop steps by 32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "lpp_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct lpp_mlp_s {
  int nl = 0;
  int w[9] = {0};
  int64_t max_batch = 0;
  hipStream_t stream = nullptr;
  int64_t nparam = 0;
  int64_t off_w[8] = {0}, off_b[8] = {0};
  float* P = nullptr;      // FP32 parameters
  uint16_t* Pb = nullptr;  // BF16 copy (weights and biases, same offsets)
  float* G = nullptr;      // gradients
  float* M1 = nullptr;     // Adam first moments
  float* M2 = nullptr;     // Adam second moments
  uint16_t* A[9] = {nullptr};  // BF16 layer inputs [max_batch][w_l], l = 0..nl-1 (hi halves)
  uint16_t* Alo[9] = {nullptr};  // their lo halves (forward only)
  float* Z[8] = {nullptr};     // FP32 pre-activations [max_batch][w_{l+1}]
  float* D[8] = {nullptr};     // FP32 deltas dL/dZ_l
  uint16_t* Db[8] = {nullptr}; // BF16 copies of the deltas
  float* loss = nullptr;       // device scalar
  int* step = nullptr;         // device Adam step counter (and batch counter of fit)
  float* lr = nullptr;         // device learning-rate schedule [steps]
  int64_t lr_cap = 0;
  int* perm = nullptr;         // device permutation of the training rows
  int64_t perm_cap = 0;
  float* Xb = nullptr;         // FP32 batch staging for fit
  float* Tb = nullptr;
  std::vector<void*> allocs;
};

namespace lpp {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
// x = hi + lo to about 16 significant bits (x - hi is exact in FP32)
__device__ __forceinline__ void f2bf_split(float x, uint16_t& hi, uint16_t& lo) {
  hi = f2bf(x);
  lo = f2bf(x - bf2f(hi));
}
__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

enum Epi { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DELTA = 2, EPI_PLAIN = 3 };

struct EpiArgs {
  const float* bias;     // HIDDEN / OUT
  float* zout;           // HIDDEN: pre-activation; OUT: output; DELTA: delta; PLAIN: result
  uint16_t* bout;        // HIDDEN: activation (bf16 hi half); DELTA: delta (bf16)
  uint16_t* blo;         // HIDDEN: activation (bf16 lo half)
  const float* zprev;    // DELTA: pre-activation of the layer the delta belongs to
  int64_t ld;            // row stride of zout / bout / zprev
};

// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak] (+ Alo[m sam + k sak]
// when Alo is not null), B(k, n) = B[k sbk + n sbn]
template <int EPI>
__global__ void __launch_bounds__(kT) gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A,
                                                     const uint16_t* __restrict__ Alo, int64_t sam, int64_t sak,
                                                     const uint16_t* __restrict__ B, int64_t sbk, int64_t sbn,
                                                     EpiArgs e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 32 + (wave >> 1) * 16, n0 = blockIdx.y * 32 + (wave & 1) * 16;
  const int am = m0 + (lane & 15), bn = n0 + (lane & 15), kq = (lane >> 4) * 8;
  f32x4 c = {0.f, 0.f, 0.f, 0.f};
  const bool split = Alo != nullptr;
  // the 8 k-values of a lane are contiguous and 16-byte aligned when the
  // operand runs along k from a 16-byte aligned base with a row stride that
  // is a multiple of 8: one 16-byte load instead of eight
  const auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  const bool avec = sak == 1 && sam % 8 == 0 && al16(A) && (!split || al16(Alo));
  const bool bvec = sbk == 1 && sbn % 8 == 0 && al16(B);
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a, al, b;
    const bool kfull = k0 + kq + 8 <= K;
    if (avec && kfull && am < M) {
      const int64_t o = am * sam + k0 + kq;
      a = *reinterpret_cast<const bf16x8*>(A + o);
      if (split) al = *reinterpret_cast<const bf16x8*>(Alo + o);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + kq + i;
        const bool in = am < M && k < K;
        a[i] = __builtin_bit_cast(__bf16, in ? A[am * sam + k * sak] : static_cast<uint16_t>(0));
        al[i] = __builtin_bit_cast(__bf16, (in && split) ? Alo[am * sam + k * sak] : static_cast<uint16_t>(0));
      }
    }
    if (bvec && kfull && bn < N) {
      b = *reinterpret_cast<const bf16x8*>(B + bn * sbn + k0 + kq);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + kq + i;
        b[i] = __builtin_bit_cast(__bf16, (bn < N && k < K) ? B[k * sbk + bn * sbn] : static_cast<uint16_t>(0));
      }
    }
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    if (split) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, c, 0, 0, 0);
  }
  const int col = n0 + (lane & 15);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = m0 + (lane >> 4) * 4 + i;
    if (row >= M || col >= N) continue;
    const int64_t o = row * e.ld + col;
    float v = c[i];
    if (EPI == EPI_HIDDEN) {
      v += e.bias[col];
      e.zout[o] = v;
      f2bf_split(v * sigm(v), e.bout[o], e.blo[o]);
    } else if (EPI == EPI_OUT) {
      e.zout[o] = v + e.bias[col];
    } else if (EPI == EPI_DELTA) {
      const float z = e.zprev[o], s = sigm(z);
      const float d = v * (s * (1.0f + z * (1.0f - s)));
      e.zout[o] = d;
      e.bout[o] = f2bf(d);
    } else {
      e.zout[o] = v;
    }
  }
}

// rows of X (FP32, [n][w]) -> BF16 hi and lo halves
__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y,
                               uint16_t* __restrict__ ylo) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    f2bf_split(x[i], y[i], ylo[i]);
}

// loss = mean (Y - T)^2, dY = 2 (Y - T) / (B w); one block, FP64 sum in fixed order
constexpr int kMseT = 1024;
__global__ void __launch_bounds__(kMseT) mse_kernel(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                                                  float* __restrict__ dY, uint16_t* __restrict__ dYb,
                                                  float* __restrict__ loss) {
  __shared__ double sh[kMseT];
  double s = 0.0;
  const float scale = 2.0f / static_cast<float>(n);
  for (int64_t i = threadIdx.x; i < n; i += kMseT) {
    const float r = Y[i] - T[i];
    s += static_cast<double>(r) * r;
    const float d = scale * r;
    dY[i] = d;
    dYb[i] = f2bf(d);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kMseT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = static_cast<float>(sh[0] / static_cast<double>(n));
}

// db[o] = sum_b D[b][o]: 64 outputs per workgroup, one per lane; each of the
// kBiasGroups wavefronts sums a run of consecutive rows in row order, then
// lane o of the first wavefront adds the runs' partials in run order (a fixed
// order, independent of timing)
constexpr int kBiasGroups = 8;
__global__ void __launch_bounds__(64 * kBiasGroups)
    bias_grad_kernel(const float* __restrict__ D, int B, int W, float* __restrict__ db) {
  __shared__ float part[kBiasGroups][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + c;
  const int per = (B + kBiasGroups - 1) / kBiasGroups;
  const int b0 = g * per, b1 = min(B, b0 + per);
  float s = 0.f;
  if (o < W) {
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += D[static_cast<int64_t>(b) * W + o];
  }
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && o < W) {
    float t = part[0][c];
    for (int j = 1; j < kBiasGroups; ++j) t += part[j][c];
    db[o] = t;
  }
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on every parameter; the step
// counter t is advanced by the caller's step kernel; lr = lr_sched[t - 1]
__global__ void adam_kernel(float* __restrict__ P, uint16_t* __restrict__ Pb, const float* __restrict__ G,
                            float* __restrict__ M1, float* __restrict__ M2, int64_t n, const int* __restrict__ step,
                            const float* __restrict__ lr_sched, float lr_fixed) {
  const int t = *step;
  const float lr = lr_sched ? lr_sched[t - 1] : lr_fixed;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, static_cast<float>(t)), c2 = 1.0f - powf(b2, static_cast<float>(t));
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float g = G[i];
    const float m = b1 * M1[i] + (1.0f - b1) * g;
    const float v = b2 * M2[i] + (1.0f - b2) * g * g;
    M1[i] = m;
    M2[i] = v;
    const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    P[i] = p;
    Pb[i] = f2bf(p);
  }
}

__global__ void bump_kernel(int* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

// fit: copy the batch rows perm[batch0 + i] of X, T into the staging buffers;
// batch0 = (*step - step_base) * B
__global__ void gather_rows_kernel(const float* __restrict__ X, const float* __restrict__ T, int win, int wout,
                                   const int* __restrict__ perm, const int* __restrict__ step, int step_base, int B,
                                   float* __restrict__ Xb, uint16_t* __restrict__ Ab, uint16_t* __restrict__ Alo,
                                   float* __restrict__ Tb) {
  const int64_t b0 = static_cast<int64_t>(*step - step_base) * B;
  const int64_t nx = static_cast<int64_t>(B) * win, nt = static_cast<int64_t>(B) * wout;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nx + nt;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (i < nx) {
      const int64_t r = i / win, c = i % win;
      const float v = X[static_cast<int64_t>(perm[b0 + r]) * win + c];
      Xb[i] = v;
      f2bf_split(v, Ab[i], Alo[i]);
    } else {
      const int64_t j = i - nx, r = j / wout, c = j % wout;
      Tb[j] = T[static_cast<int64_t>(perm[b0 + r]) * wout + c];
    }
  }
}

int blocks_for(int64_t n) { return static_cast<int>(std::min<int64_t>(4096, (n + kT - 1) / kT)); }

// ---- the emulator's encoding of the template path ----
// inputs: theta_i scaled to [-1, 1] over ranges [lo_i, hi_i];
// outputs: P~_+^(l) / (A^2 sigma8^2) (the shot noise taken out of l = 0) and
// P~_gd^(L) / (A sigma8^2), then standardised per output column.
struct EmuArgs {
  double lo[5], hi[5];
  double shot;  // 2 sigma_gamma^2 / nbar
  int nk;
};

__device__ __forceinline__ double emu_prefactor(const double* p, int o) {
  const double s2 = p[3] * p[3];
  return o < 3 ? p[0] * p[0] * s2 : p[0] * s2;
}

__global__ void emu_inputs_kernel(EmuArgs a, const double* __restrict__ params, int64_t n, float* __restrict__ X) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < 5 * n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(i % 5);
    X[i] = static_cast<float>(2.0 * (params[i] - a.lo[c]) / (a.hi[c] - a.lo[c]) - 1.0);
  }
}

// shape-normalised outputs, FP64 [n][5 nk]; *bad is set when a point's
// prefactor is zero or not finite (its shapes would be inf/NaN and spoil the
// column statistics of every point)
__global__ void emu_shapes_kernel(EmuArgs a, const double* __restrict__ params, const double* __restrict__ templ,
                                  int64_t n, double* __restrict__ shapes, int* __restrict__ bad) {
  const int w = 5 * a.nk;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n * w;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = i / w;
    const int o = static_cast<int>((i % w) / a.nk);
    const double* p = params + 5 * r;
    double v = templ[i];
    if (o == 0) v -= a.shot * p[4];
    const double pf = emu_prefactor(p, o);
    if (!(pf != 0.0) || !isfinite(pf)) {
      *bad = 1;
      shapes[i] = 0.0;
    } else {
      shapes[i] = v / pf;
    }
  }
}

// per column: mean and standard deviation over the rows (FP64, fixed order)
__global__ void __launch_bounds__(kT) column_stats_kernel(const double* __restrict__ x, int64_t n, int w,
                                                        double* __restrict__ mean, double* __restrict__ sd) {
  __shared__ double sh[kT];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kT) s += x[r * w + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double mu = sh[0] / static_cast<double>(n);
  __syncthreads();
  double q = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kT) {
    const double d = x[r * w + c] - mu;
    q += d * d;
  }
  sh[threadIdx.x] = q;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[c] = mu;
    // a column that is constant up to rounding (the plus shapes do not depend
    // on the parameters) keeps sd = 1: its targets are then ~0, not rounding
    // noise blown up to unit variance
    const double v = sh[0] / static_cast<double>(n), floor = 1e-9 * fabs(mu);
    sd[c] = v > floor * floor && v > 0.0 ? sqrt(v) : 1.0;
  }
}

__global__ void standardise_kernel(const double* __restrict__ x, int64_t n, int w, const double* __restrict__ mean,
                                   const double* __restrict__ sd, float* __restrict__ T) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n * w;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(i % w);
    T[i] = static_cast<float>((x[i] - mean[c]) / sd[c]);
  }
}

__global__ void emu_outputs_kernel(EmuArgs a, const double* __restrict__ params, const float* __restrict__ Y,
                                   int64_t n, const double* __restrict__ mean, const double* __restrict__ sd,
                                   double* __restrict__ out) {
  const int w = 5 * a.nk;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n * w;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = i / w;
    const int c = static_cast<int>(i % w), o = c / a.nk;
    const double* p = params + 5 * r;
    double v = (static_cast<double>(Y[i]) * sd[c] + mean[c]) * emu_prefactor(p, o);
    if (o == 0) v += a.shot * p[4];
    out[i] = v;
  }
}

template <int EPI>
hipError_t gemm(hipStream_t st, int M, int N, int K, const uint16_t* A, const uint16_t* Alo, int64_t sam, int64_t sak,
                const uint16_t* B, int64_t sbk, int64_t sbn, const EpiArgs& e) {
  dim3 grid((M + 31) / 32, (N + 31) / 32);
  gemm_bf16_kernel<EPI><<<grid, kT, 0, st>>>(M, N, K, A, Alo, sam, sak, B, sbk, sbn, e);
  return hipGetLastError();
}

// Inference of the whole network in one launch, 16 rows per workgroup (16
// wavefronts, one 16-column output tile each at a time): each
// layer's BF16 hi/lo activations stay in LDS (two buffers, one read while the
// next is written), the weights come from global memory (L2-resident at
// these sizes).  Every output gets the layered path's MFMA sequence (k in
// steps of 32, the hi then the lo product) and epilogue, so the results are
// the same bits as gemm_bf16_kernel's layer by layer; pre-activations of the
// hidden layers are not stored (nothing needs them outside training).
constexpr int kInferRows = 16;
constexpr int kInferMaxW = 256;  // widest layer input the fused path takes
constexpr int kInferLd = kInferMaxW + 8;
constexpr int kInferT = 1024;  // 16 wavefronts: one 16-column tile each for a 256-wide layer

struct InferArgs {
  int nl;
  int w[9];
  const uint16_t* W[8];
  const float* bias[8];
};

// the emulator's encoding of its parameter points and decoding of the
// network's outputs, done inside the fused launch (params null: plain rows
// from A0 / A0lo in, FP32 rows to Y out); the same arithmetic as
// emu_inputs_kernel + to_bf16_kernel and emu_outputs_kernel
struct InferEmu {
  const double* params;  // [M][5]
  EmuArgs a;
  const double* mean;
  const double* sd;
  double* out;  // [M][5 nk]
};

__global__ void __launch_bounds__(kInferT) mlp_infer_kernel(InferArgs g, int M, const uint16_t* __restrict__ A0,
                                                       const uint16_t* __restrict__ A0lo, float* __restrict__ Y,
                                                       InferEmu emu) {
  __shared__ __align__(16) uint16_t act[2][2][kInferRows * kInferLd];  // [buffer][hi, lo][row][k]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.x * kInferRows;
  const int w0 = g.w[0];
  for (int i = threadIdx.x; i < kInferRows * w0; i += blockDim.x) {
    const int r = i / w0, k = i % w0;
    const bool in = r0 + r < M;
    const int64_t o = static_cast<int64_t>(r0 + r) * w0 + k;
    uint16_t h = 0, hl = 0;
    if (in && emu.params) {
      const float x = static_cast<float>(2.0 * (emu.params[o] - emu.a.lo[k]) / (emu.a.hi[k] - emu.a.lo[k]) - 1.0);
      f2bf_split(x, h, hl);
    } else if (in) {
      h = A0[o];
      hl = A0lo[o];
    }
    act[0][0][r * kInferLd + k] = h;
    act[0][1][r * kInferLd + k] = hl;
  }
  __syncthreads();
  const int ar = lane & 15, kq = (lane >> 4) * 8;
  int cur = 0;
  for (int l = 0; l < g.nl; ++l) {
    const int K = g.w[l], N = g.w[l + 1];
    const uint16_t* __restrict__ W = g.W[l];
    const bool last = l + 1 == g.nl;
    const uint16_t* ah = act[cur][0] + ar * kInferLd;
    const uint16_t* alo = act[cur][1] + ar * kInferLd;
    uint16_t* oh = act[cur ^ 1][0];
    uint16_t* olo = act[cur ^ 1][1];
    const bool bvec = K % 8 == 0 && (reinterpret_cast<uintptr_t>(W) & 15) == 0;
    for (int n0 = wave * 16; n0 < N; n0 += 16 * (kInferT / 64)) {
      const int bn = n0 + (lane & 15);
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a, al, b;
        const bool kfull = k0 + kq + 8 <= K;
        if (kfull) {
          a = *reinterpret_cast<const bf16x8*>(ah + k0 + kq);
          al = *reinterpret_cast<const bf16x8*>(alo + k0 + kq);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int k = k0 + kq + i;
            a[i] = __builtin_bit_cast(__bf16, k < K ? ah[k] : static_cast<uint16_t>(0));
            al[i] = __builtin_bit_cast(__bf16, k < K ? alo[k] : static_cast<uint16_t>(0));
          }
        }
        if (bvec && kfull && bn < N) {
          b = *reinterpret_cast<const bf16x8*>(W + static_cast<int64_t>(bn) * K + k0 + kq);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int k = k0 + kq + i;
            b[i] = __builtin_bit_cast(__bf16, (bn < N && k < K) ? W[k + static_cast<int64_t>(bn) * K]
                                                                 : static_cast<uint16_t>(0));
          }
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, c, 0, 0, 0);
      }
      if (bn < N) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = (lane >> 4) * 4 + i;
          const float v = c[i] + g.bias[l][bn];
          if (!last) {
            f2bf_split(v * sigm(v), oh[row * kInferLd + bn], olo[row * kInferLd + bn]);
          } else if (r0 + row < M) {
            const int64_t r = r0 + row;
            if (emu.params) {
              const double* p = emu.params + 5 * r;
              const int o = bn / emu.a.nk;
              double d = (static_cast<double>(v) * emu.sd[bn] + emu.mean[bn]) * emu_prefactor(p, o);
              if (o == 0) d += emu.a.shot * p[4];
              emu.out[r * N + bn] = d;
            } else {
              Y[r * N + bn] = v;
            }
          }
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }
}

bool infer_fits(const lpp_mlp_s* m) {
  if (m->nl < 1 || m->nl > 8) return false;
  for (int l = 0; l < m->nl; ++l)
    if (m->w[l] > kInferMaxW) return false;
  return true;
}

// inference of B rows already in A[0], Alo[0] (BF16 hi/lo) into Y ([B][w_nl]),
// or with emu.params set, of B parameter points into emu.out
hipError_t forward_infer(lpp_mlp_s* m, int B, float* Y, const InferEmu& emu) {
  InferArgs g{};
  g.nl = m->nl;
  for (int l = 0; l <= m->nl; ++l) g.w[l] = m->w[l];
  for (int l = 0; l < m->nl; ++l) {
    g.W[l] = m->Pb + m->off_w[l];
    g.bias[l] = m->P + m->off_b[l];
  }
  mlp_infer_kernel<<<(B + kInferRows - 1) / kInferRows, kInferT, 0, m->stream>>>(g, B, m->A[0], m->Alo[0], Y, emu);
  return hipGetLastError();
}

// forward of B rows already in A[0] (BF16); Y = Z[nl-1]
hipError_t forward(lpp_mlp_s* m, int B, float* Y) {
  hipError_t e = hipSuccess;
  for (int l = 0; l < m->nl && e == hipSuccess; ++l) {
    const int in = m->w[l], out = m->w[l + 1];
    EpiArgs a{};
    a.bias = m->P + m->off_b[l];
    a.ld = out;
    const uint16_t* W = m->Pb + m->off_w[l];
    if (l + 1 < m->nl) {
      a.zout = m->Z[l];
      a.bout = m->A[l + 1];
      a.blo = m->Alo[l + 1];
      e = gemm<EPI_HIDDEN>(m->stream, B, out, in, m->A[l], m->Alo[l], in, 1, W, 1, in, a);
    } else {
      a.zout = Y ? Y : m->Z[l];
      e = gemm<EPI_OUT>(m->stream, B, out, in, m->A[l], m->Alo[l], in, 1, W, 1, in, a);
    }
  }
  return e;
}

// forward, loss, backward and Adam for B rows in A[0] with targets T
hipError_t train_step(lpp_mlp_s* m, int B, const float* T, const float* lr_sched, float lr_fixed) {
  const int L = m->nl;
  hipError_t e = forward(m, B, nullptr);
  const int wout = m->w[L];
  if (e == hipSuccess) {
    mse_kernel<<<1, kMseT, 0, m->stream>>>(m->Z[L - 1], T, static_cast<int64_t>(B) * wout, m->D[L - 1], m->Db[L - 1],
                                        m->loss);
    e = hipGetLastError();
  }
  for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
    const int in = m->w[l], out = m->w[l + 1];
    // dW_l[o][i] = sum_b D_l[b][o] A_l[b][i]
    EpiArgs g{};
    g.zout = m->G + m->off_w[l];
    g.ld = in;
    e = gemm<EPI_PLAIN>(m->stream, out, in, B, m->Db[l], nullptr, 1, out, m->A[l], in, 1, g);
    if (e != hipSuccess) break;
    bias_grad_kernel<<<(out + 63) / 64, 64 * kBiasGroups, 0, m->stream>>>(m->D[l], B, out, m->G + m->off_b[l]);
    e = hipGetLastError();
    if (l > 0 && e == hipSuccess) {
      // D_{l-1}[b][i] = (sum_o D_l[b][o] W_l[o][i]) silu'(Z_{l-1}[b][i])
      EpiArgs d{};
      d.zout = m->D[l - 1];
      d.bout = m->Db[l - 1];
      d.zprev = m->Z[l - 1];
      d.ld = in;
      e = gemm<EPI_DELTA>(m->stream, B, in, out, m->Db[l], nullptr, out, 1, m->Pb + m->off_w[l], in, 1, d);
    }
  }
  if (e == hipSuccess) {
    bump_kernel<<<1, 64, 0, m->stream>>>(m->step);
    adam_kernel<<<blocks_for(m->nparam), kT, 0, m->stream>>>(m->P, m->Pb, m->G, m->M1, m->M2, m->nparam, m->step,
                                                             lr_sched, lr_fixed);
    e = hipGetLastError();
  }
  return e;
}

template <typename T>
bool dalloc(lpp_mlp_s* m, T** p, int64_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
  m->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return true;
}

void free_all(lpp_mlp_s* m) {
  for (void* q : m->allocs) (void)hipFree(q);
  m->allocs.clear();
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

lpp_status status_of(hipError_t e) {
  if (e == hipSuccess) return LPP_OK;
  return e == hipErrorOutOfMemory ? LPP_E_NOMEM : LPP_E_DEVICE;
}

uint16_t host_f2bf(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

}  // namespace
}  // namespace lpp

using namespace lpp;

extern "C" {

lpp_status lpp_mlp_create(const int32_t* widths, int32_t n_layers, int64_t max_batch, uint64_t seed, lpp_mlp* out) {
  if (!widths || !out || n_layers < 1 || n_layers > 8 || max_batch < 1 || max_batch > (int64_t{1} << 24))
    return LPP_E_INVALID;
  for (int i = 0; i <= n_layers; ++i)
    if (widths[i] < 1 || widths[i] > 4096) return LPP_E_INVALID;
  *out = nullptr;
  lpp_mlp_s* m = new (std::nothrow) lpp_mlp_s();
  if (!m) return LPP_E_NOMEM;
  m->nl = n_layers;
  for (int i = 0; i <= n_layers; ++i) m->w[i] = widths[i];
  m->max_batch = max_batch;
  int64_t off = 0;
  for (int l = 0; l < n_layers; ++l) {
    m->off_w[l] = off;
    off += static_cast<int64_t>(widths[l + 1]) * widths[l];
    m->off_b[l] = off;
    off += widths[l + 1];
  }
  m->nparam = off;
  bool ok = dalloc(m, &m->P, off) && dalloc(m, &m->Pb, off) && dalloc(m, &m->G, off) && dalloc(m, &m->M1, off) &&
            dalloc(m, &m->M2, off) && dalloc(m, &m->loss, 1) && dalloc(m, &m->step, 1);
  for (int l = 0; l < n_layers && ok; ++l) {
    ok = dalloc(m, &m->A[l], max_batch * widths[l]) && dalloc(m, &m->Alo[l], max_batch * widths[l]) &&
         dalloc(m, &m->Z[l], max_batch * widths[l + 1]) &&
         dalloc(m, &m->D[l], max_batch * widths[l + 1]) && dalloc(m, &m->Db[l], max_batch * widths[l + 1]);
  }
  ok = ok && dalloc(m, &m->Xb, max_batch * widths[0]) && dalloc(m, &m->Tb, max_batch * widths[n_layers]);
  if (!ok) {
    free_all(m);
    delete m;
    return LPP_E_NOMEM;
  }
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases from a splitmix64 stream
  std::vector<float> h(off);
  uint64_t s = seed;
  for (int l = 0; l < n_layers; ++l) {
    const float a = 1.0f / std::sqrt(static_cast<float>(widths[l]));
    for (int64_t i = m->off_w[l]; i < m->off_b[l] + widths[l + 1]; ++i)
      h[i] = a * (2.0f * static_cast<float>((splitmix(s) >> 40) * (1.0 / 16777216.0)) - 1.0f);
  }
  std::vector<uint16_t> hb(off);
  for (int64_t i = 0; i < off; ++i) hb[i] = host_f2bf(h[i]);
  const int zero = 0;
  if (hipMemcpy(m->P, h.data(), 4 * off, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->Pb, hb.data(), 2 * off, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->M1, 0, 4 * off) != hipSuccess || hipMemset(m->M2, 0, 4 * off) != hipSuccess ||
      hipMemset(m->G, 0, 4 * off) != hipSuccess ||
      hipMemcpy(m->step, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) {
    free_all(m);
    delete m;
    return LPP_E_DEVICE;
  }
  *out = m;
  return LPP_OK;
}

lpp_status lpp_mlp_destroy(lpp_mlp m) {
  if (!m) return LPP_E_INVALID;
  free_all(m);
  delete m;
  return LPP_OK;
}

lpp_status lpp_mlp_set_stream(lpp_mlp m, void* stream) {
  if (!m) return LPP_E_INVALID;
  m->stream = static_cast<hipStream_t>(stream);
  return LPP_OK;
}

lpp_status lpp_mlp_num_params(lpp_mlp m, int64_t* n) {
  if (!m || !n) return LPP_E_INVALID;
  *n = m->nparam;
  return LPP_OK;
}

lpp_status lpp_mlp_get_params(lpp_mlp m, float* host, float* grads_host) {
  if (!m || (!host && !grads_host)) return LPP_E_INVALID;
  if (hipStreamSynchronize(m->stream) != hipSuccess) return LPP_E_DEVICE;
  if (host && hipMemcpy(host, m->P, 4 * m->nparam, hipMemcpyDeviceToHost) != hipSuccess) return LPP_E_DEVICE;
  if (grads_host && hipMemcpy(grads_host, m->G, 4 * m->nparam, hipMemcpyDeviceToHost) != hipSuccess)
    return LPP_E_DEVICE;
  return LPP_OK;
}

lpp_status lpp_mlp_set_params(lpp_mlp m, const float* host) {
  if (!m || !host) return LPP_E_INVALID;
  std::vector<uint16_t> hb(m->nparam);
  for (int64_t i = 0; i < m->nparam; ++i) hb[i] = host_f2bf(host[i]);
  if (hipStreamSynchronize(m->stream) != hipSuccess ||
      hipMemcpy(m->P, host, 4 * m->nparam, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->Pb, hb.data(), 2 * m->nparam, hipMemcpyHostToDevice) != hipSuccess)
    return LPP_E_DEVICE;
  return LPP_OK;
}

lpp_status lpp_mlp_forward(lpp_mlp m, const float* X, int64_t B, float* Y) {
  if (!m || !X || !Y || B < 0 || B > m->max_batch) return LPP_E_INVALID;
  if (B == 0) return LPP_OK;
  const int64_t n = B * m->w[0];
  to_bf16_kernel<<<blocks_for(n), kT, 0, m->stream>>>(X, n, m->A[0], m->Alo[0]);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = forward(m, static_cast<int>(B), Y);
  return status_of(e);
}

lpp_status lpp_mlp_train_step(lpp_mlp m, const float* X, const float* T, int64_t B, float lr, float* loss_host) {
  if (!m || !X || !T || B < 1 || B > m->max_batch || !(lr >= 0.0f)) return LPP_E_INVALID;
  const int64_t n = B * m->w[0];
  to_bf16_kernel<<<blocks_for(n), kT, 0, m->stream>>>(X, n, m->A[0], m->Alo[0]);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = train_step(m, static_cast<int>(B), T, nullptr, lr);
  if (e == hipSuccess && loss_host) {
    e = hipMemcpyAsync(loss_host, m->loss, 4, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  }
  return status_of(e);
}

lpp_status lpp_emulator_encode(const double* params, const double* templ, int64_t n, int32_t n_k,
                               const double* ranges, double nbar, double sigma_gamma, float* X, float* T,
                               double* mean, double* sd, void* stream) {
  if (!params || !templ || !ranges || !X || !T || !mean || !sd || n < 1 || n_k < 1 || !(nbar > 0.0)) return LPP_E_INVALID;
  EmuArgs a{};
  for (int i = 0; i < 5; ++i) {
    a.lo[i] = ranges[2 * i];
    a.hi[i] = ranges[2 * i + 1];
    if (!(a.hi[i] > a.lo[i])) return LPP_E_INVALID;
  }
  a.shot = 2.0 * sigma_gamma * sigma_gamma / nbar;
  a.nk = n_k;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int w = 5 * n_k;
  double* shapes = nullptr;
  // the shapes, then one flag word
  if (hipMalloc(&shapes, 8 * (static_cast<size_t>(n) * w + 1)) != hipSuccess) return LPP_E_NOMEM;
  int* bad = reinterpret_cast<int*>(shapes + static_cast<size_t>(n) * w);
  int bad_host = 0;
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), st);
  if (e == hipSuccess) {
    emu_shapes_kernel<<<blocks_for(n * w), kT, 0, st>>>(a, params, templ, n, shapes, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && bad_host) {
    // A = 0 or sigma8 = 0 (or a non-finite value) in a training point: nothing is written
    (void)hipFree(shapes);
    return LPP_E_INVALID;
  }
  if (e == hipSuccess) {
    emu_inputs_kernel<<<blocks_for(5 * n), kT, 0, st>>>(a, params, n, X);
    column_stats_kernel<<<w, kT, 0, st>>>(shapes, n, w, mean, sd);
    standardise_kernel<<<blocks_for(n * w), kT, 0, st>>>(shapes, n, w, mean, sd, T);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(shapes);
  return status_of(e);
}

lpp_status lpp_emulator_predict(lpp_mlp m, const double* params, int64_t n, int32_t n_k, const double* ranges,
                                double nbar, double sigma_gamma, const double* mean, const double* sd, double* out) {
  if (!m || !params || !ranges || !mean || !sd || !out || n < 0 || n_k < 1 || !(nbar > 0.0) ||
      m->w[0] != 5 || m->w[m->nl] != 5 * n_k)
    return LPP_E_INVALID;
  EmuArgs a{};
  for (int i = 0; i < 5; ++i) {
    a.lo[i] = ranges[2 * i];
    a.hi[i] = ranges[2 * i + 1];
    if (!(a.hi[i] > a.lo[i])) return LPP_E_INVALID;
  }
  a.shot = 2.0 * sigma_gamma * sigma_gamma / nbar;
  a.nk = n_k;
  hipError_t e = hipSuccess;
  const bool fused = infer_fits(m);
  for (int64_t r0 = 0; r0 < n && e == hipSuccess; r0 += m->max_batch) {
    const int64_t B = std::min<int64_t>(m->max_batch, n - r0);
    if (fused) {
      const InferEmu ie{params + 5 * r0, a, mean, sd, out + r0 * 5 * n_k};
      e = forward_infer(m, static_cast<int>(B), nullptr, ie);
      continue;
    }
    emu_inputs_kernel<<<blocks_for(5 * B), kT, 0, m->stream>>>(a, params + 5 * r0, B, m->Xb);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    to_bf16_kernel<<<blocks_for(5 * B), kT, 0, m->stream>>>(m->Xb, 5 * B, m->A[0], m->Alo[0]);
    e = forward(m, static_cast<int>(B), nullptr);
    if (e != hipSuccess) break;
    emu_outputs_kernel<<<blocks_for(B * 5 * n_k), kT, 0, m->stream>>>(a, params + 5 * r0, m->Z[m->nl - 1], B, mean,
                                                                       sd, out + r0 * 5 * n_k);
    e = hipGetLastError();
  }
  return status_of(e);
}

lpp_status lpp_mlp_fit(lpp_mlp m, const float* X, const float* T, int64_t n, int32_t batch, int32_t epochs,
                       float lr0, float lr1, uint64_t seed, float* final_loss) {
  if (!m || !X || !T || n < 1 || batch < 1 || batch > m->max_batch || batch > n || epochs < 1 || !(lr0 > 0.0f) ||
      !(lr1 >= 0.0f))
    return LPP_E_INVALID;
  const int64_t spe = n / batch;  // steps per epoch (the last partial batch is dropped)
  const int64_t steps = spe * epochs;
  if (m->perm_cap < n) {
    if (!dalloc(m, &m->perm, n)) return LPP_E_NOMEM;
    m->perm_cap = n;
  }
  int t0 = 0;
  if (hipMemcpy(&t0, m->step, sizeof t0, hipMemcpyDeviceToHost) != hipSuccess) return LPP_E_DEVICE;
  if (m->lr_cap < t0 + steps) {
    if (!dalloc(m, &m->lr, t0 + steps)) return LPP_E_NOMEM;
    m->lr_cap = t0 + steps;
  }
  // cosine schedule lr0 -> lr1 over this fit, indexed by the global Adam step
  std::vector<float> sched(t0 + steps, lr0);
  for (int64_t s = 0; s < steps; ++s)
    sched[t0 + s] = lr1 + 0.5f * (lr0 - lr1) * (1.0f + std::cos(static_cast<float>(M_PI) * s / steps));
  if (hipMemcpy(m->lr, sched.data(), 4 * sched.size(), hipMemcpyHostToDevice) != hipSuccess) return LPP_E_DEVICE;
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return LPP_E_DEVICE;
  hipStream_t user = m->stream;
  std::vector<int> perm(n);
  uint64_t s = seed;
  hipGraphExec_t ge = nullptr;
  hipGraph_t g = nullptr;
  lpp_status result = LPP_OK;
  for (int ep = 0; ep < epochs && result == LPP_OK; ++ep) {
    for (int64_t i = 0; i < n; ++i) perm[i] = static_cast<int>(i);
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix(s) % (i + 1)]);
    if (hipMemcpy(m->perm, perm.data(), 4 * n, hipMemcpyHostToDevice) != hipSuccess) {
      result = LPP_E_DEVICE;
      break;
    }
    const int base = t0 + static_cast<int>(ep * spe);
    // one graph per epoch: the step base differs; each replay is one step
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    ge = nullptr;
    g = nullptr;
    m->stream = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      gather_rows_kernel<<<blocks_for(static_cast<int64_t>(batch) * (m->w[0] + m->w[m->nl])), kT, 0, cap>>>(
          X, T, m->w[0], m->w[m->nl], m->perm, m->step, base, batch, m->Xb, m->A[0], m->Alo[0], m->Tb);
      e = hipGetLastError();
      if (e == hipSuccess) e = train_step(m, batch, m->Tb, m->lr, 0.0f);
      const hipError_t e2 = hipStreamEndCapture(cap, &g);
      if (e == hipSuccess) e = e2;
    }
    m->stream = user;
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    for (int64_t k = 0; k < spe && e == hipSuccess; ++k) e = hipGraphLaunch(ge, user);
    if (e != hipSuccess) result = status_of(e);
  }
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  if (result == LPP_OK && final_loss) {
    if (hipMemcpyAsync(final_loss, m->loss, 4, hipMemcpyDeviceToHost, user) != hipSuccess) result = LPP_E_DEVICE;
  }
  if (hipStreamSynchronize(user) != hipSuccess && result == LPP_OK) result = LPP_E_DEVICE;
  (void)hipStreamDestroy(cap);
  return result;
}

}  // extern "C"
