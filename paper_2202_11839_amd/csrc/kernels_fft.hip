// Forward 3D complex DFT of an N^3 mesh (index x + N*(y + N*z)), computed
// as three batched 1D Stockham passes, one per axis.
//
// Each 1D line of length N is transformed by N/8 threads holding 8 values
// each: radix-8 passes (and one final radix-2 or radix-4 pass when N is not a
// power of 8) with the autosort (Stockham) index map, so no bit reversal is
// needed.  The first pass reads straight from HBM and the last writes
// straight to HBM; the intermediate passes exchange through LDS.  For the x
// axis the lanes of a wavefront run along a line (unit stride, coalesced);
// for the strided y and z axes a workgroup owns NCOL adjacent x-columns and
// the lanes run across the columns, so every HBM access is a contiguous
// NCOL-element row segment (LDS-staged transpose).
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

template <typename T2>
__device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T2>
__device__ __forceinline__ T2 cadd(T2 a, T2 b) {
  return T2{a.x + b.x, a.y + b.y};
}
template <typename T2>
__device__ __forceinline__ T2 csub(T2 a, T2 b) {
  return T2{a.x - b.x, a.y - b.y};
}
// multiply by -i
template <typename T2>
__device__ __forceinline__ T2 cmi(T2 a) {
  return T2{a.y, -a.x};
}

template <typename T2>
__device__ __forceinline__ void dft2(T2& a, T2& b) {
  const T2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// forward 4-point DFT of (a0, a1, a2, a3) in place
template <typename T2>
__device__ __forceinline__ void dft4(T2& a0, T2& a1, T2& a2, T2& a3) {
  const T2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const T2 s13 = cadd(a1, a3), d13 = cmi(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

// forward 8-point DFT, v[k] <- sum_j v[j] exp(-2 pi i jk/8)
template <typename T, typename T2>
__device__ __forceinline__ void dft8(T2* v) {
  T2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  T2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const T r = static_cast<T>(0.70710678118654752440);
  // o_k *= w^k, w = exp(-i pi/4)
  o1 = T2{r * (o1.x + o1.y), r * (o1.y - o1.x)};
  o2 = cmi(o2);
  o3 = T2{r * (o3.y - o3.x), -r * (o3.x + o3.y)};
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

constexpr int n_radix8(int N) {
  int a = 0;
  while (N % 8 == 0 && N > 1) {
    N /= 8;
    ++a;
  }
  return a;
}
constexpr int tail_radix(int N) {
  while (N % 8 == 0 && N > 1) N /= 8;
  return N;  // 1, 2 or 4
}

template <int N, int NCOL>
__device__ __forceinline__ int sidx(int col, int row) {
  return col * N + (row ^ (col & 15));
}

template <typename T, int N, int NCOL, bool ALONG>
__global__ void __launch_bounds__(NCOL* N / 8) fft_axis_kernel(typename V2<T>::type* __restrict__ data, int axis,
                                                              const typename V2<T>::type* __restrict__ tw) {
  using T2 = typename V2<T>::type;
  constexpr int TL = N / 8;
  constexpr int A8 = n_radix8(N);
  constexpr int TR = tail_radix(N);
  __shared__ T2 sm[NCOL * N];

  const int tid = threadIdx.x;
  int col, t;
  if (ALONG) {
    t = tid % TL;
    col = tid / TL;
  } else {
    col = tid % NCOL;
    t = tid / NCOL;
  }
  int64_t base, stride;
  if (axis == 0) {
    base = (static_cast<int64_t>(blockIdx.x) * NCOL + col) * N;
    stride = 1;
  } else {
    constexpr int nchunk = N / NCOL;
    const int chunk = blockIdx.x % nchunk;
    const int other = blockIdx.x / nchunk;
    const int x = chunk * NCOL + col;
    if (axis == 1) {
      base = x + static_cast<int64_t>(N) * N * other;
      stride = N;
    } else {
      base = x + static_cast<int64_t>(N) * other;
      stride = static_cast<int64_t>(N) * N;
    }
  }

  T2 v[8];
  // pass 0: radix 8, Ns = 1, input from HBM
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = data[base + static_cast<int64_t>(t + j * TL) * stride];
  dft8<T>(v);
  constexpr bool single = (A8 == 1 && TR == 1);
  if (single) {  // N == 8 (not used: N >= 16)
#pragma unroll
    for (int j = 0; j < 8; ++j) data[base + static_cast<int64_t>(t + j * TL) * stride] = v[j];
    return;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) sm[sidx<N, NCOL>(col, t * 8 + j)] = v[j];
  __syncthreads();

  int Ns = 8;
  // middle radix-8 passes (LDS -> LDS); the last radix-8 pass writes HBM if there is no tail
#pragma unroll
  for (int p = 1; p < A8; ++p) {
    const bool last = (p == A8 - 1) && (TR == 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = sm[sidx<N, NCOL>(col, t + j * TL)];
    const int k = t % Ns;
    const int step = N / (Ns * 8);
#pragma unroll
    for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], tw[(j * k * step) & (N - 1)]);
    dft8<T>(v);
    if (last) {
      // output index (t/Ns)*Ns*8 + k + j*Ns with Ns = N/8 > t: t + j*TL
#pragma unroll
      for (int j = 0; j < 8; ++j) data[base + static_cast<int64_t>(t + j * TL) * stride] = v[j];
      return;
    }
    __syncthreads();
    const int o = (t / Ns) * Ns * 8 + k;
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[sidx<N, NCOL>(col, o + j * Ns)] = v[j];
    __syncthreads();
    Ns *= 8;
  }
  // tail pass: radix TR in {2, 4}, Ns = N/TR, 8/TR butterflies per thread, output to HBM
  if (TR == 4) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int b = t + q * TL;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[q * 4 + j] = sm[sidx<N, NCOL>(col, b + j * (N / 4))];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int b = t + q * TL;  // k = b since Ns = N/4 > b
#pragma unroll
      for (int j = 1; j < 4; ++j) v[q * 4 + j] = cmul(v[q * 4 + j], tw[(j * b) & (N - 1)]);
      dft4(v[q * 4 + 0], v[q * 4 + 1], v[q * 4 + 2], v[q * 4 + 3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) data[base + static_cast<int64_t>(b + j * (N / 4)) * stride] = v[q * 4 + j];
    }
  } else if (TR == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = t + q * TL;
      v[q * 2 + 0] = sm[sidx<N, NCOL>(col, b)];
      v[q * 2 + 1] = sm[sidx<N, NCOL>(col, b + N / 2)];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = t + q * TL;
      v[q * 2 + 1] = cmul(v[q * 2 + 1], tw[b & (N - 1)]);
      dft2(v[q * 2 + 0], v[q * 2 + 1]);
      data[base + static_cast<int64_t>(b) * stride] = v[q * 2 + 0];
      data[base + static_cast<int64_t>(b + N / 2) * stride] = v[q * 2 + 1];
    }
  }
}

template <typename T, int N>
hipError_t fft_axis_n(void* mesh, const void* tw, int axis, hipStream_t st) {
  using T2 = typename V2<T>::type;
  constexpr int TL = N / 8;
  constexpr int NX = (256 / TL) > 0 ? (256 / TL) : 1;
  constexpr int LDSX = (sizeof(T) == 4 ? 8192 : 4096) / N;
  constexpr int NY = LDSX < N ? LDSX : N;
  T2* d = static_cast<T2*>(mesh);
  const T2* w = static_cast<const T2*>(tw);
  if (axis == 0) {
    const unsigned bx = static_cast<unsigned>(static_cast<int64_t>(N) * N / NX);
    fft_axis_kernel<T, N, NX, true><<<bx, NX * TL, 0, st>>>(d, 0, w);
  } else {
    const unsigned by = static_cast<unsigned>(static_cast<int64_t>(N / NY) * N);
    fft_axis_kernel<T, N, NY, false><<<by, NY * TL, 0, st>>>(d, axis, w);
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_fft_axis(void* mesh, int N, const void* tw, int axis, hipStream_t st) {
  switch (N) {
    case 16:
      return fft_axis_n<T, 16>(mesh, tw, axis, st);
    case 32:
      return fft_axis_n<T, 32>(mesh, tw, axis, st);
    case 64:
      return fft_axis_n<T, 64>(mesh, tw, axis, st);
    case 128:
      return fft_axis_n<T, 128>(mesh, tw, axis, st);
    case 256:
      return fft_axis_n<T, 256>(mesh, tw, axis, st);
    case 512:
      return fft_axis_n<T, 512>(mesh, tw, axis, st);
    case 1024:
      return fft_axis_n<T, 1024>(mesh, tw, axis, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_fft3d(void* mesh, int N, const void* tw, hipStream_t st) {
  for (int axis = 0; axis < 3; ++axis) {
    const hipError_t e = launch_fft_axis<T>(mesh, N, tw, axis, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_fft3d<float>(void*, int, const void*, hipStream_t);
template hipError_t launch_fft_axis<float>(void*, int, const void*, int, hipStream_t);
template hipError_t launch_fft_axis<double>(void*, int, const void*, int, hipStream_t);
template hipError_t launch_fft3d<double>(void*, int, const void*, hipStream_t);

}  // namespace lpp
