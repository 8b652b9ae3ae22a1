// Device helpers shared by the FFT and binning kernels: complex arithmetic,
// the Stockham line transform of one block of columns, the real harmonic
// weights of khat and the k-shell index.
#pragma once

#include "lpp_internal.h"

namespace lpp {
namespace dev {

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
__device__ __forceinline__ T2 cmulc(T2 a, T2 b) {  // a * conj(b)
  return T2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T2>
__device__ __forceinline__ T2 cadd(T2 a, T2 b) {
  return T2{a.x + b.x, a.y + b.y};
}
template <typename T2>
__device__ __forceinline__ T2 csub(T2 a, T2 b) {
  return T2{a.x - b.x, a.y - b.y};
}
template <typename T2>
__device__ __forceinline__ T2 cmi(T2 a) {  // multiply by -i
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
  o1 = T2{r * (o1.x + o1.y), r * (o1.y - o1.x)};   // * exp(-i pi/4)
  o2 = cmi(o2);                                     // * exp(-i pi/2)
  o3 = T2{r * (o3.y - o3.x), -r * (o3.x + o3.y)};  // * exp(-3 i pi/4)
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

// Streaming (non-temporal) access to one complex value: for data that a pass
// reads or writes once, so that it does not displace reused lines in the
// caches (the 3D transform's passes run about 10 % faster with it).
template <typename T2>
__device__ __forceinline__ T2 nt_load(const T2* p) {
  if constexpr (sizeof(T2) == 8) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return T2{v.x, v.y};
  } else {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return T2{v.x, v.y};
  }
}
template <typename T2>
__device__ __forceinline__ void nt_store(T2* p, T2 a) {
  if constexpr (sizeof(T2) == 8) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    v2 w;
    w.x = a.x;
    w.y = a.y;
    __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
  } else {
    typedef double v2 __attribute__((ext_vector_type(2)));
    v2 w;
    w.x = a.x;
    w.y = a.y;
    __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
  }
}

// LDS slot of row `row` of column `col`: the row is XOR-ed with a per-column
// value swz (< N) so that the lanes of one access fall into different banks.
// col & 15 suits lanes that run across the columns; a workgroup whose lanes
// run along 8 rows of 8 columns at a time takes (col & 7) * 9.
template <int N>
__device__ __forceinline__ int sidx(int col, int row, int swz) {
  return col * N + (row ^ swz);
}
template <int N>
__device__ __forceinline__ int swizzle_rows8(int col) {
  return N >= 64 ? (col & 7) * 9 : (col & 15);
}

// Output rows of the column transform below, per thread t (the Stockham
// index map of the last pass): v[q] of fft_column_regs ends at row[q].
template <int N>
__device__ __forceinline__ void fft_rows(int t, int* row) {
  constexpr int TL = N / 8;
  constexpr int TR = tail_radix(N);
  if (TR == 1) {
#pragma unroll
    for (int j = 0; j < 8; ++j) row[j] = t + j * TL;
  } else if (TR == 4) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) row[q * 4 + j] = t + q * TL + j * (N / 4);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      row[q * 2 + 0] = t + q * TL;
      row[q * 2 + 1] = t + q * TL + N / 2;
    }
  }
}

// Forward DFT of length N of the columns of one block, N/8 threads per
// column: on entry v[j] holds element t + j*N/8 of the column, on
// return v[q] is output row fft_rows(t)[q] of column col.  sm (NCOL*N values)
// is free again on return.  Every thread of the block must call it.  swz: the
// LDS row swizzle of the column (sidx), -1 for col & 15.
template <typename T, int N>
__device__ __forceinline__ void fft_column_regs(const typename V2<T>::type* __restrict__ tw,
                                                typename V2<T>::type* sm, int col, int t, typename V2<T>::type* v,
                                                int swz = -1) {
  constexpr int TL = N / 8;
  constexpr int A8 = n_radix8(N);
  constexpr int TR = tail_radix(N);
  static_assert(A8 >= 1 && (A8 > 1 || TR > 1), "N >= 16");
  const int sw = swz >= 0 ? swz : (col & 15);
  // pass 0: radix 8, Ns = 1
  dft8<T>(v);
#pragma unroll
  for (int j = 0; j < 8; ++j) sm[sidx<N>(col, t * 8 + j, sw)] = v[j];
  __syncthreads();
  int Ns = 8;
#pragma unroll
  for (int p = 1; p < A8; ++p) {
    const bool last = (p == A8 - 1) && (TR == 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = sm[sidx<N>(col, t + j * TL, sw)];
    const int k = t % Ns;
    const int step = N / (Ns * 8);
#pragma unroll
    for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], tw[(j * k * step) & (N - 1)]);
    dft8<T>(v);
    __syncthreads();
    if (last) return;  // outputs at t + j*TL
    const int o = (t / Ns) * Ns * 8 + k;
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[sidx<N>(col, o + j * Ns, sw)] = v[j];
    __syncthreads();
    Ns *= 8;
  }
  // tail pass: radix TR in {2, 4}, Ns = N/TR, 8/TR butterflies per thread
  if (TR == 4) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int b = t + q * TL;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[q * 4 + j] = sm[sidx<N>(col, b + j * (N / 4), sw)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int b = t + q * TL;  // k = b since Ns = N/4 > b
#pragma unroll
      for (int j = 1; j < 4; ++j) v[q * 4 + j] = cmul(v[q * 4 + j], tw[(j * b) & (N - 1)]);
      dft4(v[q * 4 + 0], v[q * 4 + 1], v[q * 4 + 2], v[q * 4 + 3]);
    }
  } else if (TR == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = t + q * TL;
      v[q * 2 + 0] = sm[sidx<N>(col, b, sw)];
      v[q * 2 + 1] = sm[sidx<N>(col, b + N / 2, sw)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = t + q * TL;
      v[q * 2 + 1] = cmul(v[q * 2 + 1], tw[b & (N - 1)]);
      dft2(v[q * 2 + 0], v[q * 2 + 1]);
    }
  }
}

// ---- k-space weights and shells ----

template <typename T>
struct KSpec {  // h_{L,M,cs}(khat) = Q_{LM}(khat_z) Re|Im (khat_x + i khat_y)^M
  int M, cs, nq;
  T q[9];
};

template <typename T>
KSpec<T> kspec_of(const FieldSpec& f) {
  KSpec<T> k{};
  k.M = f.M;
  k.cs = f.cs;
  k.nq = f.nq[0];
  for (int i = 0; i < 9; ++i) k.q[i] = static_cast<T>(f.q[0][i]);
  return k;
}

template <typename T>
__device__ __forceinline__ T harmonic(const KSpec<T>& h, T kx, T ky, T kz) {
  T Q = 0;
  for (int i = h.nq - 1; i >= 0; --i) Q = Q * kz + h.q[i];
  T er = 1, ei = 0;
  for (int m = 0; m < h.M; ++m) {
    const T t = er * kx - ei * ky;
    ei = er * ky + ei * kx;
    er = t;
  }
  return Q * (h.cs ? ei : er);
}

__device__ __forceinline__ int sgn_mode(int i, int N) { return i < N / 2 ? i : i - N; }

// Shell of |n|^2 = q, or -1 (DC or beyond the last edge).  thr: thresholds T_0..T_nb.
__device__ __forceinline__ int shell_of(int q, const int* thr, int nb, float inv_dn) {
  if (q <= 0 || q >= thr[nb]) return -1;
  int b = static_cast<int>(sqrtf(static_cast<float>(q)) * inv_dn);
  b = b < 0 ? 0 : (b >= nb ? nb - 1 : b);
  while (b + 1 < nb && thr[b + 1] <= q) ++b;
  while (b > 0 && thr[b] > q) --b;
  return b;
}

// combined, compensated transform from the two interlaced copies; ph is
// exp(-i k.s) of the mode (unused without interlacing)
template <typename T, typename T2>
__device__ __forceinline__ T2 combine(T2 f1, T2 f2, int interlace, T2 ph, T invw) {
  if (interlace) {
    const T2 s = cmul(ph, f2);
    return T2{static_cast<T>(0.5) * (f1.x + s.x) * invw, static_cast<T>(0.5) * (f1.y + s.y) * invw};
  }
  return T2{f1.x * invw, f1.y * invw};
}

}  // namespace dev
}  // namespace lpp
