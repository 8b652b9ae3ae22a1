// Mass assignment of line-of-sight-weighted fields onto the mesh.
//
// Objects arrive sorted by tile (TT^3 cells).  One workgroup owns one tile:
// it accumulates its objects' NGP/CIC/TSC stencils into an LDS copy of the
// tile plus a halo ((TT+3)^3 nodes cover every stencil node of the grid and
// of the interlaced grid shifted by H/2), then adds the non-zero LDS nodes to
// the HBM mesh with one coalesced pass of atomic adds (the halo overlaps the
// neighbouring tiles, so every node receives contributions from at most 8
// workgroups).  The mesh must be zero on entry.
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

// Per-axis stencil: nodes (relative to the object's cell) and weights.
// shifted = 0: grid nodes at integer u; shifted = 1: grid nodes at u = c + 1/2.
template <typename T, int P>
__device__ __forceinline__ void stencil(T f, int shifted, int* node, T* w) {
  const T half = static_cast<T>(0.5);
  if (P == 1) {
    node[0] = shifted ? 0 : (f >= half ? 1 : 0);
    w[0] = 1;
  } else if (P == 2) {
    if (!shifted) {
      node[0] = 0;
      node[1] = 1;
      w[0] = 1 - f;
      w[1] = f;
    } else {
      const int up = f >= half;
      const T fr = up ? f - half : f + half;
      node[0] = up ? 0 : -1;
      node[1] = node[0] + 1;
      w[0] = 1 - fr;
      w[1] = fr;
    }
  } else {
    int c0;
    T d;
    if (!shifted) {
      c0 = f >= half ? 1 : 0;
      d = f - static_cast<T>(c0);
    } else {
      c0 = 0;
      d = f - half;
    }
    node[0] = c0 - 1;
    node[1] = c0;
    node[2] = c0 + 1;
    w[0] = half * (half - d) * (half - d);
    w[1] = static_cast<T>(0.75) - d * d;
    w[2] = half * (half + d) * (half + d);
  }
}

template <typename T>
__device__ __forceinline__ void gadd(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

template <typename T, int TT, int P, int MODE>
__global__ void __launch_bounds__(256) deposit_kernel(ObjSet<T> o, const uint32_t* __restrict__ starts, int N,
                                                      int interlace, T H, T relx, T rely, T relz, SpecT<T> f,
                                                      typename V2<T>::type* __restrict__ mesh) {
  using T2 = typename V2<T>::type;
  constexpr int E = TT + 3;
  constexpr int E3 = E * E * E;
  __shared__ T2 tile[E3];
  const int nt = N / TT;
  const int tid = blockIdx.x;
  const uint32_t beg = starts[tid], end = starts[tid + 1];
  if (beg == end) return;
  const int tx = tid % nt, ty = (tid / nt) % nt, tz = tid / (nt * nt);
  const int t0x = tx * TT, t0y = ty * TT, t0z = tz * TT;
  for (int i = threadIdx.x; i < E3; i += blockDim.x) tile[i] = T2{0, 0};
  __syncthreads();

  const bool shape = (MODE != 0);
  for (uint32_t k = beg + threadIdx.x; k < end; k += blockDim.x) {
    const uint32_t key = o.key[k];
    const int cx = key & 1023u, cy = (key >> 10) & 1023u, cz = (key >> 20) & 1023u;
    const T fx = o.fx[k], fy = o.fy[k], fz = o.fz[k];
    // line of sight of the object
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
    T vr, vi;
    if (shape) {
      const T ar = o.wr[k], ai = o.wi[k];
      vr = ar * gr - ai * gi;
      vi = ar * gi + ai * gr;
    } else {
      vr = o.wr[k] * gr;
      vi = 0;
    }
    const int lx = cx - t0x + 1, ly = cy - t0y + 1, lz = cz - t0z + 1;
    for (int copy = 0; copy < 2; ++copy) {
      int shifted;
      if (MODE == 0) {
        if (copy == 1 && !interlace) break;
        shifted = copy;
      } else {
        if (copy == 1) break;
        shifted = (MODE == 2);
      }
      int nx[3], ny[3], nz[3];
      T wx[3], wy[3], wz[3];
      stencil<T, P>(fx, shifted, nx, wx);
      stencil<T, P>(fy, shifted, ny, wy);
      stencil<T, P>(fz, shifted, nz, wz);
      for (int c = 0; c < P; ++c) {
        const int iz = (lz + nz[c]) * E;
        for (int b = 0; b < P; ++b) {
          const int iy = (iz + ly + ny[b]) * E;
          const T wzy = wz[c] * wy[b];
          for (int a = 0; a < P; ++a) {
            const T ww = wzy * wx[a];
            T* dst = reinterpret_cast<T*>(&tile[iy + lx + nx[a]]);
            if (MODE == 0) {
              atomicAdd(dst + copy, ww * vr);
            } else {
              atomicAdd(dst, ww * vr);
              atomicAdd(dst + 1, ww * vi);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  const int mask = N - 1;
  for (int i = threadIdx.x; i < E3; i += blockDim.x) {
    const T2 v = tile[i];
    if (v.x == 0 && v.y == 0) continue;
    const int lx = i % E, ly = (i / E) % E, lz = i / (E * E);
    const int gx = (t0x - 1 + lx) & mask, gy = (t0y - 1 + ly) & mask, gz = (t0z - 1 + lz) & mask;
    T* dst = reinterpret_cast<T*>(&mesh[static_cast<int64_t>(gx) + N * (static_cast<int64_t>(gy) + static_cast<int64_t>(N) * gz)]);
    if (v.x != 0) gadd(dst, v.x);
    if (v.y != 0) gadd(dst + 1, v.y);
  }
}

template <typename T, int TT, int MODE>
hipError_t dispatch_p(int p, dim3 grid, const ObjSet<T>& o, const uint32_t* starts, const Geometry& g,
                      const SpecT<T>& f, void* mesh, hipStream_t st) {
  using T2 = typename V2<T>::type;
  const T H = static_cast<T>(g.H), rx = static_cast<T>(g.rel[0]), ry = static_cast<T>(g.rel[1]),
          rz = static_cast<T>(g.rel[2]);
  T2* m = static_cast<T2*>(mesh);
  switch (p) {
    case 1:
      deposit_kernel<T, TT, 1, MODE><<<grid, 256, 0, st>>>(o, starts, g.N, g.interlace, H, rx, ry, rz, f, m);
      break;
    case 2:
      deposit_kernel<T, TT, 2, MODE><<<grid, 256, 0, st>>>(o, starts, g.N, g.interlace, H, rx, ry, rz, f, m);
      break;
    default:
      deposit_kernel<T, TT, 3, MODE><<<grid, 256, 0, st>>>(o, starts, g.N, g.interlace, H, rx, ry, rz, f, m);
      break;
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_deposit(const ObjSet<T>& o, const uint32_t* starts, const Geometry& g, int tile,
                          const FieldSpec& f, int mode, void* mesh, hipStream_t st) {
  constexpr int TT = sizeof(T) == 4 ? kTileF32 : kTileF64;
  if (tile != TT || g.N % TT != 0) return hipErrorInvalidValue;
  const int nt = g.N / TT;
  dim3 grid(static_cast<unsigned>(nt) * nt * nt);
  const SpecT<T> sp = to_spec<T>(f);
  switch (mode) {
    case 0:
      return dispatch_p<T, TT, 0>(g.p, grid, o, starts, g, sp, mesh, st);
    case 1:
      return dispatch_p<T, TT, 1>(g.p, grid, o, starts, g, sp, mesh, st);
    default:
      return dispatch_p<T, TT, 2>(g.p, grid, o, starts, g, sp, mesh, st);
  }
}

template hipError_t launch_deposit<float>(const ObjSet<float>&, const uint32_t*, const Geometry&, int,
                                          const FieldSpec&, int, void*, hipStream_t);
template hipError_t launch_deposit<double>(const ObjSet<double>&, const uint32_t*, const Geometry&, int,
                                           const FieldSpec&, int, void*, hipStream_t);

}  // namespace lpp
