// Mass assignment as a gather over cell-sorted objects.
//
// Objects are counting-sorted by mesh cell (cell_start[c] .. cell_start[c+1]
// are the objects whose position lies in cell c).  One workgroup owns a tile
// of TX x TT x TT mesh nodes; the nodes of the tile can only receive weight from
// objects in the cells [t0-2, t0+TX] (x) and [t0-2, t0+TT] (y, z) (the TSC stencil
// of the grid reaches nodes c-1..c+2 of an object in cell c, the interlaced
// grid nodes c-1..c+1).  The workgroup stages those objects in LDS (in
// chunks of at most CAP objects, to which every region row gives an equal
// share of its objects), computing each object's line-of-sight weighted
// value once, and every thread then sums the contributions to one x-row of TX
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

// 1D assignment window W_p(x), x = (object - node) in cells, written without
// branches (the inner gather loop evaluates it for every node of a row):
//   NGP: 1 on [-1/2, 1/2);  CIC: max(0, 1-|x|);
//   TSC: 3/4 - x^2 for |x| < 1/2, (1/2) max(0, 3/2 - |x|)^2 otherwise.
template <typename T, int P>
__device__ __forceinline__ T window(T x) {
  if (P == 1) {
    const bool in = (x >= static_cast<T>(-0.5)) & (x < static_cast<T>(0.5));
    return in ? static_cast<T>(1) : static_cast<T>(0);
  }
  const T ax = fabs(x);
  if (P == 2) return fmax(static_cast<T>(0), static_cast<T>(1) - ax);
  const T inner = static_cast<T>(0.75) - ax * ax;
  const T d = fmax(static_cast<T>(0), static_cast<T>(1.5) - ax);
  const T outer = static_cast<T>(0.5) * d * d;
  return ax < static_cast<T>(0.5) ? inner : outer;
}

// w times the 1D window of the nodes at integer coordinates c, for an object
// at coordinate u (w >= 0).  TSC: with i the node nearest to u and d = u - i
// in [-1/2, 1/2], node c = i + e gets W(d - e); the quadratic
//   f(e) = 3/4 - d^2 + e d/2 + e^2 (3 d^2/2 - 5/8)
// takes the three values 1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2 at
// e = -1, 0, 1, and is <= 0 at every other integer e (its e^2 coefficient is
// negative on |d| <= 1/2, and f(+-2) = -7/4 +- d + 5 d^2 <= 0 there), so
// W = max(0, f(e)) on every node: two FMAs and a max per node instead of
// the piecewise window.
template <typename T, int P>
struct AxisWeights {
  T u, w, i, b, a1, a2;
  __device__ __forceinline__ AxisWeights(T u_, T w_) {
    if constexpr (P == 3) {
      i = rint(u_);
      const T d = u_ - i, dd = d * d;
      b = w_ * (static_cast<T>(0.75) - dd);
      a1 = w_ * (static_cast<T>(0.5) * d);
      a2 = w_ * (static_cast<T>(1.5) * dd - static_cast<T>(0.625));
    } else {
      u = u_;
      w = w_;
    }
  }
  __device__ __forceinline__ T at(int c) const;
};

constexpr int TT = 8;          // tile edge in y and z (nodes); in x a kernel parameter TX (4 or 8)
constexpr int R = TT + 3;      // region edge in y and z (cells t0-2 .. t0+TT)

template <typename T, int P>
__device__ __forceinline__ T AxisWeights<T, P>::at(int c) const {
  if constexpr (P == 3) {
    const T e = static_cast<T>(c) - i;
    return fmax(static_cast<T>(0), fma(e, fma(e, a2, a1), b));
  } else {
    return w * window<T, P>(u - static_cast<T>(c));
  }
}
constexpr int R2 = R * R;      // region rows (y, z)
constexpr int kRows = TT * TT;          // x-rows of the tile
constexpr int kParts = 4;               // threads per row: one z-offset of the stencil range each
constexpr int kThreads = kRows * kParts;
constexpr int kMaxMeshes = 8;
constexpr int kXcds = 8;  // accelerator complex dies of the device

template <typename T, int NF>
struct SpecSet {
  SpecT<T> f[NF];
};

template <typename T>
struct MeshSet {
  typename V2<T>::type* m[kMaxMeshes];
};

// staged object values per field and component, plus three positions
template <typename T, int K, int NF>
constexpr int rows_of() {
  return 3 + K * NF;
}

// accumulators per thread ([f][copy][component][x]) and per reduction round
template <int K, int NF, int TX>
constexpr int nacc_of() {
  return NF * 2 * K * TX;
}
template <int K, int NF, int TX>
constexpr int round_of() {
  return nacc_of<K, NF, TX>() % 16 == 0 ? 16 : 8;
}

template <typename T, int K, int NF, int TX>
constexpr int cap_of() {
  // the staging buffer must also hold the cross-part reduction rounds and the output rows
  constexpr int need = (kParts - 1) * kRows * (round_of<K, NF, TX>() + 1) + 2 * (TX + 1) * kRows;
  // (a 4-node x edge reaches 7 cells of objects in x instead of 11: smaller chunks)
  constexpr int base = TX == 4 ? (sizeof(T) == 4 ? 640 : 400) : (sizeof(T) == 4 ? 1024 : 640);
  constexpr int rows = rows_of<T, K, NF>();
  return base * rows >= need ? base : (need + rows - 1) / rows;
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

// Node (x, y, z) of an output mesh, z-blocked or plain.
__device__ __forceinline__ int64_t node_at(int x, int y, int z, int N, int zblocked) {
  return zblocked ? zb_index(x, y, z, N) : x + static_cast<int64_t>(N) * (y + static_cast<int64_t>(N) * z);
}
// The i-th node that a workgroup stores: node (kx, r % TT, r / TT) of the
// tile (kx < TX), in memory order, so that consecutive lanes write
// consecutive addresses: x fastest in the plain layout, z fastest and then x
// when z-blocked (a tile is TT runs of 8 TX contiguous nodes there).
template <int TX>
__device__ __forceinline__ void store_order(int i, int zblocked, int& kx, int& r) {
  if (zblocked) {
    kx = (i / TT) % TX;
    r = (i / (TT * TX)) + TT * (i % TT);
  } else {
    kx = i % TX;
    r = i / TX;
  }
}

// K = 1: NF real (density) fields, each written packed: grid -> .x, interlaced
//        grid -> .y of mesh f (.y is zero without interlacing).
// K = 2: NF complex (shape) fields; with interlacing grid -> mesh 2f and
//        interlaced grid -> mesh 2f+1, without it grid -> mesh f.  (The
//        library instantiates K = 1: the shape fields, few objects per
//        tile, go through gather_nodes_kernel below.)
// The tile is TX x TT x TT nodes (x, y, z); a 4-node x edge halves the
// accumulators per thread and the window work per object (most of the 8 x
// nodes of a row are out of an object's reach) for more tiles.
template <typename T, int P, int K, int NF, int TX>
__global__ void __launch_bounds__(kThreads) gather_kernel(GObjSet<T> o, const uint32_t* __restrict__ cell_start,
                                                          int N, int lgN, int interlace, T H, T relx, T rely, T relz,
                                                          SpecSet<T, NF> fs, MeshSet<T> out,
                                                          const uint8_t* __restrict__ tile_flags, int zblocked) {
  using T2 = typename V2<T>::type;
  constexpr int CAP = cap_of<T, K, NF, TX>();
  constexpr int ROWS = rows_of<T, K, NF>();
  constexpr int NACC = nacc_of<K, NF, TX>();  // accumulators per thread: [f][copy][component][x]
  constexpr int RW = round_of<K, NF, TX>();
  static_assert(TX == 4 || TX == TT, "x edge of 4 or 8 nodes");
  // each region row (cells x in [t0x-2, t0x+TX] at fixed y, z) is at most two
  // contiguous ranges of the cell-sorted objects (two when the row wraps)
  __shared__ uint32_t seg_beg[R2][2];
  __shared__ uint32_t seg_cnt[R2];   // objects in the first range
  __shared__ uint32_t roff[R2 + 1];  // offsets of the rows in the sorted order of the region
  __shared__ uint32_t soff[R2 + 1];  // first slot of each row in a chunk's staging order
  __shared__ uint32_t sq[R2];        // each row's share of a chunk, ceil(n_r / chunks)
  __shared__ uint32_t nchunks;
  __shared__ __align__(16) T su[ROWS][CAP];  // [0..2] region-local positions, then the values
  static_assert(R2 <= 2 * 64, "row scan uses two values per lane of one wavefront");
  const int copies = (K == 2 && interlace) ? 2 : 1;
  const int nmesh = NF * copies;

  const int nt = N / TT, ntx = N / TX;
  const int mask = N - 1;
  const int tid = threadIdx.x;
  // Workgroups are dispatched round-robin over the XCDs, each with its own L2.
  // Deal whole x tile-rows to the XCDs in turn (tile-row r to XCD r % kXcds),
  // so that x-neighbouring tiles, which read overlapping cell_start rows and
  // objects, run on the same XCD and share its L2, while every XCD still
  // gets an even share of the footprint (plain order when nt^2 is not a
  // multiple of kXcds, i.e. N = 16).
  const int xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const int tile = (nt * nt) % kXcds == 0 ? ((local / ntx) * kXcds + xcd) * ntx + local % ntx
                                           : static_cast<int>(blockIdx.x);
  const int tx = tile % ntx, ty = (tile / ntx) % nt, tz = tile / (ntx * nt);
  const int t0x = tx * TX, t0y = ty * TT, t0z = tz * TT;
  // outside the footprint (flags of the TT^3 cubes): every node of the tile
  // is zero and is never read
  if (tile_flags != nullptr && tile_flags[t0x / TT + nt * (ty + nt * tz)] == 0) return;

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
        const int xa = t0x - 2, xb = t0x + TX;  // inclusive cell range
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
    // chunks: the fewest whose per-row shares, ceil(n_r / chunks), fit in CAP;
    // row r takes the slots [soff[r], soff[r] + share) of every chunk
    const uint32_t all = __shfl(inc, 63, 64);
    uint32_t n = all <= static_cast<uint32_t>(CAP) ? 1u : (all + CAP - 1) / CAP;
    if (n > 1) {
      while (__shfl(wave_inclusive_scan((cnt[0] + n - 1) / n + (cnt[1] + n - 1) / n), 63, 64) >
             static_cast<uint32_t>(CAP))
        ++n;
    }
    if (tid == 0) nchunks = n;
    const uint32_t q0 = (cnt[0] + n - 1) / n, q1 = (cnt[1] + n - 1) / n;
    const uint32_t qinc = wave_inclusive_scan(q0 + q1);
    if (tid * 2 < R2) {
      soff[tid * 2] = qinc - q0 - q1;
      sq[tid * 2] = q0;
    }
    if (tid * 2 + 1 < R2) {
      soff[tid * 2 + 1] = qinc - q1;
      sq[tid * 2 + 1] = q1;
    }
    if (tid == 63) soff[R2] = qinc;
  }
  __syncthreads();
  const uint32_t total = roff[R2];

  // empty region: the tile is zero in every output mesh
  if (total == 0) {
    for (int i = tid; i < kRows * TX; i += kThreads) {
      int kx, r;
      store_order<TX>(i, zblocked, kx, r);
      const int64_t idx = node_at(t0x + kx, t0y + r % TT, t0z + r / TT, N, zblocked);
      for (int m = 0; m < nmesh; ++m) out.m[m][idx] = T2{0, 0};
    }
    return;
  }

  // this thread's node row: (t0x + k, t0y + ny, t0z + nz), k = 0..TX-1.  The kParts threads of a
  // row take one z-offset dz each: region rows y in [ny, ny+3] at z = nz + dz are contiguous.
  const int rowid = tid % kRows, part = tid / kRows;
  const int ny = rowid % TT, nz = rowid / TT;
  static_assert(kParts == 4, "one thread per z-offset of the stencil range");
  T acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0;

  // More objects than fit in LDS are staged in chunks, and every region row
  // gives each chunk an equal share of its objects (its next ceil(n_r / nch)
  // in sorted order, in slots of its own; a row's last share may leave slots
  // empty, which are staged as objects of zero weight), so that every thread
  // has objects in every chunk: cut into ranges of the sorted order instead,
  // a chunk would hold a few z layers of the region and leave the threads of
  // the other rows idle.  (One chunk when everything fits: the staged order
  // is then the sorted order.)
  // (block-uniform counts kept in scalar registers: read from LDS they would
  // otherwise take vector registers from the accumulators)
  const uint32_t nch = __builtin_amdgcn_readfirstlane(nchunks);
  for (uint32_t ch = 0; ch < nch; ++ch) {
    const uint32_t nc = __builtin_amdgcn_readfirstlane(soff[R2]);
    // stage the chunk: each thread takes slots d, finds the row by bisection
    for (uint32_t d = tid; d < nc; d += kThreads) {
      int lo = 0, hi = R2;  // soff[lo] <= d < soff[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (soff[mid] <= d) lo = mid; else hi = mid;
      }
      const int r = lo;
      const uint32_t j = ch * sq[r] + (d - soff[r]);  // the row's j-th object
      if (j >= roff[r + 1] - roff[r]) {  // an empty slot of the row's last share
#pragma unroll
        for (int q = 0; q < ROWS; ++q) su[q][d] = static_cast<T>(0);
        continue;
      }
      const uint32_t src = j < seg_cnt[r] ? seg_beg[r][0] + j : seg_beg[r][1] + (j - seg_cnt[r]);
      const ObjPos<T> rec = o.pos[src];
      const uint32_t key = rec.key;
      const int cx = static_cast<int>(key & mask);
      const int cy = static_cast<int>((key >> lgN) & mask);
      const int cz = static_cast<int>(key >> (2 * lgN));
      const int lx = (cx - t0x + 2) & mask, ly = r % R, lz = r / R;
      const T fx = rec.fx, fy = rec.fy, fz = rec.fz;
      su[0][d] = static_cast<T>(lx) + fx;
      su[1][d] = static_cast<T>(ly) + fy;
      su[2][d] = static_cast<T>(lz) + fz;
      // line of sight of the object
      const T px = relx + (static_cast<T>(cx) + fx) * H;
      const T py = rely + (static_cast<T>(cy) + fy) * H;
      const T pz = relz + (static_cast<T>(cz) + fz) * H;
      const T rinv = static_cast<T>(1) / sqrt(px * px + py * py + pz * pz);
      const T xx = px * rinv, xy = py * rinv, xz = pz * rinv;
      const T st = sqrt(xx * xx + xy * xy);
      const T cp = st > 0 ? xx / st : static_cast<T>(1);
      const T sp = st > 0 ? xy / st : static_cast<T>(0);
      const T ar = o.wr[src];
      const T ai = K == 2 ? o.wi[src] : static_cast<T>(0);
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        T gr = 1, gi = 0;
        if (fs.f[q].L > 0 || fs.f[q].s > 0) los_weight(fs.f[q], xz, st, cp, sp, gr, gi);
        if (K == 1) {
          su[3 + q][d] = ar * gr;
        } else {
          su[3 + 2 * q][d] = ar * gr - ai * gi;
          su[4 + 2 * q][d] = ar * gi + ai * gr;
        }
      }
    }
    __syncthreads();
    {
      const T nyc = static_cast<T>(ny + 2), nzc = static_cast<T>(nz + 2);
      const int row = ny + (nz + part) * R;  // rows y = ny..ny+3 at z = nz + part are contiguous
      const uint32_t lo = soff[row], hi = soff[row + 4];
      const T half = static_cast<T>(0.5);
      for (uint32_t d = lo; d < hi; ++d) {
        const T ux = su[0][d], uy = su[1][d], uz = su[2][d];
        const T w0 = window<T, P>(uy - nyc) * window<T, P>(uz - nzc);
        const T w1 = interlace ? window<T, P>(uy - nyc - half) * window<T, P>(uz - nzc - half) : static_cast<T>(0);
        T val[K * NF];
#pragma unroll
        for (int q = 0; q < K * NF; ++q) val[q] = su[3 + q][d];
        const AxisWeights<T, P> xw0(ux, w0), xw1(ux - half, w1);
#pragma unroll
        for (int kx = 0; kx < TX; ++kx) {
          const T wx0 = xw0.at(kx + 2);  // node kx sits at region coordinate kx + 2
          const T wx1 = xw1.at(kx + 2);
#pragma unroll
          for (int q = 0; q < NF; ++q)
#pragma unroll
            for (int c = 0; c < K; ++c) {
              acc[((q * 2 + 0) * K + c) * TX + kx] += val[q * K + c] * wx0;
              acc[((q * 2 + 1) * K + c) * TX + kx] += val[q * K + c] * wx1;
            }
        }
      }
    }
    __syncthreads();
  }
  // combine the kParts partial rows in a fixed order, RW accumulators per round
  constexpr int RS = RW + 1;  // padded against LDS bank conflicts
  T* red = &su[0][0];
#pragma unroll
  for (int r0 = 0; r0 < NACC; r0 += RW) {
    if (part > 0) {
#pragma unroll
      for (int i = 0; i < RW; ++i) red[((part - 1) * kRows + rowid) * RS + i] = acc[r0 + i];
    }
    __syncthreads();
    if (part == 0) {
#pragma unroll
      for (int q = 1; q < kParts; ++q)
#pragma unroll
        for (int i = 0; i < RW; ++i) acc[r0 + i] += red[((q - 1) * kRows + rowid) * RS + i];
    }
    __syncthreads();
  }
  // store each output mesh through LDS: consecutive lanes write consecutive nodes (store_order)
  T2* stage = reinterpret_cast<T2*>(red);
  static_assert(ROWS * CAP >= 2 * (TX + 1) * kRows, "output staging fits");
  // (the loops over fields and copies are unrolled: acc[] is only ever indexed
  // with compile-time constants, which keeps it in registers)
#pragma unroll
  for (int q = 0; q < NF; ++q) {
#pragma unroll
    for (int cpy = 0; cpy < K; ++cpy) {
      if (K == 2 && cpy >= copies) continue;
      const int m = K == 1 ? q : q * copies + cpy;
      if (part == 0) {
#pragma unroll
        for (int kx = 0; kx < TX; ++kx) {
          T2 v;
          if (K == 1)  // field q: (grid, interlaced grid)
            v = T2{acc[(q * 2 + 0) * TX + kx], acc[(q * 2 + 1) * TX + kx]};
          else         // field q, copy cpy: (re, im)
            v = T2{acc[((q * 2 + cpy) * K + 0) * TX + kx], acc[((q * 2 + cpy) * K + 1) * TX + kx]};
          stage[rowid * (TX + 1) + kx] = v;
        }
      }
      __syncthreads();
      T2* __restrict__ dst = out.m[m];
      for (int i = tid; i < kRows * TX; i += kThreads) {
        int kx, r;
        store_order<TX>(i, zblocked, kx, r);
        dst[node_at(t0x + kx, t0y + r % TT, t0z + r / TT, N, zblocked)] = stage[r * (TX + 1) + kx];
      }
      __syncthreads();
    }
  }
}

// ---- node-parallel deposit ----
//
// For the sparse shape set (galaxies only: a few tens of objects per tile
// region) the row kernel above is bound by its per-tile chain of dependent
// loads and the cross-thread reduction of its partial rows, at one pass per
// four fields.  This kernel deposits up to kNodeFields complex fields per
// pass: one thread per node of an 8^3 tile with all fields' accumulators in
// its registers, so there is no cross-thread reduction.  (It also takes real
// fields, K = 1; for the dense density set it measured slower than the row
// kernel, whose per-row window products serve several nodes, so the
// library instantiates only K = 2.)
//   1. the tile region's 11^3 cells: per cell the object count, one exclusive
//      scan over the region in (z, y, x) cell order, and each cell's first
//      object in the sorted set;
//   2. staging, in chunks of kNodeCap objects: region-local positions and
//      line-of-sight angles, then the line-of-sight weighted values with one
//      field per wavefront (the lanes do not diverge);
//   3. every node sums, in a fixed order, the objects of the 4 x 4 x 4 cells
//      that reach it (cells n-2 .. n+1 per axis): 16 runs of 4 consecutive
//      cells in the staged order, walked as one sequence per lane;
//   4. one store per field (real fields: grid and interlaced grid packed)
//      or per field and grid copy (complex fields); a wavefront writes 64
//      consecutive nodes (one y row of a z-group in the z-blocked order).
// The result is bitwise reproducible and equal, node by node, to the row
// kernel's sum over the same objects in another order, up to rounding.

constexpr int kNodeT = 512;            // threads: one per node of the 8^3 tile
constexpr int kNodeCells = R * R * R;  // 11^3 region cells
constexpr int kNodeCap = 256;          // staged objects per chunk

template <typename T>
struct MeshSetN {
  typename V2<T>::type* m[2 * kNodeFields];
};

// block-wide exclusive scan of one value per thread (512 threads, 8 wavefronts)
__device__ __forceinline__ uint32_t block_scan512(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kNodeT / 64; ++i) {
    const uint32_t s = sh[i];
    base += i < w ? s : 0u;
    tot += s;
  }
  total = tot;
  __syncthreads();
  return base + inc - v;
}

// K = 1: NF real fields, mesh q <- (grid, interlaced grid) of field q;
// K = 2: NF complex fields, mesh q * copies + c <- grid copy c of field q.
template <typename T, int P, int K, int NF>
__global__ void __launch_bounds__(kNodeT, (sizeof(T) == 4 ? 6 : 4)) gather_nodes_kernel(GObjSet<T> o, const uint32_t* __restrict__ cell_start,
                                                                 int N, int lgN, int interlace, T H, T relx, T rely,
                                                                 T relz, const SpecT<T>* __restrict__ specs,
                                                                 MeshSetN<T> out,
                                                                 const uint8_t* __restrict__ tile_flags,
                                                                 int zblocked) {
  using T2 = typename V2<T>::type;
  constexpr int ROWS = 3 + K * NF;
  constexpr int NA = 2 * K * NF;             // accumulators: [field][copy][component]
  __shared__ uint32_t coff[kNodeCells + 1];  // staged offset of each region cell (z, y, x order)
  __shared__ uint32_t cbeg[kNodeCells];      // its first object in the sorted set
  __shared__ uint32_t wsum[kNodeT / 64];
  __shared__ __align__(16) T su[ROWS][kNodeCap];
  __shared__ T trig[4][kNodeCap];            // cos theta, sin theta, cos phi, sin phi of the staged objects
  __shared__ T amp[K][kNodeCap];             // w (K = 1); w g1, w g2 (K = 2)
  __shared__ SpecT<T> sspec[NF];             // the fields' line-of-sight polynomials
  const int copies = interlace ? 2 : 1;
  const int nt = N / TT;
  const int mask = N - 1;
  const int tid = threadIdx.x;
  // whole x tile-rows to the XCDs in turn, as in gather_kernel
  const int xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const int tile = (nt * nt) % kXcds == 0 ? ((local / nt) * kXcds + xcd) * nt + local % nt
                                           : static_cast<int>(blockIdx.x);
  const int tx = tile % nt, ty = (tile / nt) % nt, tz = tile / (nt * nt);
  const int t0x = tx * TT, t0y = ty * TT, t0z = tz * TT;
  if (tile_flags != nullptr && tile_flags[tx + nt * (ty + nt * tz)] == 0) return;
  if (tid < NF) sspec[tid] = specs[tid];

  // 1. region cells: counts, scan, first objects.  Thread t takes the three
  //    consecutive cells 3t .. 3t+2 of the (z, y, x) order.
  uint32_t cnt[3], beg[3];
  uint32_t mine = 0;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int c = 3 * tid + u;
    cnt[u] = 0;
    beg[u] = 0;
    if (c < kNodeCells) {
      const int lx = c % R, ly = (c / R) % R, lz = c / (R * R);
      const int gx = (t0x - 2 + lx) & mask, gy = (t0y - 2 + ly) & mask, gz = (t0z - 2 + lz) & mask;
      const int64_t g = gx + static_cast<int64_t>(N) * (gy + static_cast<int64_t>(N) * gz);
      const uint32_t a = cell_start[g], b = cell_start[g + 1];
      beg[u] = a;
      cnt[u] = b - a;
    }
    mine += cnt[u];
  }
  uint32_t total;
  uint32_t run = block_scan512(mine, wsum, total);
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int c = 3 * tid + u;
    if (c < kNodeCells) {
      coff[c] = run;
      cbeg[c] = beg[u];
    }
    run += cnt[u];
  }
  if (tid == 0) coff[kNodeCells] = total;
  // the same in every lane: keep it (and the chunk bounds below) in scalar registers
  total = __builtin_amdgcn_readfirstlane(total);
  __syncthreads();

  // this thread's node and its place in the stores
  int kx, ky, kz;
  if (zblocked) {
    kz = tid & 7;
    kx = (tid >> 3) & 7;
    ky = tid >> 6;
  } else {
    kx = tid & 7;
    ky = (tid >> 3) & 7;
    kz = tid >> 6;
  }
  T acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0;

  const T half = static_cast<T>(0.5);
  for (uint32_t c0 = 0; c0 < total; c0 += kNodeCap) {
    const uint32_t c1 = min(total, c0 + static_cast<uint32_t>(kNodeCap));
    const int nc = static_cast<int>(c1 - c0);
    // 2a. positions, line-of-sight angles and weights of the chunk's objects
    for (int d = tid; d < nc; d += kNodeT) {
      const uint32_t k = c0 + d;
      int lo = 0, hi = kNodeCells;  // coff[lo] <= k < coff[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (coff[mid] <= k) lo = mid; else hi = mid;
      }
      const uint32_t src = cbeg[lo] + (k - coff[lo]);
      const ObjPos<T> rec = o.pos[src];
      const uint32_t key = rec.key;
      const int cx = static_cast<int>(key & mask);
      const int cy = static_cast<int>((key >> lgN) & mask);
      const int cz = static_cast<int>(key >> (2 * lgN));
      const int lx = lo % R, ly = (lo / R) % R, lz = lo / (R * R);
      su[0][d] = static_cast<T>(lx) + rec.fx;
      su[1][d] = static_cast<T>(ly) + rec.fy;
      su[2][d] = static_cast<T>(lz) + rec.fz;
      const T px = relx + (static_cast<T>(cx) + rec.fx) * H;
      const T py = rely + (static_cast<T>(cy) + rec.fy) * H;
      const T pz = relz + (static_cast<T>(cz) + rec.fz) * H;
      const T rinv = static_cast<T>(1) / sqrt(px * px + py * py + pz * pz);
      const T xx = px * rinv, xy = py * rinv, xz = pz * rinv;
      const T st = sqrt(xx * xx + xy * xy);
      trig[0][d] = xz;
      trig[1][d] = st;
      trig[2][d] = st > 0 ? xx / st : static_cast<T>(1);
      trig[3][d] = st > 0 ? xy / st : static_cast<T>(0);
      amp[0][d] = o.wr[src];
      if (K == 2) amp[K - 1][d] = o.wi[src];
    }
    __syncthreads();
    // 2b. the line-of-sight weighted values: wavefront w takes the fields
    //     q = w, w + 8, .. (one polynomial per wavefront, so its lanes do not
    //     diverge), its lanes the objects
    {
      const int wave = tid >> 6, lane = tid & 63;
      for (int q = wave; q < NF; q += kNodeT / 64) {
        const SpecT<T>& f = sspec[q];
        const bool plain = f.L == 0 && f.s == 0;
        for (int d = lane; d < nc; d += 64) {
          T gr = 1, gi = 0;
          if (!plain) los_weight(f, trig[0][d], trig[1][d], trig[2][d], trig[3][d], gr, gi);
          if (K == 1) {
            su[3 + q][d] = amp[0][d] * gr;
          } else {
            const T ar = amp[0][d], ai = amp[K - 1][d];
            su[3 + 2 * q][d] = ar * gr - ai * gi;
            su[3 + 2 * q + (K - 1)][d] = ar * gi + ai * gr;
          }
        }
      }
    }
    __syncthreads();
    // 3. this node's sums: cells x in kx..kx+3, y in ky..ky+3, z in kz..kz+3 of
    //    the region, as 16 runs r = 4 dz + dy of four cells along x.  The
    //    non-empty runs (a 16-bit mask per lane) are walked as one sequence
    //    per lane, so that a wavefront spends as many steps as its busiest
    //    node has objects, not the sum over the runs of the busiest node's
    //    objects in each run (most runs are empty or hold one object).  The
    //    order of the terms is the same as run by run.
    const T nxc = static_cast<T>(kx + 2), nyc = static_cast<T>(ky + 2), nzc = static_cast<T>(kz + 2);
    {
      const int cbase = kx + R * (ky + R * kz);
      uint32_t runs = 0, left = 0;
      // (not unrolled: the run's offset stays a scalar, and sixteen cell
      // indices are not kept live across the chunks)
#pragma unroll 1
      for (int r = 0; r < 16; ++r) {
        const int cell0 = cbase + R * ((r & 3) + R * (r >> 2));
        const uint32_t lo = max(coff[cell0], c0), hi = min(coff[cell0 + 4], c1);
        if (lo < hi) {
          runs |= 1u << r;
          left += hi - lo;
        }
      }
      // one step per object of this node; the loop's only exit is its count
      // (an exit from inside the divergent branch made the compiler copy the
      // accumulators on every step)
      uint32_t k = 0, hi = 0;
      for (; left > 0; --left) {
        if (k >= hi) {
          const int r = __builtin_ctz(runs);
          runs &= runs - 1;
          const int cell0 = cbase + R * ((r & 3) + R * (r >> 2));
          k = max(coff[cell0], c0);
          hi = min(coff[cell0 + 4], c1);
        }
        {
          const int d = static_cast<int>(k - c0);
          const T ux = su[0][d], uy = su[1][d], uz = su[2][d];
          const T w0 = window<T, P>(ux - nxc) * window<T, P>(uy - nyc) * window<T, P>(uz - nzc);
          const T w1 = interlace ? window<T, P>(ux - nxc - half) * window<T, P>(uy - nyc - half) *
                                       window<T, P>(uz - nzc - half)
                                 : static_cast<T>(0);
#pragma unroll
          for (int q = 0; q < NF; ++q)
#pragma unroll
            for (int c = 0; c < K; ++c) {
              const T v = su[3 + K * q + c][d];
              acc[(2 * q + 0) * K + c] += v * w0;
              acc[(2 * q + 1) * K + c] += v * w1;
            }
        }
        ++k;
      }
    }
    __syncthreads();
  }
  // 4. stores
  const int64_t idx = node_at(t0x + kx, t0y + ky, t0z + kz, N, zblocked);
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    if (K == 1) {
      out.m[q][idx] = T2{acc[2 * q], acc[2 * q + 1]};
    } else {
      out.m[q * copies][idx] = T2{acc[(2 * q) * K], acc[(2 * q) * K + 1]};
      if (interlace) out.m[q * copies + 1][idx] = T2{acc[(2 * q + 1) * K], acc[(2 * q + 1) * K + 1]};
    }
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
__global__ void cell_scatter_kernel(RawCat c, Geometry g, double wscale, const double* __restrict__ wscale_dev,
                                    int shape, const uint32_t* starts, const uint32_t* rank,
                                    const uint32_t* cell_of_obj, GObjSet<T> out, uint32_t* __restrict__ order,
                                    uint32_t index_base) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= c.n) return;
  if (wscale_dev != nullptr) wscale *= *wscale_dev;
  const int N = g.N;
  const double ux = (ldc(c.x, i, c.dtype) - g.origin[0]) / g.H;
  const double uy = (ldc(c.y, i, c.dtype) - g.origin[1]) / g.H;
  const double uz = (ldc(c.z, i, c.dtype) - g.origin[2]) / g.H;
  const int cx = cell_of(ux, N), cy = cell_of(uy, N), cz = cell_of(uz, N);
  const uint32_t cell = cell_of_obj[i];
  const int64_t d = static_cast<int64_t>(starts[cell]) + rank[i];
  ObjPos<T> rec;
  rec.key = cell;
  rec.fx = static_cast<T>(ux - cx);
  rec.fy = static_cast<T>(uy - cy);
  rec.fz = static_cast<T>(uz - cz);
  out.pos[d] = rec;
  order[d] = index_base + static_cast<uint32_t>(i);
  const double w = c.w ? ldc(c.w, i, c.dtype) : 1.0;
  if (shape) {
    out.wr[d] = static_cast<T>(w * ldc(c.g1, i, c.dtype));
    out.wi[d] = static_cast<T>(w * ldc(c.g2, i, c.dtype));
  } else {
    out.wr[d] = static_cast<T>(wscale * w);
  }
}

// The atomic ranks of cell_count_kernel leave the objects of a cell in an
// order that changes from run to run, and the gather sums them in storage
// order.  This puts every cell's objects in the order of their index in the
// set (insertion sort by that index; cells hold a handful of objects), which
// makes the sort, and with it the deposit, bitwise reproducible.
constexpr int kOrderCells = 8;  // cells per thread of cell_order_kernel

template <typename T>
__global__ void cell_order_kernel(const uint32_t* __restrict__ starts, int64_t ncell, uint32_t* __restrict__ order,
                                  GObjSet<T> o, int shape) {
  const int64_t c0 = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) * kOrderCells;
  if (c0 >= ncell) return;
  // the starts of kOrderCells consecutive cells and the end of the last one
  uint32_t st[kOrderCells + 1];
#pragma unroll
  for (int u = 0; u <= kOrderCells; ++u) st[u] = c0 + u <= ncell ? starts[c0 + u] : st[u - 1];
#pragma unroll
  for (int u = 0; u < kOrderCells; ++u) {
    const uint32_t s = st[u], e = st[u + 1];
    if (e - s < 2) continue;
    for (uint32_t i = s + 1; i < e; ++i) {
      const uint32_t k = order[i];
      const ObjPos<T> rec = o.pos[i];
      const T wr = o.wr[i];
      const T wi = shape ? o.wi[i] : static_cast<T>(0);
      uint32_t j = i;
      while (j > s && order[j - 1] > k) {
        order[j] = order[j - 1];
        o.pos[j] = o.pos[j - 1];
        o.wr[j] = o.wr[j - 1];
        if (shape) o.wi[j] = o.wi[j - 1];
        --j;
      }
      if (j != i) {
        order[j] = k;
        o.pos[j] = rec;
        o.wr[j] = wr;
        if (shape) o.wi[j] = wi;
      }
    }
  }
}

// exclusive scan of n counts into starts[0..n] (starts[n] = total), three phases
constexpr int kScanT = 1024;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanT * kScanPer;

// exclusive scan of one value per thread across the block: a scan within
// each wavefront (shuffles), then a scan of the wavefront totals.  sh holds
// kScanT / 64 + 1 values.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  constexpr int kWaves = kScanT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const uint32_t t = lane < kWaves ? sh[lane] : 0u;
    const uint32_t ti = wave_inclusive_scan(t);
    if (lane < kWaves) sh[lane] = ti - t;
    if (lane == kWaves - 1) sh[kWaves] = ti;
  }
  __syncthreads();
  total = sh[kWaves];
  const uint32_t r = sh[wave] + inc - v;
  __syncthreads();  // sh may be reused on return
  return r;
}

// the kScanPer values of one thread (zeros past n); 16-byte loads when the
// whole run is in range (base is a multiple of kScanPer)
__device__ __forceinline__ void scan_load(const uint32_t* in, int64_t base, int64_t n, uint32_t* v) {
  static_assert(kScanPer == 8, "two 16-byte loads per thread");
  if (base + kScanPer <= n) {
    const uint4 a = *reinterpret_cast<const uint4*>(in + base);
    const uint4 b = *reinterpret_cast<const uint4*>(in + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = base + k < n ? in[base + k] : 0u;
  }
}

__global__ void __launch_bounds__(kScanT) scan_reduce_kernel(const uint32_t* in, int64_t n, uint32_t* bsum) {
  __shared__ uint32_t sh[kScanT / 64 + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + static_cast<int64_t>(threadIdx.x) * kScanPer;
  uint32_t v[kScanPer];
  scan_load(in, base, n, v);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) s += v[k];
  uint32_t tot;
  block_exclusive_scan(s, sh, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanT) scan_blocks_kernel(uint32_t* bsum, int nb) {
  // single block: exclusive scan of nb block sums in place; bsum[nb] = grand total
  __shared__ uint32_t sh[kScanT / 64 + 1];
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
  __shared__ uint32_t sh[kScanT / 64 + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + static_cast<int64_t>(threadIdx.x) * kScanPer;
  uint32_t v[kScanPer];
  scan_load(in, base, n, v);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) s += v[k];
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, sh, tot) + bsum[blockIdx.x];
  uint32_t o[kScanPer];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    o[k] = run;
    run += v[k];
  }
  if (base + kScanPer <= n) {  // (in and out may be the same buffer: this thread's values are read above)
    *reinterpret_cast<uint4*>(out + base) = uint4{o[0], o[1], o[2], o[3]};
    *reinterpret_cast<uint4*>(out + base + 4) = uint4{o[4], o[5], o[6], o[7]};
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
      if (base + k < n) out[base + k] = o[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

// x edge of the deposit tile.  Density passes (K = 1: the randoms, many
// objects per tile, bound by the row sums) take 4 nodes: half the
// accumulators and of the window work per object, more workgroups per CU.
// FP32 shape passes (K = 2: the galaxies only, few objects per tile, bound
// by the per-tile chain of loads) keep 8, since halving the tile doubles the
// tiles; FP64 shape passes take 4, which leaves registers for four fields
// per pass instead of two (half the passes).
template <typename T, int K>
constexpr int tile_x() {
  return (K == 1 || sizeof(T) == 8) ? 4 : TT;
}

template <typename T, int K, int NF>
hipError_t dispatch(int p, const GObjSet<T>& o, const uint32_t* starts, const Geometry& g,
                    const FieldSpec* specs, void* const* meshes, const uint8_t* tiles, int zb, hipStream_t st) {
  // the line of sight of an object in cell c at fraction f: rel + (c + f) H
  const T H = static_cast<T>(g.los_h), rx = static_cast<T>(g.los_rel[0]), ry = static_cast<T>(g.los_rel[1]),
          rz = static_cast<T>(g.los_rel[2]);
  SpecSet<T, NF> fs;
  for (int q = 0; q < NF; ++q) fs.f[q] = to_spec<T>(specs[q]);
  MeshSet<T> ms{};
  const int nm = (K == 2 && g.interlace) ? 2 * NF : NF;
  for (int m = 0; m < nm; ++m) ms.m[m] = static_cast<typename V2<T>::type*>(meshes[m]);
  int lg = 0;
  while ((1 << lg) < g.N) ++lg;
  constexpr int TX = tile_x<T, K>();
  const int nt = g.N / TT;
  const dim3 grid(static_cast<unsigned>(g.N / TX) * nt * nt);
  switch (p) {
    case 1:
      gather_kernel<T, 1, K, NF, TX><<<grid, kThreads, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz, fs, ms,
                                                                 tiles, zb);
      break;
    case 2:
      gather_kernel<T, 2, K, NF, TX><<<grid, kThreads, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz, fs, ms,
                                                                 tiles, zb);
      break;
    default:
      gather_kernel<T, 3, K, NF, TX><<<grid, kThreads, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz, fs, ms,
                                                                 tiles, zb);
      break;
  }
  return hipGetLastError();
}

// ---- footprint of a cell-sorted set ----

// One thread per node row (y, z): flagged when a cell row (y + dy, z + dz),
// dy, dz in -2..1, holds an object (cell rows are contiguous in the sorted order).
__global__ void footprint_rows_kernel(const uint32_t* __restrict__ cell_start, int N, uint8_t* __restrict__ row) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= static_cast<int64_t>(N) * N) return;
  const int y = static_cast<int>(i % N), z = static_cast<int>(i / N);
  const int mask = N - 1;
  uint32_t any = 0;
  for (int dz = -2; dz <= 1; ++dz)
    for (int dy = -2; dy <= 1; ++dy) {
      const int64_t r = static_cast<int64_t>(N) * (((y + dy) & mask) + static_cast<int64_t>(N) * ((z + dz) & mask));
      any |= cell_start[r + N] - cell_start[r];
    }
  row[i] = any != 0 ? 1 : 0;
}

// One thread per tile: flagged when one of the 11 x 11 cell rows of its
// region holds an object in cells x = t0x-2 .. t0x+8 (with wrap-around).
__global__ void footprint_cubes_kernel(const uint32_t* __restrict__ cell_start, int N, uint8_t* __restrict__ cube) {
  const int nt = N / kTile;
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= static_cast<int64_t>(nt) * nt * nt) return;
  const int tx = static_cast<int>(i % nt), ty = static_cast<int>((i / nt) % nt), tz = static_cast<int>(i / (nt * nt));
  const int mask = N - 1;
  const int xa = tx * kTile - 2, xb = tx * kTile + kTile;  // inclusive cell range
  uint32_t any = 0;
  for (int dz = -2; dz <= kTile; ++dz)
    for (int dy = -2; dy <= kTile; ++dy) {
      const int64_t r = static_cast<int64_t>(N) * (((ty * kTile + dy) & mask) +
                                                   static_cast<int64_t>(N) * ((tz * kTile + dz) & mask));
      if (xa < 0) {
        any |= cell_start[r + N] - cell_start[r + N + xa];
        any |= cell_start[r + xb + 1] - cell_start[r];
      } else if (xb >= N) {
        any |= cell_start[r + N] - cell_start[r + xa];
        any |= cell_start[r + xb - N + 1] - cell_start[r];
      } else {
        any |= cell_start[r + xb + 1] - cell_start[r + xa];
      }
    }
  cube[i] = any != 0 ? 1 : 0;
}

// Threads [0, nt^2): tile-row flags; threads [nt^2, nt^2 + N): plane flags.
__global__ void footprint_reduce_kernel(int N, Footprint fp) {
  const int nt = N / kTile;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nt * nt) {
    const int ty = i % nt, tz = i / nt;
    uint8_t any = 0;
    for (int dz = 0; dz < kTile; ++dz)
      for (int dy = 0; dy < kTile; ++dy)
        any |= fp.row[(ty * kTile + dy) + static_cast<int64_t>(N) * (tz * kTile + dz)];
    fp.tile[i] = any;
  } else if (i < nt * nt + N) {
    const int z = i - nt * nt;
    uint8_t any = 0;
    for (int y = 0; y < N; ++y) any |= fp.row[y + static_cast<int64_t>(N) * z];
    fp.plane[z] = any;
  }
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
hipError_t launch_cell_scatter(const RawCat& c, const Geometry& g, double wscale, const double* wscale_dev, int shape, const uint32_t* starts,
                               const uint32_t* rank, const uint32_t* cell_of_obj, GObjSet<T> out, uint32_t* order,
                               int64_t index_base, hipStream_t st) {
  if (c.n == 0) return hipSuccess;
  cell_scatter_kernel<T><<<static_cast<unsigned>((c.n + 255) / 256), 256, 0, st>>>(
      c, g, wscale, wscale_dev, shape, starts, rank, cell_of_obj, out, order, static_cast<uint32_t>(index_base));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cell_order(const uint32_t* starts, int64_t ncell, uint32_t* order, GObjSet<T> out, int shape,
                             hipStream_t st) {
  const int64_t threads = (ncell + kOrderCells - 1) / kOrderCells;
  cell_order_kernel<T><<<static_cast<unsigned>((threads + 255) / 256), 256, 0, st>>>(starts, ncell, order, out, shape);
  return hipGetLastError();
}

template <typename T, int K, int NF>
hipError_t dispatch_nodes(int p, const GObjSet<T>& o, const uint32_t* starts, const Geometry& g,
                          const SpecT<T>* specs, void* const* meshes, const uint8_t* tiles, int zb,
                          hipStream_t st) {
  const T H = static_cast<T>(g.los_h), rx = static_cast<T>(g.los_rel[0]), ry = static_cast<T>(g.los_rel[1]),
          rz = static_cast<T>(g.los_rel[2]);
  MeshSetN<T> ms{};
  const int nm = (K == 2 && g.interlace) ? 2 * NF : NF;
  for (int m = 0; m < nm; ++m) ms.m[m] = static_cast<typename V2<T>::type*>(meshes[m]);
  int lg = 0;
  while ((1 << lg) < g.N) ++lg;
  const int nt = g.N / TT;
  const dim3 grid(static_cast<unsigned>(nt) * nt * nt);
  switch (p) {
    case 1:
      gather_nodes_kernel<T, 1, K, NF><<<grid, kNodeT, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz,
                                                                 specs, ms, tiles, zb);
      break;
    case 2:
      gather_nodes_kernel<T, 2, K, NF><<<grid, kNodeT, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz,
                                                                 specs, ms, tiles, zb);
      break;
    default:
      gather_nodes_kernel<T, 3, K, NF><<<grid, kNodeT, 0, st>>>(o, starts, g.N, lg, g.interlace, H, rx, ry, rz,
                                                                 specs, ms, tiles, zb);
      break;
  }
  return hipGetLastError();
}

template <typename T, int K, int NF>
hipError_t nodes_upto(int nf, int p, const GObjSet<T>& o, const uint32_t* starts, const Geometry& g,
                      const SpecT<T>* specs, void* const* meshes, const uint8_t* tiles, int zb, hipStream_t st) {
  if constexpr (NF == 0) {
    return hipErrorInvalidValue;
  } else {
    if (nf == NF) return dispatch_nodes<T, K, NF>(p, o, starts, g, specs, meshes, tiles, zb, st);
    return nodes_upto<T, K, NF - 1>(nf, p, o, starts, g, specs, meshes, tiles, zb, st);
  }
}

hipError_t launch_gather_nodes(const GObjSet<float>& o, const uint32_t* cell_start, const Geometry& g,
                               const SpecT<float>* specs, int nf, void* const* meshes, const uint8_t* tile_flags,
                               bool zblocked, hipStream_t st) {
  const int zb = zblocked ? 1 : 0;
  if (g.N % TT != 0 || nf < 1) return hipErrorInvalidValue;
  return nodes_upto<float, 2, kNodeFields>(nf, g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
}

hipError_t launch_gather_nodes(const GObjSet<double>& o, const uint32_t* cell_start, const Geometry& g,
                               const SpecT<double>* specs, int nf, void* const* meshes,
                               const uint8_t* tile_flags, bool zblocked, hipStream_t st) {
  const int zb = zblocked ? 1 : 0;
  if (g.N % TT != 0 || nf < 1) return hipErrorInvalidValue;
  return nodes_upto<double, 2, kNodeFieldsF64>(nf, g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
}

template <typename T>
hipError_t launch_gather(const GObjSet<T>& o, const uint32_t* cell_start, const Geometry& g, const FieldSpec* specs,
                         int nf, void* const* meshes, const uint8_t* tile_flags, bool zblocked, hipStream_t st) {
  static_assert(TT == kTile && TT == kZb, "footprint tiles are gather tiles and z-groups");
  const int zb = zblocked ? 1 : 0;
  if (g.N % TT != 0) return hipErrorInvalidValue;
  static_assert(kGatherMaxReal == 8 && kGatherMaxRealF64 == 8, "real passes of 1 to 8 fields");
  switch (nf) {
    case 1: return dispatch<T, 1, 1>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 2: return dispatch<T, 1, 2>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 3: return dispatch<T, 1, 3>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 4: return dispatch<T, 1, 4>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 5: return dispatch<T, 1, 5>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 6: return dispatch<T, 1, 6>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 7: return dispatch<T, 1, 7>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    case 8: return dispatch<T, 1, 8>(g.p, o, cell_start, g, specs, meshes, tile_flags, zb, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_footprint(const uint32_t* cell_start, int N, Footprint fp, hipStream_t st) {
  if (N % kTile != 0) return hipErrorInvalidValue;
  const int64_t rows = static_cast<int64_t>(N) * N;
  footprint_rows_kernel<<<static_cast<unsigned>((rows + 255) / 256), 256, 0, st>>>(cell_start, N, fp.row);
  const int nt = N / kTile;
  const int nred = nt * nt + N;
  footprint_reduce_kernel<<<(nred + 255) / 256, 256, 0, st>>>(N, fp);
  const int64_t ncube = static_cast<int64_t>(nt) * nt * nt;
  footprint_cubes_kernel<<<static_cast<unsigned>((ncube + 255) / 256), 256, 0, st>>>(cell_start, N, fp.cube);
  return hipGetLastError();
}

template hipError_t launch_cell_scatter<float>(const RawCat&, const Geometry&, double, const double*, int, const uint32_t*,
                                               const uint32_t*, const uint32_t*, GObjSet<float>, uint32_t*, int64_t,
                                               hipStream_t);
template hipError_t launch_cell_scatter<double>(const RawCat&, const Geometry&, double, const double*, int, const uint32_t*,
                                                const uint32_t*, const uint32_t*, GObjSet<double>, uint32_t*, int64_t,
                                                hipStream_t);
template hipError_t launch_cell_order<float>(const uint32_t*, int64_t, uint32_t*, GObjSet<float>, int, hipStream_t);
template hipError_t launch_cell_order<double>(const uint32_t*, int64_t, uint32_t*, GObjSet<double>, int, hipStream_t);
template hipError_t launch_gather<float>(const GObjSet<float>&, const uint32_t*, const Geometry&, const FieldSpec*,
                                         int, void* const*, const uint8_t*, bool, hipStream_t);
template hipError_t launch_gather<double>(const GObjSet<double>&, const uint32_t*, const Geometry&, const FieldSpec*,
                                         int, void* const*, const uint8_t*, bool, hipStream_t);

}  // namespace lpp
