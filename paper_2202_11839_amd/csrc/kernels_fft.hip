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
//
// With a footprint (FftPrune) the passes skip what is known to be zero or
// never read: the x pass skips unflagged rows and reads the segments of
// flagged cubes only; the y pass skips unflagged
// planes, reads flagged rows only and stores the (kx, ky) inside the last
// k-shell only; the z pass reads flagged planes only, skips the (kx, ky)
// columns outside the last k-shell and stores the modes inside it only.
//
// The estimator's meshes are z-blocked (lpp_internal.h): fft_zb_kernel runs
// the same three passes on that layout, with every workgroup owning whole
// groups of 8 z-values, so that each HBM access is a run of 64 (FP32) or 128
// (FP64) contiguous bytes per line, and the lanes of a wavefront cover 8
// such runs side by side wherever the lines allow it.  Every element is read
// and written once per pass, with non-temporal (streaming) accesses where
// the runs are long enough.
#include <climits>

#include "device_common.h"

namespace lpp {

namespace {

using dev::V2;

template <typename T, int N, int NCOL, bool ALONG>
__global__ void __launch_bounds__(NCOL* N / 8) fft_axis_kernel(typename V2<T>::type* __restrict__ data, int axis,
                                                              const typename V2<T>::type* __restrict__ tw,
                                                              FftPrune pr) {
  using T2 = typename V2<T>::type;
  constexpr int TL = N / 8;
  __shared__ T2 sm[NCOL * N];
  __shared__ T2 stw[N];  // twiddles: reading them from LDS instead of global memory
                         // keeps them out of the path of the strided data accesses
  const int tid = threadIdx.x;
  int col, t;
  if constexpr (ALONG) {
    t = tid % TL;
    col = tid / TL;
  } else {
    col = tid % NCOL;
    t = tid / NCOL;
  }
  int64_t base, stride;
  bool live = true;            // this column is read and written
  // outputs are stored where qline + m^2 < qstore, m the output's signed mode:
  // the y pass keeps nx^2 + ny^2 < qmax and the z pass |n|^2 < qmax
  int qline = 0, qstore = INT_MAX;
  const uint8_t* lflag = nullptr;  // load flags along the line (nullable): element e reads lflag[e >> lshift]
  int lshift = 0;
  if constexpr (ALONG) {  // the x axis
    const int64_t line = static_cast<int64_t>(blockIdx.x) * NCOL + col;  // y + N z
    base = line * N;
    stride = 1;
    if (pr.row) {
      // the rows of a block are consecutive: skip the block when none is flagged
      int any = 0;
      const int64_t l0 = static_cast<int64_t>(blockIdx.x) * NCOL;
#pragma unroll
      for (int c = 0; c < NCOL; ++c) any |= pr.row[l0 + c];
      if (!any) return;
      live = pr.row[line] != 0;
    }
    if (pr.cube) {
      const int64_t y = line % N, z = line / N;
      const int nt = N / kTile;
      lflag = pr.cube + nt * ((y / kTile) + nt * (z / kTile));
      lshift = 3;
      static_assert(kTile == 8, "segment flags by x >> 3");
    }
  } else {
    static_assert(NCOL <= N, "column blocks within one line of the other axis");
    constexpr int nchunk = N / NCOL;
    const int chunk = blockIdx.x % nchunk;
    const int other = blockIdx.x / nchunk;
    const int x = chunk * NCOL + col;
    if (axis == 1) {  // other = z
      if (pr.plane && !pr.plane[other]) return;  // the whole plane is zero
      base = x + static_cast<int64_t>(N) * N * other;
      stride = N;
      if (pr.row) {
        lflag = pr.row + static_cast<int64_t>(N) * other;
      }
      const int nx = dev::sgn_mode(x, N);
      qline = nx * nx;
      qstore = pr.qmax;
    } else {  // other = y index (ky after the y pass), x = kx
      // the whole block of columns outside the last k-shell: nothing to do
      const int c0 = chunk * NCOL;  // NCOL | N/2, so the chunk's modes share a sign
      const int mx = c0 < N / 2 ? c0 : N - c0 - (NCOL - 1);
      const int nyb = dev::sgn_mode(other, N);
      if (mx * mx + nyb * nyb >= pr.qmax) return;
      base = x + static_cast<int64_t>(N) * other;
      stride = static_cast<int64_t>(N) * N;
      const int nx = dev::sgn_mode(x, N), ny = dev::sgn_mode(other, N);
      live = nx * nx + ny * ny < pr.qmax;
      lflag = pr.plane;
      qline = nx * nx + ny * ny;
      qstore = pr.qmax;
    }
  }
  // pass-0 inputs of this thread: elements t + j*N/8.  The flags are loaded
  // first, all together, so that the predicated data loads are then in flight
  // together too.
  bool rd[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) rd[j] = live;
  if (lflag != nullptr) {
    uint8_t f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = lflag[(t + j * TL) >> lshift];
#pragma unroll
    for (int j = 0; j < 8; ++j) rd[j] = rd[j] && f[j] != 0;
  }
  T2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    v[j] = T2{0, 0};
    if (rd[j]) v[j] = data[base + static_cast<int64_t>(t + j * TL) * stride];
  }
  // (fft_column_regs has a barrier after its first exchange, before the first twiddle is read)
  for (int i = tid; i < N; i += NCOL * TL) stw[i] = tw[i];
  dev::fft_column_regs<T, N>(stw, sm, col, t, v);
  if (!live) return;
  int row[8];
  dev::fft_rows<N>(t, row);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int m = dev::sgn_mode(row[q], N);
    if (qline + m * m < qstore) data[base + static_cast<int64_t>(row[q]) * stride] = v[q];
  }
}

// The passes on a z-blocked mesh.  Lines of a workgroup:
//   x pass: the 8 z of one z-group for NL/8 consecutive rows y; the lanes run
//           over z%8 first and then along x, so that 8 lanes read the 64
//           contiguous values of 8 consecutive x;
//   y pass: the 8 z of one z-group for NL/8 consecutive columns x; the lanes
//           run across the lines (one contiguous run of NL values per y);
//   z pass: NL consecutive columns x of one row y; the lanes run over z%8
//           first and then across the columns (for N >= 64).
// Pruning as in fft_axis_kernel.  Element e of a thread's line sits at
// base + (e >> 3) * hi + (e & 7) * lo.
// waves per SIMD that the LDS allows (up to two workgroups per CU): the
// kernel must leave registers for them
template <typename T, int N, int NL>
constexpr int zb_min_waves() {
  constexpr int threads = NL * N / 8;
  constexpr size_t lds = static_cast<size_t>(NL + 1) * N * sizeof(typename V2<T>::type);
  constexpr int blocks = lds * 2 <= 160 * 1024 ? 2 : 1;
  constexpr int w = blocks * threads / 256;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <typename T, int N, int NL, bool ALONG, bool NT>
__global__ void __launch_bounds__(NL* N / 8, (zb_min_waves<T, N, NL>())) fft_zb_kernel(typename V2<T>::type* __restrict__ data, int axis,
                                                           const typename V2<T>::type* __restrict__ tw,
                                                           FftPrune pr) {
  using T2 = typename V2<T>::type;
  constexpr int TL = N / 8;
  constexpr int G = NL / kZb;  // rows (x pass) or columns (y pass) per workgroup
  static_assert(NL % kZb == 0, "whole z-groups");
  __shared__ T2 sm[NL * N];
  __shared__ T2 stw[N];
  const int tid = threadIdx.x;
  const int64_t NN = static_cast<int64_t>(N) * N;
  int col, t, swz;
  int64_t base, hi, lo;
  bool live = true;
  int qline = 0, qstore = INT_MAX;
  const uint8_t* lflag = nullptr;  // load flags along the line (nullable): element e reads lflag[e >> lshift]
  int lshift = 0;
  if constexpr (ALONG) {
    const int c = tid & 7, g = tid / (8 * TL);
    t = (tid >> 3) % TL;
    col = c + 8 * g;
    swz = dev::swizzle_rows8<N>(col);
    const int yb = blockIdx.x % (N / G), zg = blockIdx.x / (N / G);
    const int y = yb * G + g, z = zg * kZb + c;
    if (pr.row) {
      int any = 0;
#pragma unroll
      for (int r = 0; r < G; ++r)
#pragma unroll
        for (int cc = 0; cc < kZb; ++cc) any |= pr.row[yb * G + r + static_cast<int64_t>(N) * (zg * kZb + cc)];
      if (!any) return;
      live = pr.row[y + static_cast<int64_t>(N) * z] != 0;
    }
    if (pr.cube) {
      const int nt = N / kTile;
      lflag = pr.cube + nt * ((y / kTile) + nt * (z / kTile));
      lshift = 3;
    }
    base = zb_index(0, y, z, N);
    hi = 8 * kZb;
    lo = kZb;
  } else if (axis == 1) {
    col = tid % NL;
    t = tid / NL;
    swz = col & 15;
    int bid = blockIdx.x;
    if constexpr (G == 1 && sizeof(T) == 4) {
      // one FP32 column per workgroup reads 64-byte runs, and the columns
      // x = 2p and 2p + 1 share every 128-byte line: both go to the same XCD
      // (workgroups are dealt to the eight XCDs in turn, so blocks b and
      // b + 8 of each 16 share one; the grid is a multiple of 16)
      const int r = bid & 15;
      bid = (bid & ~15) | ((r & 7) << 1) | (r >> 3);
    }
    const int xc = bid % (N / G), zg = bid / (N / G);
    const int x = xc * G + (col >> 3), z = zg * kZb + (col & 7);
    if (pr.plane) {
      int any = 0;
#pragma unroll
      for (int cc = 0; cc < kZb; ++cc) any |= pr.plane[zg * kZb + cc];
      if (!any) return;  // the whole z-group is zero
      live = pr.plane[z] != 0;
    }
    if (pr.row) lflag = pr.row + static_cast<int64_t>(N) * z;
    base = zb_index(x, 0, z, N);
    hi = 8 * static_cast<int64_t>(N) * kZb;
    lo = static_cast<int64_t>(N) * kZb;
    const int nx = dev::sgn_mode(x, N);
    qline = nx * nx;
    qstore = pr.qmax;
  } else {
    if (TL >= 8) {
      col = (tid >> 3) % NL;
      t = (tid & 7) | ((tid / (8 * NL)) << 3);
      swz = dev::swizzle_rows8<N>(col);
    } else {
      col = tid % NL;
      t = tid / NL;
      swz = col & 15;
    }
    const int xc = blockIdx.x % (N / NL), y = blockIdx.x / (N / NL);
    // the whole block of columns outside the last k-shell: nothing to do
    // (mx is the chunk's smallest |nx| when NL | N/2, and 0 otherwise)
    const int c0 = xc * NL;
    const int mx = c0 < N / 2 ? c0 : N - c0 - (NL - 1);
    const int nyb = dev::sgn_mode(y, N);
    if (mx * mx + nyb * nyb >= pr.qmax) return;
    const int x = c0 + col;
    const int nx = dev::sgn_mode(x, N), ny = dev::sgn_mode(y, N);
    live = nx * nx + ny * ny < pr.qmax;
    lflag = pr.plane;
    qline = nx * nx + ny * ny;
    qstore = pr.qmax;
    base = zb_index(x, y, 0, N);
    hi = NN * kZb;
    lo = 1;
  }
  bool rd[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) rd[j] = live;
  if (lflag != nullptr) {
    uint8_t f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = lflag[(t + j * TL) >> lshift];
#pragma unroll
    for (int j = 0; j < 8; ++j) rd[j] = rd[j] && f[j] != 0;
  }
  T2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = t + j * TL;
    const T2* src = &data[base + (e >> 3) * hi + (e & 7) * lo];
    v[j] = T2{0, 0};
    if (rd[j]) {
      if constexpr (NT)
        v[j] = dev::nt_load(src);
      else
        v[j] = *src;
    }
  }
  for (int i = tid; i < N; i += NL * TL) stw[i] = tw[i];
  dev::fft_column_regs<T, N>(stw, sm, col, t, v, swz);
  if (!live) return;
  int row[8];
  dev::fft_rows<N>(t, row);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int m = dev::sgn_mode(row[q], N);
    if (qline + m * m < qstore) {
      T2* dst = &data[base + (row[q] >> 3) * hi + (row[q] & 7) * lo];
      if constexpr (NT)
        dev::nt_store(dst, v[q]);
      else
        *dst = v[q];
    }
  }
}

template <typename T, int N, int NL>
constexpr bool zb_ok() {
  using T2 = typename V2<T>::type;
  return NL * (N / 8) <= 1024 && static_cast<size_t>(NL + 1) * N * sizeof(T2) <= 160 * 1024;
}

template <typename T, int N, int NL, bool ALONG>
hipError_t fft_zb_launch(void* mesh, const void* tw, int axis, const FftPrune& pr, int streaming, hipStream_t st) {
  // (the streaming choice is a template parameter: one access path per
  // kernel keeps the register count, and two workgroups per CU)
  if constexpr (!zb_ok<T, N, NL>()) {
    return hipErrorInvalidValue;
  } else {
    using T2 = typename V2<T>::type;
    const unsigned grid = static_cast<unsigned>(static_cast<int64_t>(N) * N / NL);
    if (streaming)
      fft_zb_kernel<T, N, NL, ALONG, true><<<grid, NL * (N / 8), 0, st>>>(static_cast<T2*>(mesh), axis,
                                                                          static_cast<const T2*>(tw), pr);
    else
      fft_zb_kernel<T, N, NL, ALONG, false><<<grid, NL * (N / 8), 0, st>>>(static_cast<T2*>(mesh), axis,
                                                                           static_cast<const T2*>(tw), pr);
    return hipGetLastError();
  }
}

template <typename T, int N>
hipError_t fft_zb_n(void* mesh, const void* tw, int axis, const FftPrune& pr, int lines, int streaming,
                    hipStream_t st) {
  if (lines <= 0) lines = zb_default_lines(N, sizeof(T) == 8, axis);
  if (lines == 8)
    return axis == 0 ? fft_zb_launch<T, N, 8, true>(mesh, tw, axis, pr, streaming, st)
                     : fft_zb_launch<T, N, 8, false>(mesh, tw, axis, pr, streaming, st);
  if (lines == 16)
    return axis == 0 ? fft_zb_launch<T, N, 16, true>(mesh, tw, axis, pr, streaming, st)
                     : fft_zb_launch<T, N, 16, false>(mesh, tw, axis, pr, streaming, st);
  return hipErrorInvalidValue;
}

// Lines per workgroup that a pass supports: at most 1024 threads (N/8 per line),
// at most N columns for the strided passes, and LDS for the lines and twiddles.
template <typename T, int N, int NCOL, bool ALONG>
constexpr bool lines_ok() {
  using T2 = typename V2<T>::type;
  return NCOL * (N / 8) <= 1024 && (ALONG || NCOL <= N) &&
         static_cast<size_t>(NCOL + 1) * N * sizeof(T2) <= 160 * 1024;
}

template <typename T, int N, int NCOL, bool ALONG>
hipError_t fft_axis_launch(void* mesh, const void* tw, int axis, const FftPrune& pr, hipStream_t st) {
  if constexpr (!lines_ok<T, N, NCOL, ALONG>()) {
    return hipErrorInvalidValue;
  } else {
    using T2 = typename V2<T>::type;
    const unsigned grid = ALONG ? static_cast<unsigned>(static_cast<int64_t>(N) * N / NCOL)
                                : static_cast<unsigned>(static_cast<int64_t>(N / NCOL) * N);
    fft_axis_kernel<T, N, NCOL, ALONG><<<grid, NCOL * (N / 8), 0, st>>>(static_cast<T2*>(mesh), axis,
                                                                         static_cast<const T2*>(tw), pr);
    return hipGetLastError();
  }
}

template <typename T, int N, bool ALONG>
hipError_t fft_axis_lines(void* mesh, const void* tw, int axis, const FftPrune& pr, int lines, hipStream_t st) {
  switch (lines) {
    case 1: return fft_axis_launch<T, N, 1, ALONG>(mesh, tw, axis, pr, st);
    case 2: return fft_axis_launch<T, N, 2, ALONG>(mesh, tw, axis, pr, st);
    case 4: return fft_axis_launch<T, N, 4, ALONG>(mesh, tw, axis, pr, st);
    case 8: return fft_axis_launch<T, N, 8, ALONG>(mesh, tw, axis, pr, st);
    case 16: return fft_axis_launch<T, N, 16, ALONG>(mesh, tw, axis, pr, st);
    case 32: return fft_axis_launch<T, N, 32, ALONG>(mesh, tw, axis, pr, st);
    case 64: return fft_axis_launch<T, N, 64, ALONG>(mesh, tw, axis, pr, st);
    case 128: return fft_axis_launch<T, N, 128, ALONG>(mesh, tw, axis, pr, st);
    case 256: return fft_axis_launch<T, N, 256, ALONG>(mesh, tw, axis, pr, st);
    case 512: return fft_axis_launch<T, N, 512, ALONG>(mesh, tw, axis, pr, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N>
hipError_t fft_axis_n(void* mesh, const void* tw, int axis, const FftPrune& pr, int lines, hipStream_t st) {
  if (lines <= 0) lines = fft_default_lines(N, sizeof(T) == 8, axis);
  return axis == 0 ? fft_axis_lines<T, N, true>(mesh, tw, axis, pr, lines, st)
                   : fft_axis_lines<T, N, false>(mesh, tw, axis, pr, lines, st);
}

}  // namespace

int fft_default_lines(int N, bool fp64, int axis) {
  if (axis == 0) return std::max(1, 256 / (N / 8));  // 256 threads
  return std::min(N, (fp64 ? 4096 : 8192) / N);      // 64 KB of lines in LDS
}

bool fft_lines_supported(int N, bool fp64, int axis, int lines) {
  if (lines < 1 || (lines & (lines - 1)) != 0) return false;
  const int threads = lines * (N / 8);
  const size_t lds = static_cast<size_t>(lines + 1) * N * (fp64 ? 16 : 8);
  return threads <= 1024 && (axis == 0 || lines <= N) && lds <= 160 * 1024;
}

template <typename T>
hipError_t launch_fft_axis(void* mesh, int N, const void* tw, int axis, const FftPrune& pr, hipStream_t st,
                           int lines) {
  if (lines > 0 && !fft_lines_supported(N, sizeof(T) == 8, axis, lines)) return hipErrorInvalidValue;
  switch (N) {
    case 16:
      return fft_axis_n<T, 16>(mesh, tw, axis, pr, lines, st);
    case 32:
      return fft_axis_n<T, 32>(mesh, tw, axis, pr, lines, st);
    case 64:
      return fft_axis_n<T, 64>(mesh, tw, axis, pr, lines, st);
    case 128:
      return fft_axis_n<T, 128>(mesh, tw, axis, pr, lines, st);
    case 256:
      return fft_axis_n<T, 256>(mesh, tw, axis, pr, lines, st);
    case 512:
      return fft_axis_n<T, 512>(mesh, tw, axis, pr, lines, st);
    case 1024:
      return fft_axis_n<T, 1024>(mesh, tw, axis, pr, lines, st);
    default:
      return hipErrorInvalidValue;
  }
}

// x pass 8 lines (8 z-values of one row y); y pass 16 in FP32 up to N = 512
// (two columns x: 128-byte runs), else 8; z pass 8 (runs of 8 x-columns of
// 64 bytes each are already 512 contiguous bytes, and 8 lines leave four
// workgroups per CU instead of two).
int zb_default_lines(int N, bool fp64, int axis) {
  if (axis != 1 || fp64) return 8;
  return N <= 512 ? 16 : 8;
}

bool zb_lines_supported(int N, bool fp64, int axis, int lines) {
  (void)axis;
  if (lines != 8 && lines != 16) return false;
  const size_t lds = static_cast<size_t>(lines + 1) * N * (fp64 ? 16 : 8);
  return lines * (N / 8) <= 1024 && lds <= 160 * 1024;
}

// Non-temporal accesses pay off in a pass whose lines are read as runs of at
// least 128 contiguous bytes (an L2 line): the x and z passes always, the y
// pass when a workgroup holds two columns x (FP32, 16 lines) or runs of
// 16-byte FP64 values.  With 64-byte runs the other half of each L2 line
// belongs to the neighbouring workgroup, and the streaming hint lets it be
// evicted before that workgroup reads it.  A mesh of at most 256 MiB (256^3
// in FP32) stays in the Infinity Cache from one pass to the next if the x
// and y passes do not stream: only the z pass, whose output the shell sums
// read once, streams there (a 256^3 estimate 8.7 % faster).
int zb_default_streaming(int N, bool fp64, int lines_y) {
  if (static_cast<int64_t>(N) * N * N * (fp64 ? 16 : 8) <= (int64_t{256} << 20)) return 4;
  if (lines_y <= 0) lines_y = zb_default_lines(N, fp64, 1);
  const int run = (lines_y / 8) * 8 * (fp64 ? 16 : 8);
  return 1 | 4 | (run >= 128 ? 2 : 0);
}

template <typename T>
hipError_t launch_fft_axis_zb(void* mesh, int N, const void* tw, int axis, const FftPrune& pr, hipStream_t st,
                              int lines, int streaming) {
  if (lines > 0 && !zb_lines_supported(N, sizeof(T) == 8, axis, lines)) return hipErrorInvalidValue;
  if (streaming < 0) streaming = zb_default_streaming(N, sizeof(T) == 8, axis == 1 ? lines : 0);
  const int nt = (streaming >> axis) & 1;
  switch (N) {
    case 16:
      return fft_zb_n<T, 16>(mesh, tw, axis, pr, lines, nt, st);
    case 32:
      return fft_zb_n<T, 32>(mesh, tw, axis, pr, lines, nt, st);
    case 64:
      return fft_zb_n<T, 64>(mesh, tw, axis, pr, lines, nt, st);
    case 128:
      return fft_zb_n<T, 128>(mesh, tw, axis, pr, lines, nt, st);
    case 256:
      return fft_zb_n<T, 256>(mesh, tw, axis, pr, lines, nt, st);
    case 512:
      return fft_zb_n<T, 512>(mesh, tw, axis, pr, lines, nt, st);
    case 1024:
      return fft_zb_n<T, 1024>(mesh, tw, axis, pr, lines, nt, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_fft3d(void* mesh, int N, const void* tw, hipStream_t st) {
  const FftPrune full{nullptr, nullptr, nullptr, INT_MAX};
  for (int axis = 0; axis < 3; ++axis) {
    const hipError_t e = launch_fft_axis<T>(mesh, N, tw, axis, full, st, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_fft3d<float>(void*, int, const void*, hipStream_t);
template hipError_t launch_fft_axis<float>(void*, int, const void*, int, const FftPrune&, hipStream_t, int);
template hipError_t launch_fft_axis<double>(void*, int, const void*, int, const FftPrune&, hipStream_t, int);
template hipError_t launch_fft_axis_zb<float>(void*, int, const void*, int, const FftPrune&, hipStream_t, int, int);
template hipError_t launch_fft_axis_zb<double>(void*, int, const void*, int, const FftPrune&, hipStream_t, int, int);
template hipError_t launch_fft3d<double>(void*, int, const void*, hipStream_t);

}  // namespace lpp
