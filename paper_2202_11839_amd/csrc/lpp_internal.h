// Internal declarations shared by the host orchestration and the HIP kernels
// of liblpp.  Nothing here crosses the C ABI (include/lpp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lpp.h"

namespace lpp {

// ---------------------------------------------------------------------------
// Line-of-sight weights of one FFT field.
//
// The LPP kernels of the estimators are (k.m)^s d^s L_L/dmu^s (k.xhat) with
// m = e_theta - i e_phi, i.e. exp(-i s phi_{k,x}) L^s_L(k.xhat) (Sec. III.A,
// eqs. def_of_Xiij and def_of_Xiijkl; s = 0 for the Legendre moments).  By
// the rotation identity of App. E (eq. spherical_harmonics_identity) this is,
// as a function of khat, a degree-L spherical harmonic, and it factorises
// exactly as
//
//   sum_a kappa_a h_a(khat) * s! [t^s] h_a(xhat + t m)
//
// over the 2L+1 real harmonic polynomials h_{L,M,cos|sin}(y) =
// Q_{LM}(y_z) Re|Im (y_x + i y_y)^M with Q_{LM} = d^M L_L/dz^M, kappa_{L0} = 1,
// kappa_{LM} = 2 (L-M)!/(L+M)! (the Legendre addition theorem, eq.
// spherical_hamornics_hand), because y = xhat + t m stays on the complex unit
// sphere y.y = 1.  The t-expansion has the closed form used by the deposit
// kernel: with c = cos(theta), s = sin(theta),
//   y_x + i y_y = e^{i phi} (s + t (1+c)),  y_x - i y_y = e^{-i phi} (s - t (1-c)),
//   y_z = c - t s.
// One FFT field per (s, L, M, cos|sin): 2L+1 fields per (s, L).
struct FieldSpec {
  int32_t s, L, M, cs;     // spin 0/2/4, degree, order, 0 = cos part, 1 = sin part
  int32_t nq[5];           // number of coefficients in q[j]
  double q[5][9];          // (-1)^j / j! d^{M+j} L_L / dz^{M+j}, power basis, j = 0..s
  double binom[5];         // binom(M, s - j)
  double scale;            // kappa_{LM} * s!
};

// A FieldSpec in the deposit's precision, as the kernels read it (kernel
// arguments, or a device table for the node-parallel deposit).
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

// Family of a field and the series it accumulates into.
enum Family { FAM_DD = 0, FAM_GD = 1, FAM_PLUS = 2, FAM_MINUS = 3 };

struct Field {
  Family fam;
  int series;              // index into the accumulator series
  FieldSpec spec;
};

// Host tables built once per plan.
struct Tables {
  std::vector<std::string> series;   // output series names (incl. EE/BB)
  std::vector<int> acc_series;       // for each accumulated series: family
  std::vector<int> acc_L;            // and multipole
  std::vector<int> series_of_acc;    // output index of each accumulated series
  std::vector<Field> fields;         // all fields with L > 0 (bases are separate)
  std::vector<int64_t> thr;          // thresholds T_0..T_nb
  int dd0 = -1, plus0 = -1;          // accumulator index of DD_l0 and PLUS_l0
};

bool build_tables(const lpp_config& cfg, Tables& t);
FieldSpec make_spec(int s, int L, int M, int cs);
double prefactor(int m, int L);                 // (2L+1)(L-m)!/(L+m)!
double cmap_minus_to_legendre(int l, int L);    // (2l+1) int dmu/2 L^4_L L_l

// ---------------------------------------------------------------------------
// Cell-sorted objects for the gather deposit: the cell and the position in
// it as one aligned record (one access to store or load), the weights as
// separate columns.
template <typename T>
struct __align__(4 * sizeof(T)) ObjPos {
  uint32_t key;            // cell index cx + N (cy + N cz)
  T fx, fy, fz;            // fractional position in the cell, [0, 1)
};

template <typename T>
struct GObjSet {
  ObjPos<T>* pos;          // one 16-byte (FP32) or 32-byte (FP64) record per object
  T* wr;                   // weight (density set) or w*g1 (shape set)
  T* wi;                   // w*g2 (shape set), unused for the density set
  int64_t n;
};

// Raw catalog columns on the device, in their own dtype.
struct RawCat {
  const void* x;
  const void* y;
  const void* z;
  const void* w;
  const void* nbar;
  const void* g1;
  const void* g2;
  int64_t n;
  int dtype;
};

struct Geometry {
  int N;
  int p;                   // assignment order
  int interlace;
  double H;
  double origin[3];
  double rel[3];           // origin - observer
  double box;
  // line of sight of node c + f: los_rel + (c + f) los_h.  The object's own
  // direction (los_h = H, los_rel = rel), or one global direction (los_h = 0,
  // los_rel = the unit line of sight)
  int global_los;
  double los_h;
  double los_rel[3];
};

// ---- mesh layouts ----
// The public entry points take meshes in the plain order x + N (y + N z).
// The estimator's own meshes (deposits, transforms, bases) are z-blocked:
// node or mode (x, y, z) sits at ((z/8 N + y) N + x) 8 + z%8, so the 8 z of
// one (x, y) are contiguous and so are those groups for consecutive x.  Every
// pass of the 3D transform then reads and writes runs of 8 z-values x the
// lines it owns, and a z-column touches N/8 memory pages instead of N.
constexpr int kZb = 8;
__host__ __device__ inline int64_t zb_index(int x, int y, int z, int N) {
  return ((static_cast<int64_t>(z >> 3) * N + y) * N + x) * kZb + (z & 7);
}

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// FP64 sums over a catalog: [0] sum w, [1] sum w^2, [2] sum w^2 nbar, [3] sum w^2 |g|^2,
// [4] count of non-finite, [5] out of box, [6] at observer (as doubles).
hipError_t launch_catalog_sums(const RawCat& c, const Geometry& g, double nbar_default, double* partial,
                               int nblocks, double* out, hipStream_t st);
int catalog_sum_blocks();

// Counting sort by mesh cell and the gather deposit (kernels_gather.hip).
int64_t scan_block_count(int64_t n);
hipError_t launch_cell_count(const RawCat& c, const Geometry& g, uint32_t* counts, uint32_t* rank,
                             uint32_t* cell_of_obj, hipStream_t st);
// exclusive scan of n counts into starts[0..n]; bsum needs scan_block_count(n)+1 entries;
// counts and starts may alias
hipError_t launch_big_scan(const uint32_t* counts, int64_t n, uint32_t* bsum, uint32_t* starts, hipStream_t st);
template <typename T>
// The density weight of each object is w * wscale * (*wscale_dev) (wscale_dev nullable).
hipError_t launch_cell_scatter(const RawCat& c, const Geometry& g, double wscale, const double* wscale_dev, int shape,
                               const uint32_t* starts, const uint32_t* rank, const uint32_t* cell_of_obj,
                               GObjSet<T> out, uint32_t* order, int64_t index_base, hipStream_t st);
// Puts the objects of every cell in the order of their index in the set
// (order[d]: that index, written by the scatter as index_base + i).
template <typename T>
hipError_t launch_cell_order(const uint32_t* starts, int64_t ncell, uint32_t* order, GObjSet<T> out, int shape,
                             hipStream_t st);
// Footprint of a cell-sorted object set, as 0/1 byte flags (nt = N / kTile):
//   row[y + N z]      node row (y, z) can receive weight: some object lies in
//                     cells y-2..y+1, z-2..z+1 (the reach of every window
//                     on both grids), any x;
//   tile[ty + nt tz]  some node row of the kTile x kTile tile-row is flagged;
//   plane[z]          some node row of plane z is flagged;
//   cube[tx + nt (ty + nt tz)]  the kTile^3 tile can receive weight: some
//                     object lies in its cells t0-2 .. t0+kTile on every axis.
// Nodes outside the flagged rows or cubes are zero in every field of the set.
constexpr int kTile = 8;
struct Footprint {
  uint8_t* row;
  uint8_t* tile;
  uint8_t* plane;
  uint8_t* cube;
};
inline size_t footprint_bytes(int N) {
  const size_t n = static_cast<size_t>(N), nt = n / kTile;
  return n * n + nt * nt + n + nt * nt * nt;
}
hipError_t launch_footprint(const uint32_t* cell_start, int N, Footprint fp, hipStream_t st);

// Deposits nf real (density) fields of one object set in one pass and
// writes every node of each output mesh (no clearing needed), z-blocked or
// (zblocked = false) plain.  With tile_flags (the footprint's cube flags) the
// tiles that are not flagged are skipped and left unwritten.  nf <=
// kGatherMaxReal (kGatherMaxRealF64 in FP64): mesh q holds field q packed
// (grid -> real part, interlaced grid -> imaginary part).
constexpr int kGatherMaxReal = 8;
constexpr int kGatherMaxRealF64 = 8;
// complex (shape) fields per pass of the node-parallel deposit (FP32, FP64)
constexpr int kNodeFields = 10;
constexpr int kNodeFieldsF64 = 4;
template <typename T>
hipError_t launch_gather(const GObjSet<T>& o, const uint32_t* cell_start, const Geometry& g, const FieldSpec* specs,
                         int nf, void* const* meshes, const uint8_t* tile_flags, bool zblocked, hipStream_t st);
// Deposits nf complex (shape) fields, nf <= kNodeFields (kNodeFieldsF64 in
// FP64), with one thread per node of each 8^3 tile: with interlacing mesh 2q
// holds field q on the grid and mesh 2q+1 on the interlaced grid, without
// it mesh q holds field q; the fields' specs are read from the device table
// `specs` (nf entries).
hipError_t launch_gather_nodes(const GObjSet<float>& o, const uint32_t* cell_start, const Geometry& g,
                               const SpecT<float>* specs, int nf, void* const* meshes, const uint8_t* tile_flags,
                               bool zblocked, hipStream_t st);
hipError_t launch_gather_nodes(const GObjSet<double>& o, const uint32_t* cell_start, const Geometry& g,
                               const SpecT<double>* specs, int nf, void* const* meshes,
                               const uint8_t* tile_flags, bool zblocked, hipStream_t st);

// plain-layout 3D transform (the public entry point)
template <typename T>
hipError_t launch_fft3d(void* mesh, int N, const void* twiddles, hipStream_t st);
// Pruning of the 3D transform of a field with a known footprint, keeping only
// the modes the binning reads.  row/plane: footprint flags (nullable); input
// rows that are not flagged are taken as zero and never read.  The x pass
// leaves unflagged rows unwritten, the y pass unflagged planes and the
// (kx, ky) with nx^2 + ny^2 >= qmax, and the z pass the modes with
// |n|^2 >= qmax: the result is exact at every mode with |n|^2 < qmax and
// undefined elsewhere (without pruning, qmax = INT_MAX, everywhere exact).
struct FftPrune {
  const uint8_t* row;
  const uint8_t* plane;
  const uint8_t* cube;  // x pass: kTile-node segments of a row outside the flagged cubes are zero
  int qmax;
};
// one axis (0: x, unit stride; 1: y; 2: z) of the 3D transform; lines: lines
// per workgroup (x rows, or y / z columns), 0 = fft_default_lines
template <typename T>
hipError_t launch_fft_axis(void* mesh, int N, const void* twiddles, int axis, const FftPrune& pr, hipStream_t st,
                           int lines);
int fft_default_lines(int N, bool fp64, int axis);
bool fft_lines_supported(int N, bool fp64, int axis, int lines);
// The same passes on a z-blocked mesh.  lines per workgroup, 8 or 16 (0 =
// zb_default_lines): x pass, 8 z-values of 1 or 2 rows y; y pass, 8 z-values
// of 1 or 2 columns x; z pass, 8 or 16 columns x of one row y.
// streaming: bit a set = non-temporal loads and stores in pass a (x, y, z);
// < 0 = zb_default_streaming(N, fp64, lines of the y pass)
template <typename T>
hipError_t launch_fft_axis_zb(void* mesh, int N, const void* twiddles, int axis, const FftPrune& pr, hipStream_t st,
                              int lines, int streaming);
int zb_default_lines(int N, bool fp64, int axis);
int zb_default_streaming(int N, bool fp64, int lines_y);
bool zb_lines_supported(int N, bool fp64, int axis, int lines);

// Binning.  Tables: twiddles (N complex, exp(-2 pi i m/N)), phase (3N+1
// complex, exp(-i pi m/N) for m = -3N/2..3N/2), invw (N reals, 1/W_1(n)).
// largest number of k-shells a plan may ask for
constexpr int kMaxShells = 256;

struct BinArgs {
  int N, nb, interlace, compensate;
  const int64_t* thr;      // device thresholds [nb+1]
  const void* phase;
  const void* invw;
  double* partial;         // column-major [width][nblocks]
  int nblocks;
  int qmax;                // thr[nb] (host copy): the density kernels need qmax <= (N/2)^2
};
// The binning kernels read the transformed (z-blocked) fields only at modes
// inside the last shell, |n|^2 < T_nb, and the base kernels write the base
// only there.
int bin_blocks(int N);            // default workgroups of the shell-sum kernels
// workgroups of the density kernels (column pairs) for a budget of nblocks:
// at most one per 256 column-pair chunks
int pair_bin_blocks(int N, int nblocks);
constexpr int kMaxBinBlocks = 8192;
// the density kernels (launch_base_dd, launch_bin_dd) run a.nblocks
// workgroups: pass pair_bin_blocks(N, budget) there and to the reduction
template <typename T>
hipError_t launch_base_dd(const BinArgs& a, const void* packed, void* base, hipStream_t st);
template <typename T>
hipError_t launch_base_gg(const BinArgs& a, const void* g1, const void* g2, void* base, hipStream_t st);
// n <= kBinGroup fields of one gather pass against the same base: field i
// with harmonic f[i], rows [re, im] of width nb at 2i nb of the partial rows
// (width 2 n nb).  kind 0: G conj(B(k)) (plus / cross), 1: G B(-k) (minus);
// g2 nullable without interlacing.
constexpr int kBinGroup = 4;
constexpr int kBinGroupMax = 5;  // FP32 shape fields
// fields per shell-sum launch: kBinGroupMax for FP32 shape fields, else
// kBinGroup, fewer when 2 n nb sums per wavefront would not fit the LDS rows
int bin_group_max(bool complex_fields, bool fp64, int nb);
// The z pass of a group of complex fields fused with their shell sums
// (kernels_bin.hip): g1/g2 after the x and y passes of fft_zb_kernel, plane =
// the footprint's z-plane flags (nullable).  zbin_group_max: the most fields
// per launch whose LDS fits one CU (0: the fused kernel cannot take nb shells
// at this N).
int zbin_group_max(int N, bool fp64, int nb);
int zbin_blocks(int N, bool fp64, int nblocks);  // its workgroups (partial rows) for a budget of nblocks
template <typename T>
hipError_t launch_zbin_gg(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2,
                          int n, const void* base, int kind, const void* tw, const uint8_t* plane, hipStream_t st);
template <typename T>
hipError_t launch_bin_gg(const BinArgs& a, const FieldSpec* const* f, const void* const* g1, const void* const* g2,
                         int n, const void* base, int kind, hipStream_t st);
template <typename T>
hipError_t launch_bin_dd(const BinArgs& a, const FieldSpec* const* f, const void* const* packed, int n,
                         const void* base, hipStream_t st);
// Window multipoles (kernels_window.hip), on z-blocked meshes.  Shells of the
// separation r in cells: T_b <= |n|^2 < T_{b+1} (thr on the device).
struct WinArgs {
  int N, nb, interlace, n_rows;  // n_rows = multipoles + 2 (counts, |n| sums)
  const int64_t* thr;
  const void* phase;
  const void* invw;
};
constexpr int kWinMaxRows = 7;
int window_bin_blocks(int N);
// slot < 0: B0 = F_0 from the packed copies; 0: Zc = F_a conj(B0); 1: Zc -= i F_b conj(B0) conj'd (see source)
template <typename T>
hipError_t launch_window_product(const WinArgs& a, const void* packed, void* B0, void* Zc, int slot, hipStream_t st);
// per-block partial rows [n_rows * nb][window_bin_blocks(N)] of the shell sums of D = DFT[conj Z]
template <typename T>
hipError_t launch_window_bin(const WinArgs& a, const void* D, const FieldSpec* fa, const FieldSpec* fb, int row_a,
                             int row_b, int with_counts, double* partial, hipStream_t st);

// acc[0..width) += sum over blocks of partial, laid out [width][nblocks] (fixed order)
hipError_t launch_reduce_partials(const double* partial, int nblocks, int width, double* acc, hipStream_t st);
// n such reductions in one launch: columns [i width, (i + 1) width) of the
// partial rows are added to acc[i], in the order i = 0 .. n-1 (rows acc[i]
// may coincide; n <= kBinGroupMax)
hipError_t launch_reduce_partials_group(const double* partial, int nblocks, int width, int n, double* const* acc,
                                        hipStream_t st);

}  // namespace lpp
