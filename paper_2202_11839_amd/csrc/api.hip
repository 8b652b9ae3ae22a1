// C ABI of liblpp (include/lpp.h): plan validation, workspace, catalog
// staging and the per-estimate pipeline
//
//   FP64 catalog sums (alpha, I, shot noise, input checks)
//   -> counting sort by mesh cell of the density set (galaxies and randoms,
//      weights w and -alpha w) and of the shape set (galaxies, w*gamma)
//   -> density base: gather deposit, FFT, unpack/combine -> B_delta, DD_l0
//   -> shape base:   deposit (both grids), FFT, combine -> B_gamma, PLUS_l0
//   -> every other field: deposit, FFT, multiply by its harmonic and by the
//      base, FP64 shell sums
//   -> prefactors, normalisation, shot noise and the E/B map on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lpp_internal.h"

using namespace lpp;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int64_t igcd(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

struct lpp_plan_s {
  lpp_config cfg{};
  Tables tab;
  Geometry geo{};
  hipStream_t stream = nullptr;
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  int64_t cap_gal = 0, cap_ran = 0;
  // small tables owned by the plan
  void* tabs = nullptr;
  int64_t* d_thr = nullptr;
  void* d_tw = nullptr;
  void* d_phase = nullptr;
  void* d_invw = nullptr;
  // FP32 specs of the shape set's fields in pass order (the node-parallel deposit)
  const SpecT<float>* d_spec = nullptr;     // shape fields in deposit order (node-parallel deposit), FP32
  const SpecT<double>* d_spec64 = nullptr;  // ... and FP64
  int device = -1;
  // per-stage timing with HIP events on the plan's stream
  bool prof_on = false;
  std::vector<hipEvent_t> ev;     // pairs (start, stop)
  std::vector<int> ev_stage;      // stage of each pair
  std::vector<int> ev_launch;     // kernel launches inside each pair
  size_t ev_used = 0;             // pairs recorded since the last collection
  double prof_ms[LPP_N_STAGES] = {0};
  int64_t prof_launches[LPP_N_STAGES] = {0};
  // batch executor: the device pipelines of a batch of device-resident
  // catalogs captured into one HIP graph, replayed while the batch's
  // pointers and sizes stay the same
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  double* d_batch = nullptr;  // alpha[n], then n rows of acc_doubles
  size_t d_batch_cap = 0;     // doubles
  int64_t graph_captures = 0, graph_replays = 0;
  lpp_tuning tune{};  // 0 = default
  // the deposit of the next gather pass runs on a second stream while the
  // transforms and shell sums of the current one run on the plan's stream
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_dep[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
};

namespace {

// the second stream and the events that order the two streams (created once)
hipError_t ensure_aux(lpp_plan_s* p) {
  if (p->aux) return hipSuccess;
  hipError_t e = hipSuccess;
  auto ev = [&](hipEvent_t* x) {
    if (e == hipSuccess) e = hipEventCreateWithFlags(x, hipEventDisableTiming);
  };
  ev(&p->ev_fork);
  for (int i = 0; i < 2; ++i) {
    ev(&p->ev_dep[i]);
    ev(&p->ev_done[i]);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking);
  return e;
}

hipError_t prof_begin(lpp_plan_s* p) {
  if (!p->prof_on) return hipSuccess;
  if (2 * (p->ev_used + 1) > p->ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      p->ev.push_back(e);
    }
    p->ev_stage.push_back(0);
    p->ev_launch.push_back(0);
  }
  return hipEventRecord(p->ev[2 * p->ev_used], p->stream);
}

hipError_t prof_end(lpp_plan_s* p, int stage, int launches) {
  if (!p->prof_on) return hipSuccess;
  p->ev_stage[p->ev_used] = stage;
  p->ev_launch[p->ev_used] = launches;
  const hipError_t r = hipEventRecord(p->ev[2 * p->ev_used + 1], p->stream);
  ++p->ev_used;
  return r;
}

// after the stream has synchronised
void prof_collect(lpp_plan_s* p) {
  for (size_t i = 0; i < p->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) == hipSuccess) {
      p->prof_ms[p->ev_stage[i]] += ms;
      p->prof_launches[p->ev_stage[i]] += p->ev_launch[i];
    }
  }
  p->ev_used = 0;
}

size_t real_size(const lpp_plan_s* p) { return p->cfg.precision == LPP_F64 ? 8 : 4; }
size_t mesh_bytes(const lpp_plan_s* p) {
  const size_t n = static_cast<size_t>(p->cfg.mesh_n);
  return n * n * n * 2 * real_size(p);
}
bool need_density(const lpp_plan_s* p) { return (p->cfg.spectra & (LPP_DD | LPP_GD)) != 0; }
bool need_shape(const lpp_plan_s* p) { return (p->cfg.spectra & (LPP_GD | LPP_PLUS | LPP_MINUS)) != 0; }
int n_acc(const lpp_plan_s* p) { return static_cast<int>(p->tab.acc_series.size()); }

// Work meshes: one gather pass deposits up to kGatherMaxReal density fields
// (one packed mesh each, the row kernel) or the shape fields of one pass
// (one mesh per grid, the node-parallel kernel) into one of two sets of
// work meshes: FP32 up to N = 512 sets of kWork (kNodeFields shape fields
// per pass; 42 meshes of 1.07 GB at 512^3, which at 1024^3 would not fit
// the device), otherwise sets of kWorkRow (four shape fields per pass),
// and FP64 at N >= 1024 sets of kWorkF64Large (two sets of eight 17 GB
// meshes and the bases would not fit the device: at most four density and
// two shape fields per pass).
constexpr int kWorkRow = 8;
constexpr int kWork = 2 * kNodeFields;
constexpr int kWorkF64Large = 4;
static_assert(kWorkRow >= kGatherMaxReal && kWorkRow >= 2 * kNodeFieldsF64, "work meshes per gather pass");
static_assert(kWorkRow >= kGatherMaxRealF64, "work meshes per gather pass");
static_assert(kWork >= kWorkRow, "work mesh slots");
int work_meshes(const lpp_plan_s* p) {
  if (p->cfg.precision == LPP_F32 && p->cfg.mesh_n <= 512) return kWork;
  return (p->cfg.precision == LPP_F64 && p->cfg.mesh_n >= 1024) ? kWorkF64Large : kWorkRow;
}
int max_density_fields(const lpp_plan_s* p) {
  return std::min(p->cfg.precision == LPP_F64 ? kGatherMaxRealF64 : kGatherMaxReal, work_meshes(p));
}
// The fields of the shape set in the order the passes deposit them: the
// set's base (spin 0, L = 0) first, then its other fields in table order.
std::vector<FieldSpec> shape_specs(const lpp_plan_s* p) {
  std::vector<FieldSpec> out;
  if (p->cfg.spectra & (LPP_PLUS | LPP_MINUS)) out.push_back(make_spec(0, 0, 0, 0));
  for (const Field& f : p->tab.fields)
    if (f.fam != FAM_DD) out.push_back(f.spec);
  return out;
}
int max_shape_fields(const lpp_plan_s* p) {
  return std::min(p->cfg.precision == LPP_F64 ? kNodeFieldsF64 : kNodeFields, work_meshes(p) / 2);
}
lpp_tuning resolved_tuning(const lpp_plan_s* p);  // launch shapes with the defaults filled in
// passes of the 3D transform with non-temporal accesses (bit a for pass a), -1 = default
int streaming(const lpp_plan_s* p) { return p->tune.fft_streaming > 0 ? (p->tune.fft_streaming & 7) : -1; }
// Workspace layout (offsets in bytes), computed for capacities (ng, nr).
struct Layout {
  size_t mesh[2];  // Bd, Bg
  size_t work[2][kWork];  // two sets: one pass deposits into a set while the other is transformed
  size_t pos_d, wr_d;
  size_t pos_g, wr_g, wi_g;
  size_t cell_of, rank, order, starts_d, starts_g, bsum;
  size_t stage_gal, stage_ran;
  size_t sums_partial, sums_out;
  size_t bin_partial, acc;
  size_t fp[2];  // footprints of the density and the shape set (footprint_bytes)
  size_t rthr, wacc, wpartial;  // window multipoles: r-shell thresholds, rows, per-block partials
  size_t total;
};

Layout layout(const lpp_plan_s* p, int64_t ng, int64_t nr) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t M = mesh_bytes(p), rs = real_size(p);
  const bool dn = need_density(p), sh = need_shape(p);
  const bool il = p->cfg.interlacing != 0;
  // both bases and every work mesh, whatever the spectra: the window
  // multipoles use them too (base, pair accumulator, one gather pass)
  (void)dn;
  (void)il;
  L.mesh[0] = take(M);
  L.mesh[1] = take(M);
  for (int s = 0; s < 2; ++s)
    for (int i = 0; i < work_meshes(p); ++i) L.work[s][i] = take(M);
  const size_t nd = static_cast<size_t>(ng + nr);
  const size_t gg = static_cast<size_t>(ng);
  L.pos_d = take(4 * rs * nd);  // ObjPos<T>: 4 values of the real type
  L.wr_d = take(rs * nd);
  L.pos_g = take(4 * rs * gg);
  L.wr_g = take(rs * gg);
  L.wi_g = take(rs * gg);
  L.cell_of = take(4 * nd);
  L.rank = take(4 * nd);
  L.order = take(4 * nd);
  const size_t ncell = static_cast<size_t>(p->cfg.mesh_n) * p->cfg.mesh_n * p->cfg.mesh_n;
  L.starts_d = take(4 * (ncell + 1));  // also used by lpp_deposit_weights
  L.starts_g = sh ? take(4 * (ncell + 1)) : 0;
  L.bsum = take(4 * (static_cast<size_t>(scan_block_count(static_cast<int64_t>(ncell))) + 1));
  L.stage_gal = take(8 * 7 * gg);
  L.stage_ran = take(8 * 5 * static_cast<size_t>(nr));
  L.sums_partial = take(8 * 8 * static_cast<size_t>(catalog_sum_blocks()));
  L.sums_out = take(8 * 16);
  const int nb = p->cfg.n_kbins;
  L.bin_partial = take(8 * std::max(4, 2 * kBinGroupMax) * static_cast<size_t>(nb) *
                       std::max(bin_blocks(p->cfg.mesh_n), kMaxBinBlocks));
  L.acc = take(8 * (2 * static_cast<size_t>(nb) * n_acc(p) + 8 * static_cast<size_t>(nb)));
  for (int i = 0; i < 2; ++i) L.fp[i] = take(footprint_bytes(p->cfg.mesh_n));
  L.rthr = take(8 * (kMaxShells + 1));
  L.wacc = take(8 * static_cast<size_t>(kWinMaxRows) * kMaxShells);
  L.wpartial = take(8 * static_cast<size_t>(kWinMaxRows) * kMaxShells * window_bin_blocks(p->cfg.mesh_n));
  L.total = off;
  return L;
}

char* wsp(lpp_plan_s* p, size_t off) { return static_cast<char*>(p->ws) + off; }

Footprint footprint_at(lpp_plan_s* p, size_t off) {
  const size_t nn = static_cast<size_t>(p->cfg.mesh_n), nt = nn / kTile;
  uint8_t* b = reinterpret_cast<uint8_t*>(wsp(p, off));
  return Footprint{b, b + nn * nn, b + nn * nn + nt * nt, b + nn * nn + nt * nt + nn};
}

lpp_status hip_status(hipError_t e) {
  if (e == hipSuccess) return LPP_OK;
  if (e == hipErrorOutOfMemory) return LPP_E_NOMEM;
  return LPP_E_DEVICE;
}

#define LPP_TRY(expr)                         \
  do {                                        \
    const hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) return hip_status(e_); \
  } while (0)

lpp_status ensure_device(lpp_plan_s* p) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return LPP_E_DEVICE;
  if (p->device < 0) {
    int d = 0;
    LPP_TRY(hipGetDevice(&d));
    p->device = d;
  }
  return LPP_OK;
}

lpp_status ensure_tables(lpp_plan_s* p) {
  lpp_status s = ensure_device(p);
  if (s != LPP_OK) return s;
  if (p->tabs) return LPP_OK;
  const int N = p->cfg.mesh_n, nb = p->cfg.n_kbins;
  const size_t rs = real_size(p);
  const size_t o_thr = 0;
  const size_t o_tw = align_up(8 * (nb + 1));
  const size_t o_ph = o_tw + align_up(2 * rs * N);
  const size_t o_iw = o_ph + align_up(2 * rs * (3 * N + 1));
  const std::vector<FieldSpec> sg = shape_specs(p);
  const size_t o_sg = o_iw + align_up(rs * N);
  const size_t o_sg64 = o_sg + align_up(sizeof(SpecT<float>) * sg.size());
  const size_t total = o_sg64 + align_up(sizeof(SpecT<double>) * sg.size());
  std::vector<char> host(total, 0);
  std::memcpy(host.data() + o_thr, p->tab.thr.data(), 8 * (nb + 1));
  for (size_t i = 0; i < sg.size(); ++i) {
    const SpecT<float> v = to_spec<float>(sg[i]);
    std::memcpy(host.data() + o_sg + i * sizeof(SpecT<float>), &v, sizeof v);
    const SpecT<double> w = to_spec<double>(sg[i]);
    std::memcpy(host.data() + o_sg64 + i * sizeof(SpecT<double>), &w, sizeof w);
  }
  const int pw = p->cfg.assignment;
  for (int m = 0; m < N; ++m) {
    const double a = -2.0 * M_PI * m / N;
    const int n = m < N / 2 ? m : m - N;
    double w1 = 1.0;
    if (p->cfg.compensate && n != 0) {
      const double x = M_PI * n / N;
      w1 = std::pow(std::sin(x) / x, pw);
    }
    if (rs == 8) {
      double* tw = reinterpret_cast<double*>(host.data() + o_tw);
      tw[2 * m] = std::cos(a);
      tw[2 * m + 1] = std::sin(a);
      reinterpret_cast<double*>(host.data() + o_iw)[m] = 1.0 / w1;
    } else {
      float* tw = reinterpret_cast<float*>(host.data() + o_tw);
      tw[2 * m] = static_cast<float>(std::cos(a));
      tw[2 * m + 1] = static_cast<float>(std::sin(a));
      reinterpret_cast<float*>(host.data() + o_iw)[m] = static_cast<float>(1.0 / w1);
    }
  }
  for (int m = 0; m <= 3 * N; ++m) {
    const double a = -M_PI * (m - 1.5 * N) / N;  // exp(-i pi (nx+ny+nz)/N)
    if (rs == 8) {
      double* ph = reinterpret_cast<double*>(host.data() + o_ph);
      ph[2 * m] = std::cos(a);
      ph[2 * m + 1] = std::sin(a);
    } else {
      float* ph = reinterpret_cast<float*>(host.data() + o_ph);
      ph[2 * m] = static_cast<float>(std::cos(a));
      ph[2 * m + 1] = static_cast<float>(std::sin(a));
    }
  }
  void* d = nullptr;
  LPP_TRY(hipMalloc(&d, total));
  const hipError_t e = hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_status(e);
  }
  p->tabs = d;
  char* c = static_cast<char*>(d);
  p->d_thr = reinterpret_cast<int64_t*>(c + o_thr);
  p->d_tw = c + o_tw;
  p->d_phase = c + o_ph;
  p->d_invw = c + o_iw;
  p->d_spec = reinterpret_cast<const SpecT<float>*>(c + o_sg);
  p->d_spec64 = reinterpret_cast<const SpecT<double>*>(c + o_sg64);
  return LPP_OK;
}

lpp_status ensure_workspace(lpp_plan_s* p, int64_t ng, int64_t nr) {
  const Layout L = layout(p, ng, nr);
  if (p->ws && ng <= p->cap_gal && nr <= p->cap_ran) return LPP_OK;
  if (p->ws && !p->own_ws) {
    // caller workspace: must be large enough for this request
    if (L.total > p->ws_bytes) return LPP_E_WORKSPACE;
    p->cap_gal = ng;
    p->cap_ran = nr;
    return LPP_OK;
  }
  if (p->ws && p->own_ws) {
    (void)hipFree(p->ws);
    p->ws = nullptr;
  }
  void* d = nullptr;
  if (hipMalloc(&d, L.total) != hipSuccess) {
    (void)hipGetLastError();
    return LPP_E_NOMEM;
  }
  p->ws = d;
  p->ws_bytes = L.total;
  p->own_ws = true;
  p->cap_gal = ng;
  p->cap_ran = nr;
  return LPP_OK;
}

// Make a device RawCat for a catalog, staging host columns into the workspace.
lpp_status stage(lpp_plan_s* p, const lpp_catalog* c, size_t stage_off, int ncols_max, RawCat& out) {
  out = RawCat{c->x, c->y, c->z, c->w, c->nbar, c->g1, c->g2, c->n, c->dtype};
  if (c->on_device) return LPP_OK;
  const size_t es = c->dtype == LPP_F64 ? 8 : 4;
  const size_t col = es * static_cast<size_t>(c->n);
  char* base = wsp(p, stage_off);
  const void* src[7] = {c->x, c->y, c->z, c->w, c->nbar, c->g1, c->g2};
  const void** dst[7] = {&out.x, &out.y, &out.z, &out.w, &out.nbar, &out.g1, &out.g2};
  int k = 0;
  for (int i = 0; i < 7; ++i) {
    if (!src[i]) {
      *dst[i] = nullptr;
      continue;
    }
    if (k >= ncols_max) return LPP_E_INVALID;
    char* d = base + static_cast<size_t>(k) * col;
    LPP_TRY(hipMemcpyAsync(d, src[i], col, hipMemcpyHostToDevice, p->stream));
    *dst[i] = d;
    ++k;
  }
  return LPP_OK;
}

lpp_status check_catalog_args(const lpp_catalog* c, bool shapes) {
  if (!c || c->n < 1 || !c->x || !c->y || !c->z) return LPP_E_INVALID;
  if (c->dtype != LPP_F32 && c->dtype != LPP_F64) return LPP_E_INVALID;
  if (shapes && (!c->g1 || !c->g2)) return LPP_E_INVALID;
  if (c->n > (int64_t{1} << 31) - 1) return LPP_E_UNSUPPORTED;
  return LPP_OK;
}

template <typename T>
GObjSet<T> objset(lpp_plan_s* p, const Layout& L, bool shape_set, int64_t n) {
  GObjSet<T> o{};
  if (shape_set) {
    o.pos = reinterpret_cast<ObjPos<T>*>(wsp(p, L.pos_g));
    o.wr = reinterpret_cast<T*>(wsp(p, L.wr_g));
    o.wi = reinterpret_cast<T*>(wsp(p, L.wi_g));
  } else {
    o.pos = reinterpret_cast<ObjPos<T>*>(wsp(p, L.pos_d));
    o.wr = reinterpret_cast<T*>(wsp(p, L.wr_d));
    o.wi = nullptr;
  }
  o.n = n;
  return o;
}

// Counting sort of the catalogs (cats[0..k), weight scale per catalog) by mesh
// cell into one object set; cell_start (N^3 + 1 entries) receives the offsets.
template <typename T>
lpp_status sort_set(lpp_plan_s* p, const Layout& L, const RawCat* cats, const double* wscale,
                    const double* const* wscale_dev, int k, bool shape, GObjSet<T> out, hipStream_t st) {
  const int64_t ncell = static_cast<int64_t>(p->cfg.mesh_n) * p->cfg.mesh_n * p->cfg.mesh_n;
  uint32_t* starts = reinterpret_cast<uint32_t*>(wsp(p, shape ? L.starts_g : L.starts_d));
  uint32_t* cell_of = reinterpret_cast<uint32_t*>(wsp(p, L.cell_of));
  uint32_t* rank = reinterpret_cast<uint32_t*>(wsp(p, L.rank));
  uint32_t* order = reinterpret_cast<uint32_t*>(wsp(p, L.order));
  uint32_t* bsum = reinterpret_cast<uint32_t*>(wsp(p, L.bsum));
  LPP_TRY(prof_begin(p));
  LPP_TRY(launch_fill_zero(starts, 4 * static_cast<size_t>(ncell + 1), st));
  int64_t off = 0;
  for (int i = 0; i < k; ++i) {
    LPP_TRY(launch_cell_count(cats[i], p->geo, starts, rank + off, cell_of + off, st));
    off += cats[i].n;
  }
  LPP_TRY(launch_big_scan(starts, ncell, bsum, starts, st));
  off = 0;
  for (int i = 0; i < k; ++i) {
    LPP_TRY(launch_cell_scatter<T>(cats[i], p->geo, wscale[i], wscale_dev[i], shape ? 1 : 0, starts, rank + off,
                                   cell_of + off, out, order, off, st));
    off += cats[i].n;
  }
  LPP_TRY(launch_cell_order<T>(starts, ncell, order, out, shape ? 1 : 0, st));
  LPP_TRY(prof_end(p, LPP_STAGE_SORT, 5 + 2 * k));
  return LPP_OK;
}

// sums[0..8) galaxies, [8..16) randoms (see launch_catalog_sums)
lpp_status catalog_sums(lpp_plan_s* p, const Layout& L, const RawCat& g, const RawCat* r, double nbar_default,
                        double* host16) {
  double* part = reinterpret_cast<double*>(wsp(p, L.sums_partial));
  double* out = reinterpret_cast<double*>(wsp(p, L.sums_out));
  LPP_TRY(launch_catalog_sums(g, p->geo, nbar_default, part, catalog_sum_blocks(), out, p->stream));
  if (r) LPP_TRY(launch_catalog_sums(*r, p->geo, nbar_default, part, catalog_sum_blocks(), out + 8, p->stream));
  LPP_TRY(hipMemcpyAsync(host16, out, 8 * (r ? 16 : 8), hipMemcpyDeviceToHost, p->stream));
  LPP_TRY(hipStreamSynchronize(p->stream));
  return LPP_OK;
}

lpp_status sums_status(const double* s) {
  if (s[4] > 0) return LPP_E_NONFINITE;
  if (s[5] > 0) return LPP_E_OUT_OF_BOX;
  if (s[6] > 0) return LPP_E_AT_OBSERVER;
  return LPP_OK;
}

// Host-side scalars of one estimate (Sec. III.A normalisation and shot noise).
struct Scalars {
  double alpha, I, shot_dd, shot_plus, swg, swr;
};

// Validation, staging and the FP64 catalog sums of one estimate: the part
// that needs the host (one synchronisation).  rg / rr point at the caller's
// device columns, or at the staged copies of host columns.
lpp_status prepare(lpp_plan_s* p, const Layout& L, const lpp_catalog* gal, const lpp_catalog* ran, RawCat& rg,
                   RawCat& rr, Scalars& sc) {
  lpp_status s;
  const lpp_config& cfg = p->cfg;
  const double vol = cfg.box_size * cfg.box_size * cfg.box_size;
  lpp_catalog gcat = *gal, rcat = *ran;
  rcat.g1 = rcat.g2 = nullptr;  // shapes of randoms are ignored
  if (!need_shape(p)) gcat.g1 = gcat.g2 = nullptr;
  if ((s = stage(p, &gcat, L.stage_gal, 7, rg)) != LPP_OK) return s;
  if ((s = stage(p, &rcat, L.stage_ran, 5, rr)) != LPP_OK) return s;

  // FP64 sums; nbar defaults to sum(w_gal)/V
  double sums[16];
  if ((s = catalog_sums(p, L, rg, nullptr, 0.0, sums)) != LPP_OK) return s;
  if ((s = sums_status(sums)) != LPP_OK) return s;
  const double nbar_default = sums[0] / vol;
  if ((s = catalog_sums(p, L, rg, &rr, nbar_default, sums)) != LPP_OK) return s;
  if ((s = sums_status(sums + 8)) != LPP_OK) return s;
  sc.swg = sums[0];
  sc.swr = sums[8];
  if (!(sc.swr != 0.0)) return LPP_E_NO_RANDOMS;
  sc.alpha = sc.swg / sc.swr;
  sc.I = sc.alpha * sums[10];
  if (!(sc.I > 0.0) || !std::isfinite(sc.I)) return LPP_E_NO_RANDOMS;
  sc.shot_dd = (sums[1] + sc.alpha * sc.alpha * sums[9]) / sc.I;
  sc.shot_plus = sums[3] / sc.I;
  return LPP_OK;
}

size_t acc_doubles(const lpp_plan_s* p) {
  const size_t nb = static_cast<size_t>(p->cfg.n_kbins);
  return 2 * nb * static_cast<size_t>(n_acc(p)) + 8 * nb;
}

// The device part of one estimate: counting sort, footprint, gathers, 3D
// transforms and shell sums into acc (acc_doubles(p) FP64 values: the series
// rows [na][2nb], then the two bases as [re, im, counts, ksum] rows of width
// 4nb).  No host synchronisation and no host-side reads, so that it can be
// captured into a graph.  The randoms enter the density set with weight
// -alpha w, alpha = alpha_host * (*alpha_dev) (alpha_dev nullable).
template <typename T>
lpp_status device_pipeline(lpp_plan_s* p, const Layout& L, const RawCat& rg, const RawCat& rr, double alpha_host,
                           const double* alpha_dev, double* acc, hipStream_t st) {
  lpp_status s;
  const lpp_config& cfg = p->cfg;
  const int N = cfg.mesh_n, nb = cfg.n_kbins;
  void* Bd = wsp(p, L.mesh[0]);
  void* Bg = wsp(p, L.mesh[1]);
  void* Wset[2][kWork];
  for (int s2 = 0; s2 < 2; ++s2)
    for (int i = 0; i < kWork; ++i) Wset[s2][i] = L.work[s2][i] ? wsp(p, L.work[s2][i]) : nullptr;
  const bool il = cfg.interlacing != 0;
  // Gather pass j deposits into work set j & 1 on the deposit stream gs; the
  // transforms and shell sums of pass j run on st once it is deposited, and
  // the deposit of pass j + 2 waits until they are done with the set.  With
  // profiling on (or serial tuning) both run on st, one after the other.
  const bool overlap = p->aux != nullptr && !p->prof_on && p->tune.serial == 0;
  const hipStream_t gs = overlap ? p->aux : st;
  int pass = 0;

  GObjSet<T> setd = objset<T>(p, L, false, rg.n + rr.n);
  GObjSet<T> setg = objset<T>(p, L, true, rg.n);
  const uint32_t* starts_d = reinterpret_cast<const uint32_t*>(wsp(p, L.starts_d));
  const uint32_t* starts_g = reinterpret_cast<const uint32_t*>(wsp(p, L.starts_g));
  const Footprint fpd = footprint_at(p, L.fp[0]), fpg = footprint_at(p, L.fp[1]);
  if (need_density(p)) {
    const RawCat cs[2] = {rg, rr};
    const double ws[2] = {1.0, -alpha_host};
    const double* wd[2] = {nullptr, alpha_dev};
    if ((s = sort_set<T>(p, L, cs, ws, wd, 2, false, setd, st)) != LPP_OK) return s;
    LPP_TRY(prof_begin(p));
    LPP_TRY(launch_footprint(starts_d, N, fpd, st));
    LPP_TRY(prof_end(p, LPP_STAGE_SORT, 2));
  }
  if (need_shape(p)) {
    const double ws[1] = {1.0};
    const double* wd[1] = {nullptr};
    if ((s = sort_set<T>(p, L, &rg, ws, wd, 1, true, setg, st)) != LPP_OK) return s;
    LPP_TRY(prof_begin(p));
    LPP_TRY(launch_footprint(starts_g, N, fpg, st));
    LPP_TRY(prof_end(p, LPP_STAGE_SORT, 2));
  }

  const int na = n_acc(p);
  // [na][2nb] series rows, then the two bases as [re, im, counts, ksum] rows of width 4nb
  double* partial = reinterpret_cast<double*>(wsp(p, L.bin_partial));
  const size_t acc_len = acc_doubles(p);
  LPP_TRY(launch_fill_zero(acc, 8 * acc_len, st));
  BinArgs ba{};
  ba.N = N;
  ba.nb = nb;
  ba.interlace = il ? 1 : 0;
  ba.compensate = cfg.compensate;
  ba.thr = p->d_thr;
  ba.phase = p->d_phase;
  ba.invw = p->d_invw;
  ba.partial = partial;
  ba.nblocks = p->tune.bin_blocks > 0 ? p->tune.bin_blocks : bin_blocks(N);
  ba.qmax = static_cast<int>(p->tab.thr[nb]);
  // the density kernels walk column pairs: fewer workgroups
  BinArgs bd = ba;
  bd.nblocks = pair_bin_blocks(N, ba.nblocks);
  const FieldSpec s0 = make_spec(0, 0, 0, 0);
  // The base kernels write rows [re, im, cnt, ksum] of width 4nb; they are
  // reduced into their own rows after the series rows.
  double* base_rows[2] = {acc + static_cast<size_t>(2) * nb * na, acc + static_cast<size_t>(2) * nb * na + 4 * nb};
  // kernel groups, each timed as one stage when profiling is on
  auto deposit = [&](const GObjSet<T>& set, const uint32_t* starts, const FieldSpec* specs, int nf, int cplx,
                     const Footprint& fp, void* const* W, size_t j0) -> hipError_t {
    hipError_t e = prof_begin(p);
    if (e == hipSuccess) {
      if (cplx) {
        if constexpr (std::is_same<T, float>::value)
          e = launch_gather_nodes(set, starts, p->geo, p->d_spec + j0, nf, W, fp.cube, true, gs);
        else
          e = launch_gather_nodes(set, starts, p->geo, p->d_spec64 + j0, nf, W, fp.cube, true, gs);
      } else {
        e = launch_gather<T>(set, starts, p->geo, specs, nf, W, fp.cube, true, gs);
      }
    }
    if (e == hipSuccess) e = prof_end(p, LPP_STAGE_DEPOSIT, 1);
    return e;
  };
  // the binning reads modes inside the last shell only
  const int qmax = static_cast<int>(p->tab.thr[nb]);
  // (zpass false: the z pass is left to the fused shell-sum kernel)
  auto fft = [&](void* m, const Footprint& fp, bool zpass) -> hipError_t {
    const FftPrune pr{fp.row, fp.plane, fp.cube, qmax};
    hipError_t e = prof_begin(p);
    if (e == hipSuccess) e = launch_fft_axis_zb<T>(m, N, p->d_tw, 0, pr, st, p->tune.fft_rows_x, streaming(p));
    if (e == hipSuccess) e = prof_end(p, LPP_STAGE_FFT_X, 1);
    if (e == hipSuccess) e = prof_begin(p);
    if (e == hipSuccess) e = launch_fft_axis_zb<T>(m, N, p->d_tw, 1, pr, st, p->tune.fft_cols_y, streaming(p));
    if (e == hipSuccess && zpass)
      e = launch_fft_axis_zb<T>(m, N, p->d_tw, 2, pr, st, p->tune.fft_cols_z, streaming(p));
    if (e == hipSuccess) e = prof_end(p, LPP_STAGE_FFT_YZ, zpass ? 2 : 1);
    return e;
  };
  // Fields in gather order: each set's base first (its spectrum is the
  // reference the other fields of the set are binned against), then the
  // set's other fields; the density set goes first since GD bins against B_delta.
  struct Job {
    FieldSpec spec;
    int fam, series;  // series < 0: base of the set
  };
  std::vector<Job> dens, shape;
  if (need_density(p)) dens.push_back(Job{s0, FAM_DD, -1});
  if (cfg.spectra & (LPP_PLUS | LPP_MINUS)) shape.push_back(Job{s0, FAM_PLUS, -1});
  for (const Field& f : p->tab.fields) (f.fam == FAM_DD ? dens : shape).push_back(Job{f.spec, f.fam, f.series});
  const int copies = il ? 2 : 1;
  auto run_set = [&](const std::vector<Job>& jobs, const GObjSet<T>& set, const uint32_t* starts, int cplx,
                     const Footprint& fp) -> lpp_status {
    const lpp_tuning tn = resolved_tuning(p);
    const int per = cplx ? tn.gather_shape : tn.gather_density;
    for (size_t j0 = 0; j0 < jobs.size(); j0 += per, ++pass) {
      const int nf = static_cast<int>(std::min<size_t>(per, jobs.size() - j0));
      FieldSpec specs[kWork];
      for (int q = 0; q < nf; ++q) specs[q] = jobs[j0 + q].spec;
      void* const* W = Wset[pass & 1];
      if (overlap && pass >= 2) LPP_TRY(hipStreamWaitEvent(gs, p->ev_done[pass & 1], 0));
      LPP_TRY(deposit(set, starts, specs, nf, cplx, fp, W, j0));
      if (overlap) {
        LPP_TRY(hipEventRecord(p->ev_dep[pass & 1], gs));
        LPP_TRY(hipStreamWaitEvent(st, p->ev_dep[pass & 1], 0));
      }
      // The complex fields other than the set's base take their z pass inside
      // the fused shell-sum kernel, in groups of up to zmax fields (zmax = 0:
      // the unfused tuning, or a shell count the fused kernel's LDS could not
      // hold: every field takes the three passes and then the shell-sum kernel).
      const int zmax = (cplx && p->tune.unfused == 0) ? zbin_group_max(N, std::is_same<T, double>::value, nb) : 0;
      for (int m = 0; m < nf * (cplx ? copies : 1); ++m) {
        const bool fused = zmax > 0 && jobs[j0 + m / copies].series >= 0;
        LPP_TRY(fft(W[m], fp, !fused));
      }
      // the set's base first (if it is in this pass), then the other fields in
      // groups of up to bin_group_max fields that share the base and the kind of product
      for (int q = 0; q < nf;) {
        const Job& jb = jobs[j0 + q];
        const int m0 = cplx ? q * copies : q;
        if (jb.series < 0) {
          void* g1 = W[m0];
          void* g2 = (cplx && il) ? W[m0 + 1] : nullptr;
          LPP_TRY(prof_begin(p));
          if (cplx) LPP_TRY(launch_base_gg<T>(ba, g1, g2, Bg, st));
          else LPP_TRY(launch_base_dd<T>(bd, g1, Bd, st));
          LPP_TRY(prof_end(p, LPP_STAGE_BIN, 1));
          LPP_TRY(prof_begin(p));
          LPP_TRY(launch_reduce_partials(partial, cplx ? ba.nblocks : bd.nblocks, 4 * nb, base_rows[cplx], st));
          LPP_TRY(prof_end(p, LPP_STAGE_OTHER, 1));
          ++q;
          continue;
        }
        const void* base = !cplx ? Bd : (jb.fam == FAM_GD ? Bd : Bg);
        const int kind = (cplx && jb.fam == FAM_MINUS) ? 1 : 0;
        const FieldSpec* fs[kBinGroupMax];
        const void* g1[kBinGroupMax];
        const void* g2[kBinGroupMax];
        int series[kBinGroupMax];
        int n = 0;
        const int gmax = zmax > 0 ? zmax : bin_group_max(cplx != 0, std::is_same<T, double>::value, nb);
        while (q < nf && n < gmax) {
          const Job& jq = jobs[j0 + q];
          if (jq.series < 0) break;
          const void* bq = !cplx ? Bd : (jq.fam == FAM_GD ? Bd : Bg);
          const int kq = (cplx && jq.fam == FAM_MINUS) ? 1 : 0;
          if (bq != base || kq != kind) break;
          const int mq = cplx ? q * copies : q;
          fs[n] = &jq.spec;
          g1[n] = W[mq];
          g2[n] = (cplx && il) ? W[mq + 1] : nullptr;
          series[n] = jq.series;
          ++n;
          ++q;
        }
        LPP_TRY(prof_begin(p));
        if (!cplx) LPP_TRY(launch_bin_dd<T>(bd, fs, g1, n, base, st));
        else if (zmax > 0)
          LPP_TRY(launch_zbin_gg<T>(ba, fs, g1, il ? g2 : nullptr, n, base, kind, p->d_tw, fp.plane, st));
        else LPP_TRY(launch_bin_gg<T>(ba, fs, g1, il ? g2 : nullptr, n, base, kind, st));
        LPP_TRY(prof_end(p, LPP_STAGE_BIN, 1));
        LPP_TRY(prof_begin(p));
        const int nblk = !cplx ? bd.nblocks : (zmax > 0 ? zbin_blocks(N, std::is_same<T, double>::value, ba.nblocks)
                                                        : ba.nblocks);
        double* rows[kBinGroupMax];
        for (int i = 0; i < n; ++i) rows[i] = acc + static_cast<size_t>(2) * nb * series[i];
        LPP_TRY(launch_reduce_partials_group(partial, nblk, 2 * nb, n, rows, st));
        LPP_TRY(prof_end(p, LPP_STAGE_OTHER, 1));
      }
      if (overlap) LPP_TRY(hipEventRecord(p->ev_done[pass & 1], st));
    }
    return LPP_OK;
  };
  if (overlap) {  // the deposit stream starts after everything enqueued on st so far
    LPP_TRY(hipEventRecord(p->ev_fork, st));
    LPP_TRY(hipStreamWaitEvent(gs, p->ev_fork, 0));
  }
  if ((s = run_set(dens, setd, starts_d, 0, fpd)) != LPP_OK) return s;
  if ((s = run_set(shape, setg, starts_g, 1, fpg)) != LPP_OK) return s;
  return LPP_OK;
}

// FP64 assembly on the host from the shell sums: prefactors, normalisation,
// shot noise (monopoles only) and the truncated E/B map.
void assemble(const lpp_plan_s* p, const Scalars& sc, std::vector<double>& host_acc, lpp_result* out) {
  const lpp_config& cfg = p->cfg;
  const int nb = cfg.n_kbins, na = n_acc(p);
  const double I = sc.I;
  out->alpha = sc.alpha;
  out->norm_I = sc.I;
  out->shot_dd = sc.shot_dd;
  out->shot_plus = sc.shot_plus;
  out->sum_w_gal = sc.swg;
  out->sum_w_ran = sc.swr;
  // the mode counts come from whichever base was computed (both give the same)
  const double* brow = host_acc.data() + static_cast<size_t>(2) * nb * na + (need_density(p) ? 0 : 4 * nb);
  std::vector<double> counts(brow + 2 * nb, brow + 3 * nb), ksum(brow + 3 * nb, brow + 4 * nb);
  if (p->tab.dd0 >= 0)
    for (int b = 0; b < 2 * nb; ++b) host_acc[static_cast<size_t>(2) * nb * p->tab.dd0 + b] = host_acc[2 * nb * na + b];
  if (p->tab.plus0 >= 0)
    for (int b = 0; b < 2 * nb; ++b)
      host_acc[static_cast<size_t>(2) * nb * p->tab.plus0 + b] = host_acc[2 * nb * na + 4 * nb + b];

  // ---- assembly (FP64, host) ----
  const double kf = 2.0 * M_PI / cfg.box_size;
  const double dn = static_cast<double>(cfg.dn_num) / cfg.dn_den;
  for (int b = 0; b < nb; ++b) {
    out->n_modes[b] = static_cast<int64_t>(llround(counts[b]));
    out->k_eff[b] = counts[b] > 0 ? ksum[b] * kf / counts[b] : 0.0;
    out->k_lo[b] = b * dn * kf;
    out->k_hi[b] = (b + 1) * dn * kf;
  }
  const int ns = static_cast<int>(p->tab.series.size());
  for (int i = 0; i < ns * nb; ++i) out->re[i] = out->im[i] = 0.0;
  for (int a = 0; a < na; ++a) {
    const int fam = p->tab.acc_series[a], Lm = p->tab.acc_L[a];
    const int m = fam == FAM_GD ? 2 : (fam == FAM_MINUS ? 4 : 0);
    const double pref = prefactor(m, Lm);
    const int si = p->tab.series_of_acc[a];
    for (int b = 0; b < nb; ++b) {
      const double c = counts[b] > 0 ? counts[b] : 1.0;
      double re = host_acc[static_cast<size_t>(2) * nb * a + b] * pref / (I * c);
      const double im = host_acc[static_cast<size_t>(2) * nb * a + nb + b] * pref / (I * c);
      if (a == p->tab.dd0) re -= out->shot_dd;
      if (a == p->tab.plus0) re -= out->shot_plus;
      out->re[si * nb + b] = re;
      out->im[si * nb + b] = im;
    }
  }
  // E/B: (P_+^(l) +- sum_L C_lL Re P_-^(L)) / 2
  if ((cfg.spectra & LPP_PLUS) && (cfg.spectra & LPP_MINUS) && cfg.lmax >= 4) {
    auto idx = [&](const std::string& name) {
      for (int i = 0; i < ns; ++i)
        if (p->tab.series[i] == name) return i;
      return -1;
    };
    char nm[32];
    for (int l = 0; l <= cfg.lmax; l += 2) {
      std::snprintf(nm, sizeof nm, "PLUS_l%d", l);
      const int ip = idx(nm);
      std::snprintf(nm, sizeof nm, "EE_l%d", l);
      const int ie = idx(nm);
      std::snprintf(nm, sizeof nm, "BB_l%d", l);
      const int ib = idx(nm);
      for (int b = 0; b < nb; ++b) {
        double mix = 0.0;
        for (int Lm = 4; Lm <= cfg.lmax; Lm += 2) {
          std::snprintf(nm, sizeof nm, "MINUS_L%d", Lm);
          mix += cmap_minus_to_legendre(l, Lm) * out->re[idx(nm) * nb + b];
        }
        out->re[ie * nb + b] = 0.5 * (out->re[ip * nb + b] + mix);
        out->re[ib * nb + b] = 0.5 * (out->re[ip * nb + b] - mix);
      }
    }
  }
}

template <typename T>
lpp_status run_estimate(lpp_plan_s* p, const lpp_catalog* gal, const lpp_catalog* ran, lpp_result* out) {
  lpp_status s;
  if ((s = check_catalog_args(gal, need_shape(p))) != LPP_OK) return s;
  if ((s = check_catalog_args(ran, false)) != LPP_OK) return s;
  if (!out || !out->re || !out->im || !out->n_modes || !out->k_eff || !out->k_lo || !out->k_hi) return LPP_E_INVALID;
  if ((s = ensure_tables(p)) != LPP_OK) return s;
  if ((s = ensure_workspace(p, gal->n, ran->n)) != LPP_OK) return s;
  LPP_TRY(ensure_aux(p));
  const Layout L = layout(p, p->cap_gal, p->cap_ran);
  RawCat rg, rr;
  Scalars sc{};
  if ((s = prepare(p, L, gal, ran, rg, rr, sc)) != LPP_OK) return s;
  double* acc = reinterpret_cast<double*>(wsp(p, L.acc));
  if ((s = device_pipeline<T>(p, L, rg, rr, sc.alpha, nullptr, acc, p->stream)) != LPP_OK) return s;
  std::vector<double> host_acc(acc_doubles(p));
  LPP_TRY(hipMemcpyAsync(host_acc.data(), acc, 8 * host_acc.size(), hipMemcpyDeviceToHost, p->stream));
  LPP_TRY(hipStreamSynchronize(p->stream));
  prof_collect(p);
  assemble(p, sc, host_acc, out);
  return LPP_OK;
}

template <typename T>
lpp_status run_deposit(lpp_plan_s* p, const lpp_catalog* c, double scale, void* mesh) {
  lpp_status s;
  if ((s = check_catalog_args(c, false)) != LPP_OK) return s;
  if (!mesh) return LPP_E_INVALID;
  if ((s = ensure_tables(p)) != LPP_OK) return s;
  if ((s = ensure_workspace(p, std::max<int64_t>(p->cap_gal, 1), std::max(p->cap_ran, c->n))) != LPP_OK) return s;
  const Layout L = layout(p, p->cap_gal, p->cap_ran);
  RawCat rc;
  lpp_catalog cc = *c;
  cc.g1 = cc.g2 = nullptr;  // only the weights are deposited
  if ((s = stage(p, &cc, L.stage_ran, 5, rc)) != LPP_OK) return s;
  double sums[16];
  if ((s = catalog_sums(p, L, rc, nullptr, 1.0, sums)) != LPP_OK) return s;
  if ((s = sums_status(sums)) != LPP_OK) return s;
  GObjSet<T> setd = objset<T>(p, L, false, c->n);
  const double ws[1] = {scale};
  const double* wd[1] = {nullptr};
  if ((s = sort_set<T>(p, L, &rc, ws, wd, 1, false, setd, p->stream)) != LPP_OK) return s;
  const FieldSpec s0 = make_spec(0, 0, 0, 0);
  void* meshes[1] = {mesh};
  LPP_TRY(launch_gather<T>(setd, reinterpret_cast<const uint32_t*>(wsp(p, L.starts_d)), p->geo, &s0, 1, meshes,
                           nullptr, false, p->stream));
  LPP_TRY(hipStreamSynchronize(p->stream));
  return LPP_OK;
}

// Window multipoles Q_l(r) / I of a random catalog (Sec. III.B, eq.
// windowQ_ell, end-point line of sight): see kernels_window.hip.
template <typename T>
lpp_status run_window(lpp_plan_s* p, const lpp_catalog* ran, double alpha, int lmax, int nbr, double rmax, double* Q,
                      double* r_eff, int64_t* counts, double* norm_I) {
  lpp_status s;
  const lpp_config& cfg = p->cfg;
  if ((s = check_catalog_args(ran, false)) != LPP_OK) return s;
  if (!(alpha > 0.0) || !std::isfinite(alpha) || lmax < 0 || lmax > 8 || lmax % 2 || nbr < 1 || nbr > kMaxShells ||
      !(rmax > 0.0) || !std::isfinite(rmax) || !Q || !r_eff || !counts || !norm_I)
    return LPP_E_INVALID;
  if ((s = ensure_tables(p)) != LPP_OK) return s;
  if ((s = ensure_workspace(p, std::max<int64_t>(p->cap_gal, 1), std::max(p->cap_ran, ran->n))) != LPP_OK) return s;
  const Layout L = layout(p, p->cap_gal, p->cap_ran);
  const hipStream_t st = p->stream;
  const int N = cfg.mesh_n;
  RawCat rr;
  lpp_catalog rcat = *ran;
  rcat.g1 = rcat.g2 = nullptr;
  if ((s = stage(p, &rcat, L.stage_ran, 5, rr)) != LPP_OK) return s;
  double sums[16];
  const double vol = cfg.box_size * cfg.box_size * cfg.box_size;
  if ((s = catalog_sums(p, L, rr, nullptr, 0.0, sums)) != LPP_OK) return s;
  if ((s = sums_status(sums)) != LPP_OK) return s;
  if (!ran->nbar && (s = catalog_sums(p, L, rr, nullptr, alpha * sums[0] / vol, sums)) != LPP_OK) return s;
  const double I = alpha * sums[2];
  if (!(I > 0.0) || !std::isfinite(I)) return LPP_E_NO_RANDOMS;

  GObjSet<T> setd = objset<T>(p, L, false, rr.n);
  const uint32_t* starts = reinterpret_cast<const uint32_t*>(wsp(p, L.starts_d));
  const Footprint fp = footprint_at(p, L.fp[0]);
  {
    const double ws[1] = {alpha};
    const double* wd[1] = {nullptr};
    if ((s = sort_set<T>(p, L, &rr, ws, wd, 1, false, setd, st)) != LPP_OK) return s;
  }
  LPP_TRY(launch_footprint(starts, N, fp, st));
  // r-shell thresholds, FP64 in this order: T_b = ceil((b u)(b u)), u = (rmax / nbr) / H
  std::vector<int64_t> thr(static_cast<size_t>(nbr) + 1);
  const double u = (rmax / nbr) / (cfg.box_size / N);
  for (int b = 0; b <= nbr; ++b) thr[b] = static_cast<int64_t>(std::ceil((b * u) * (b * u)));
  int64_t* d_thr = reinterpret_cast<int64_t*>(wsp(p, L.rthr));
  LPP_TRY(hipMemcpyAsync(d_thr, thr.data(), 8 * thr.size(), hipMemcpyHostToDevice, st));
  const int nell = lmax / 2 + 1, nrow = nell + 2;
  WinArgs wa{};
  wa.N = N;
  wa.nb = nbr;
  wa.interlace = cfg.interlacing;
  wa.n_rows = nrow;
  wa.thr = d_thr;
  wa.phase = p->d_phase;
  wa.invw = p->d_invw;
  double* wacc = reinterpret_cast<double*>(wsp(p, L.wacc));
  double* part = reinterpret_cast<double*>(wsp(p, L.wpartial));
  LPP_TRY(launch_fill_zero(wacc, 8 * static_cast<size_t>(nrow) * nbr, st));
  void* B0 = wsp(p, L.mesh[0]);
  void* Zc = wsp(p, L.mesh[1]);
  void* W[kWork];
  for (int i = 0; i < kWork; ++i) W[i] = L.work[0][i] ? wsp(p, L.work[0][i]) : nullptr;
  // the fields: kappa_a h_a(xhat) for every real harmonic of degree l = 0, 2, ..., lmax
  struct WField {
    FieldSpec spec;
    int row;
  };
  std::vector<WField> fields;
  for (int l = 0; l <= lmax; l += 2)
    for (int M = 0; M <= l; ++M)
      for (int cs = 0; cs < (M ? 2 : 1); ++cs) fields.push_back(WField{make_spec(0, l, M, cs), l / 2});
  const FftPrune in_fp{fp.row, fp.plane, fp.cube, INT_MAX};
  const FftPrune full{nullptr, nullptr, nullptr, INT_MAX};
  auto fft = [&](void* m, const FftPrune& pr) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int axis = 0; axis < 3 && e == hipSuccess; ++axis)
      e = launch_fft_axis_zb<T>(m, N, p->d_tw, axis, pr, st,
                                axis == 0 ? p->tune.fft_rows_x : (axis == 1 ? p->tune.fft_cols_y : p->tune.fft_cols_z),
                                streaming(p));
    return e;
  };
  // one packed mesh each, in work set 0 (the row kernel: at most kGatherMaxReal per pass)
  const int per = std::min(resolved_tuning(p).gather_density, kGatherMaxReal);
  int pending = -1;  // field waiting in slot 0 of Zc
  bool counted = false;
  auto bin_pair = [&](int fa, int fb) -> hipError_t {
    hipError_t e = fft(Zc, full);
    if (e == hipSuccess)
      e = launch_window_bin<T>(wa, Zc, &fields[fa].spec, fb >= 0 ? &fields[fb].spec : nullptr, fields[fa].row,
                               fb >= 0 ? fields[fb].row : -1, counted ? 0 : 1, part, st);
    if (e == hipSuccess) e = launch_reduce_partials(part, window_bin_blocks(N), nrow * nbr, wacc, st);
    counted = true;
    return e;
  };
  for (size_t j0 = 0; j0 < fields.size(); j0 += per) {
    const int nf = static_cast<int>(std::min<size_t>(per, fields.size() - j0));
    FieldSpec specs[kWork];
    for (int q = 0; q < nf; ++q) specs[q] = fields[j0 + q].spec;
    LPP_TRY(launch_gather<T>(setd, starts, p->geo, specs, nf, W, fp.cube, true, st));
    for (int q = 0; q < nf; ++q) LPP_TRY(fft(W[q], in_fp));
    for (int q = 0; q < nf; ++q) {
      const int gi = static_cast<int>(j0) + q;
      if (gi == 0) LPP_TRY(launch_window_product<T>(wa, W[q], B0, nullptr, -1, st));
      if (pending < 0) {
        LPP_TRY(launch_window_product<T>(wa, W[q], B0, Zc, 0, st));
        pending = gi;
      } else {
        LPP_TRY(launch_window_product<T>(wa, W[q], B0, Zc, 1, st));
        LPP_TRY(bin_pair(pending, gi));
        pending = -1;
      }
    }
  }
  if (pending >= 0) LPP_TRY(bin_pair(pending, -1));
  std::vector<double> h(static_cast<size_t>(nrow) * nbr);
  LPP_TRY(hipMemcpyAsync(h.data(), wacc, 8 * h.size(), hipMemcpyDeviceToHost, st));
  LPP_TRY(hipStreamSynchronize(st));
  const double H = cfg.box_size / N, n3 = static_cast<double>(N) * N * N;
  for (int b = 0; b < nbr; ++b) {
    const double c = h[static_cast<size_t>(nell) * nbr + b];
    counts[b] = static_cast<int64_t>(std::llround(c));
    r_eff[b] = c > 0 ? h[static_cast<size_t>(nell + 1) * nbr + b] * H / c : 0.0;
    for (int i = 0; i < nell; ++i)
      Q[static_cast<size_t>(i) * nbr + b] =
          c > 0 ? (4 * i + 1) * h[static_cast<size_t>(i) * nbr + b] / (n3 * c * H * H * H * I) : 0.0;
  }
  *norm_I = I;
  return LPP_OK;
}

void drop_graph(lpp_plan_s* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->gkey.clear();
}

uint64_t key_of(const void* ptr) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(ptr)); }

// A batch of catalogs.  Every catalog is validated and its scalars computed
// first (one synchronisation each).  When all catalogs are device-resident,
// the device pipelines of the valid ones are captured into one HIP graph
// (on a capture stream of the plan) and the graph is launched on the plan's
// stream; a later call with the same pointers, sizes and workspace replays
// it without capturing again.  The randoms' -alpha weight of catalog i is
// read from a device table, so the graph does not depend on the scalars.
// Catalogs on the host go through lpp_estimate one by one.
template <typename T>
lpp_status run_batch(lpp_plan_s* p, int32_t n, const lpp_catalog* gals, const lpp_catalog* rans, lpp_result* outs,
                     lpp_status* per) {
  lpp_status s;
  int64_t mg = 1, mr = 1;
  bool device = true;
  for (int i = 0; i < n; ++i) {
    mg = std::max(mg, gals[i].n);
    mr = std::max(mr, rans[i].n);
    device = device && gals[i].on_device && rans[i].on_device;
  }
  if (n == 0) return LPP_OK;
  if ((s = ensure_tables(p)) != LPP_OK) return s;
  if ((s = ensure_workspace(p, mg, mr)) != LPP_OK) return s;
  LPP_TRY(ensure_aux(p));
  lpp_status first = LPP_OK;
  if (!device) {
    for (int i = 0; i < n; ++i) {
      per[i] = lpp_estimate(p, &gals[i], &rans[i], &outs[i]);
      if (per[i] != LPP_OK && first == LPP_OK) first = per[i];
    }
    return first;
  }
  const Layout L = layout(p, p->cap_gal, p->cap_ran);
  std::vector<RawCat> rg(n), rr(n);
  std::vector<Scalars> sc(n);
  std::vector<int> valid;
  for (int i = 0; i < n; ++i) {
    per[i] = check_catalog_args(&gals[i], need_shape(p));
    if (per[i] == LPP_OK) per[i] = check_catalog_args(&rans[i], false);
    const lpp_result* o = &outs[i];
    if (per[i] == LPP_OK && (!o->re || !o->im || !o->n_modes || !o->k_eff || !o->k_lo || !o->k_hi))
      per[i] = LPP_E_INVALID;
    if (per[i] == LPP_OK) per[i] = prepare(p, L, &gals[i], &rans[i], rg[i], rr[i], sc[i]);
    if (per[i] == LPP_OK)
      valid.push_back(i);
    else if (first == LPP_OK)
      first = per[i];
  }
  if (valid.empty()) return first;
  const size_t nv = valid.size(), acc_len = acc_doubles(p);
  const size_t need = nv * (1 + acc_len);
  if (need > p->d_batch_cap) {
    drop_graph(p);
    if (p->d_batch) (void)hipFree(p->d_batch);
    p->d_batch = nullptr;
    p->d_batch_cap = 0;
    if (hipMalloc(&p->d_batch, 8 * need) != hipSuccess) {
      (void)hipGetLastError();
      return LPP_E_NOMEM;
    }
    p->d_batch_cap = need;
  }
  double* d_alpha = p->d_batch;
  double* d_rows = p->d_batch + nv;
  std::vector<double> alpha(nv);
  for (size_t j = 0; j < nv; ++j) alpha[j] = sc[valid[j]].alpha;
  LPP_TRY(hipMemcpyAsync(d_alpha, alpha.data(), 8 * nv, hipMemcpyHostToDevice, p->stream));

  // what the graph depends on: workspace, tables, batch buffers and every catalog column
  std::vector<uint64_t> key = {key_of(p->ws), key_of(p->d_batch), static_cast<uint64_t>(p->cap_gal),
                               static_cast<uint64_t>(p->cap_ran), nv};
  for (int i : valid)
    for (const RawCat* c : {&rg[i], &rr[i]}) {
      for (const void* q : {c->x, c->y, c->z, c->w, c->nbar, c->g1, c->g2}) key.push_back(key_of(q));
      key.push_back(static_cast<uint64_t>(c->n));
      key.push_back(static_cast<uint64_t>(c->dtype));
    }
  if (!p->gexec || key != p->gkey) {
    drop_graph(p);
    if (!p->cap_stream) LPP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    const bool prof = p->prof_on;
    p->prof_on = false;  // no timing events inside the graph
    LPP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    lpp_status cs = LPP_OK;
    for (size_t j = 0; j < nv && cs == LPP_OK; ++j) {
      const int i = valid[j];
      cs = device_pipeline<T>(p, L, rg[i], rr[i], 1.0, d_alpha + j, d_rows + j * acc_len, p->cap_stream);
    }
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
    p->prof_on = prof;
    if (cs != LPP_OK || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return cs != LPP_OK ? cs : hip_status(ce);
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_status(ie);
    }
    p->graph = g;
    p->gexec = ge;
    p->gkey = key;
    ++p->graph_captures;
  }
  LPP_TRY(hipGraphLaunch(p->gexec, p->stream));
  ++p->graph_replays;
  std::vector<double> rows(nv * acc_len);
  LPP_TRY(hipMemcpyAsync(rows.data(), d_rows, 8 * rows.size(), hipMemcpyDeviceToHost, p->stream));
  LPP_TRY(hipStreamSynchronize(p->stream));
  for (size_t j = 0; j < nv; ++j) {
    std::vector<double> h(rows.begin() + j * acc_len, rows.begin() + (j + 1) * acc_len);
    assemble(p, sc[valid[j]], h, &outs[valid[j]]);
  }
  return first;
}

constexpr int kMinBinBlocks = 64;

lpp_tuning resolved_tuning(const lpp_plan_s* p) {
  const int N = p->cfg.mesh_n;
  const bool f64 = p->cfg.precision == LPP_F64;
  lpp_tuning t = p->tune;
  if (t.fft_rows_x <= 0) t.fft_rows_x = zb_default_lines(N, f64, 0);
  if (t.fft_cols_y <= 0) t.fft_cols_y = zb_default_lines(N, f64, 1);
  if (t.fft_cols_z <= 0) t.fft_cols_z = zb_default_lines(N, f64, 2);
  if (t.bin_blocks <= 0) t.bin_blocks = bin_blocks(N);
  if (t.gather_density <= 0) t.gather_density = max_density_fields(p);
  if (t.gather_shape <= 0) t.gather_shape = max_shape_fields(p);
  if (t.fft_streaming <= 0) t.fft_streaming = 8 | zb_default_streaming(N, f64, t.fft_cols_y);
  return t;
}

bool tuning_valid(const lpp_plan_s* p, const lpp_tuning& t) {
  const int N = p->cfg.mesh_n;
  const bool f64 = p->cfg.precision == LPP_F64;
  if (t.fft_rows_x != 0 && !zb_lines_supported(N, f64, 0, t.fft_rows_x)) return false;
  if (t.fft_cols_y != 0 && !zb_lines_supported(N, f64, 1, t.fft_cols_y)) return false;
  if (t.fft_cols_z != 0 && !zb_lines_supported(N, f64, 2, t.fft_cols_z)) return false;
  if (t.bin_blocks != 0 && (t.bin_blocks < kMinBinBlocks || t.bin_blocks > kMaxBinBlocks)) return false;
  if (t.gather_density < 0 || t.gather_density > max_density_fields(p)) return false;
  if (t.gather_shape < 0 || t.gather_shape > max_shape_fields(p)) return false;
  if (t.serial != 0 && t.serial != 1) return false;
  if (t.fft_streaming != 0 && (t.fft_streaming < 8 || t.fft_streaming > 15)) return false;
  if (t.unfused != 0 && t.unfused != 1) return false;
  return true;
}

std::string tuning_key(const lpp_plan_s* p) {
  char k[96];
  std::snprintf(k, sizeof k, "N%d_%s_p%d_il%d", p->cfg.mesh_n, p->cfg.precision == LPP_F64 ? "f64" : "f32",
                p->cfg.assignment, p->cfg.interlacing);
  return k;
}

// One JSON object per line: {"key": "...", "fft_rows_x": a, "fft_cols_y": b, "fft_cols_z": c, ...}
bool parse_tuning_line(const std::string& line, std::string& key, lpp_tuning& t) {
  auto field = [&](const char* name, int32_t& v) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t i = line.find(pat);
    if (i == std::string::npos) return false;
    v = static_cast<int32_t>(std::strtol(line.c_str() + i + pat.size(), nullptr, 10));
    return true;
  };
  const std::string kp = "\"key\":";
  size_t i = line.find(kp);
  if (i == std::string::npos) return false;
  i = line.find('"', i + kp.size());
  const size_t j = i == std::string::npos ? i : line.find('"', i + 1);
  if (j == std::string::npos) return false;
  key = line.substr(i + 1, j - i - 1);
  if (!field("serial", t.serial)) t.serial = 0;  // optional
  if (!field("fft_streaming", t.fft_streaming)) t.fft_streaming = 0;
  if (!field("fft_cols_z", t.fft_cols_z)) t.fft_cols_z = 0;
  if (!field("unfused", t.unfused)) t.unfused = 0;
  return field("fft_rows_x", t.fft_rows_x) && field("fft_cols_y", t.fft_cols_y) &&
         field("bin_blocks", t.bin_blocks) && field("gather_density", t.gather_density) &&
         field("gather_shape", t.gather_shape);
}

std::string tuning_line(const std::string& key, const lpp_tuning& t) {
  char b[320];
  std::snprintf(b, sizeof b,
                "{\"key\": \"%s\", \"fft_rows_x\": %d, \"fft_cols_y\": %d, \"fft_cols_z\": %d, "
                "\"bin_blocks\": %d, \"gather_density\": %d, \"gather_shape\": %d, \"serial\": %d, "
                "\"fft_streaming\": %d, \"unfused\": %d}",
                key.c_str(), t.fft_rows_x, t.fft_cols_y, t.fft_cols_z, t.bin_blocks, t.gather_density, t.gather_shape,
                t.serial, t.fft_streaming, t.unfused);
  return b;
}

void load_tuning_cache(lpp_plan_s* p, const char* path) {
  if (!path || !*path) return;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string want = tuning_key(p);
  char buf[512];
  while (std::fgets(buf, sizeof buf, f)) {
    std::string key;
    lpp_tuning t{};
    if (parse_tuning_line(buf, key, t) && key == want && tuning_valid(p, t)) p->tune = t;
  }
  std::fclose(f);
}

bool store_tuning_cache(const lpp_plan_s* p, const char* path) {
  std::vector<std::string> keep;
  const std::string want = tuning_key(p);
  if (std::FILE* f = std::fopen(path, "r")) {
    char buf[512];
    while (std::fgets(buf, sizeof buf, f)) {
      std::string line(buf), key;
      while (!line.empty() && (line.back() == '\n' || line.back() == '\r')) line.pop_back();
      lpp_tuning t{};
      if (parse_tuning_line(line, key, t) && key != want) keep.push_back(line);
    }
    std::fclose(f);
  }
  keep.push_back(tuning_line(want, p->tune));
  std::FILE* f = std::fopen(path, "w");
  if (!f) return false;
  for (const std::string& l : keep) std::fprintf(f, "%s\n", l.c_str());
  return std::fclose(f) == 0;
}

// Coordinate search over the launch shapes: for each dimension in turn, one
// estimate per candidate with stage timing on, keeping the fastest by the
// time of the stage that dimension drives.
template <typename T>
lpp_status run_autotune(lpp_plan_s* p, const lpp_catalog* gal, const lpp_catalog* ran) {
  std::vector<int64_t> nm(static_cast<size_t>(p->cfg.n_kbins));
  std::vector<double> kv(4 * static_cast<size_t>(p->cfg.n_kbins));
  std::vector<double> ri(2 * p->tab.series.size() * static_cast<size_t>(p->cfg.n_kbins));
  lpp_result r{};
  r.n_modes = nm.data();
  r.k_eff = kv.data();
  r.k_lo = kv.data() + p->cfg.n_kbins;
  r.k_hi = kv.data() + 2 * p->cfg.n_kbins;
  r.re = ri.data();
  r.im = ri.data() + ri.size() / 2;
  const bool prof = p->prof_on;
  const lpp_tuning saved_tune = p->tune;
  double saved_ms[LPP_N_STAGES];
  int64_t saved_l[LPP_N_STAGES];
  std::copy(p->prof_ms, p->prof_ms + LPP_N_STAGES, saved_ms);
  std::copy(p->prof_launches, p->prof_launches + LPP_N_STAGES, saved_l);
  lpp_status s = run_estimate<T>(p, gal, ran, &r);  // warm-up and argument check
  if (s != LPP_OK) return s;
  p->prof_on = true;
  lpp_tuning best = resolved_tuning(p);
  auto measure = [&](const lpp_tuning& t, std::initializer_list<int> stages, double& ms) -> lpp_status {
    p->tune = t;
    for (int i = 0; i < LPP_N_STAGES; ++i) p->prof_ms[i] = 0.0;
    const lpp_status e = run_estimate<T>(p, gal, ran, &r);
    ms = 0.0;
    for (int st : stages) ms += p->prof_ms[st];
    return e;
  };
  auto search = [&](int32_t lpp_tuning::*field, const std::vector<int>& cands, std::initializer_list<int> stages)
      -> lpp_status {
    double best_ms = 1e300;
    int best_v = best.*field;
    for (int v : cands) {
      lpp_tuning t = best;
      t.*field = v;
      if (!tuning_valid(p, t)) continue;
      double ms = 0.0;
      const lpp_status e = measure(t, stages, ms);
      if (e != LPP_OK) return e;
      if (ms < best_ms) {
        best_ms = ms;
        best_v = v;
      }
    }
    best.*field = best_v;
    return LPP_OK;
  };
  s = search(&lpp_tuning::fft_rows_x, {8, 16}, {LPP_STAGE_FFT_X});
  if (s == LPP_OK) s = search(&lpp_tuning::fft_cols_y, {8, 16}, {LPP_STAGE_FFT_YZ});
  if (s == LPP_OK) s = search(&lpp_tuning::fft_cols_z, {8, 16}, {LPP_STAGE_FFT_YZ});
  if (s == LPP_OK)  // non-temporal accesses: all passes, none, or the z pass only (x, y cached)
    s = search(&lpp_tuning::fft_streaming, {8 | 7, 8, 8 | 4, 8 | 5}, {LPP_STAGE_FFT_X, LPP_STAGE_FFT_YZ});
  if (s == LPP_OK) s = search(&lpp_tuning::bin_blocks, {1024, 2048, 4096, 8192}, {LPP_STAGE_BIN});
  if (s == LPP_OK) s = search(&lpp_tuning::gather_density, {2, 4, 6, 8}, {LPP_STAGE_DEPOSIT});
  if (s == LPP_OK) s = search(&lpp_tuning::gather_shape, {1, 2, 4, 6, 8, 10}, {LPP_STAGE_DEPOSIT});
  p->prof_on = prof;
  std::copy(saved_ms, saved_ms + LPP_N_STAGES, p->prof_ms);
  std::copy(saved_l, saved_l + LPP_N_STAGES, p->prof_launches);
  p->tune = s == LPP_OK ? best : saved_tune;
  if (s == LPP_OK) drop_graph(p);  // a captured batch used the old shapes
  return s;
}

}  // namespace

extern "C" {

const char* lpp_version(void) { return "liblpp 0.1 (gfx950)"; }

const char* lpp_status_string(lpp_status s) {
  switch (s) {
    case LPP_OK:
      return "ok";
    case LPP_E_INVALID:
      return "invalid argument or configuration";
    case LPP_E_NONFINITE:
      return "non-finite value in a catalog";
    case LPP_E_OUT_OF_BOX:
      return "object outside the box";
    case LPP_E_AT_OBSERVER:
      return "object at the observer position";
    case LPP_E_NO_RANDOMS:
      return "random catalog has zero total weight";
    case LPP_E_WORKSPACE:
      return "workspace too small";
    case LPP_E_NOMEM:
      return "out of memory";
    case LPP_E_DEVICE:
      return "HIP device error or no device";
    case LPP_E_UNSUPPORTED:
      return "unsupported request";
  }
  return "unknown status";
}

lpp_status lpp_plan_create(const lpp_config* cfg_in, lpp_plan* out) {
  if (!cfg_in || !out) return LPP_E_INVALID;
  *out = nullptr;
  lpp_config cfg = *cfg_in;
  const int N = cfg.mesh_n;
  if (!is_pow2(N) || N < 16 || N > 1024) return LPP_E_INVALID;
  if (!(cfg.box_size > 0.0) || !std::isfinite(cfg.box_size)) return LPP_E_INVALID;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(cfg.box_origin[i]) || !std::isfinite(cfg.observer[i])) return LPP_E_INVALID;
  if (cfg.assignment < 1 || cfg.assignment > 3) return LPP_E_INVALID;
  if ((cfg.interlacing != 0 && cfg.interlacing != 1) || (cfg.compensate != 0 && cfg.compensate != 1))
    return LPP_E_INVALID;
  if (cfg.precision != LPP_F32 && cfg.precision != LPP_F64) return LPP_E_INVALID;
  if (cfg.lmax < 0 || cfg.lmax > 8 || cfg.lmax % 2) return LPP_E_INVALID;
  if (cfg.spectra == 0 || (cfg.spectra & ~static_cast<uint32_t>(LPP_ALL))) return LPP_E_INVALID;
  if (cfg.n_kbins < 1 || cfg.n_kbins > kMaxShells) return LPP_E_INVALID;
  if (cfg.dn_num == 0 && cfg.dn_den == 0) {
    int64_t a = N, b = 2 * static_cast<int64_t>(cfg.n_kbins);
    const int64_t g = igcd(a, b);
    cfg.dn_num = static_cast<int32_t>(a / g);
    cfg.dn_den = static_cast<int32_t>(b / g);
  }
  if (cfg.dn_num <= 0 || cfg.dn_den <= 0) return LPP_E_INVALID;
  // the last edge must not pass the Nyquist frequency: n_kbins * num / den <= N/2
  if (static_cast<int64_t>(cfg.n_kbins) * cfg.dn_num * 2 > static_cast<int64_t>(N) * cfg.dn_den) return LPP_E_INVALID;
  double los_norm = 0.0;
  if (cfg.global_los != 0 && cfg.global_los != 1) return LPP_E_INVALID;
  double los_unit[3] = {0.0, 0.0, 0.0};
  if (cfg.global_los) {
    double m = 0.0;  // scale by the largest component: no overflow or underflow
    for (int i = 0; i < 3; ++i) {
      if (!std::isfinite(cfg.los[i])) return LPP_E_INVALID;
      m = std::max(m, std::fabs(cfg.los[i]));
    }
    if (!(m > 0.0)) return LPP_E_INVALID;
    for (int i = 0; i < 3; ++i) los_norm += (cfg.los[i] / m) * (cfg.los[i] / m);
    los_norm = std::sqrt(los_norm);
    for (int i = 0; i < 3; ++i) los_unit[i] = (cfg.los[i] / m) / los_norm;
  }
  // a spectrum needs its multipoles: GD needs lmax >= 2, MINUS needs lmax >= 4
  if ((cfg.spectra & LPP_GD) && cfg.lmax < 2) return LPP_E_INVALID;
  if ((cfg.spectra & LPP_MINUS) && cfg.lmax < 4) return LPP_E_INVALID;
  lpp_plan_s* p = new (std::nothrow) lpp_plan_s();
  if (!p) return LPP_E_NOMEM;
  p->cfg = cfg;
  build_tables(cfg, p->tab);
  p->geo.N = N;
  p->geo.p = cfg.assignment;
  p->geo.interlace = cfg.interlacing;
  p->geo.H = cfg.box_size / N;
  p->geo.box = cfg.box_size;
  load_tuning_cache(p, std::getenv("LPP_AUTOTUNE_CACHE"));
  p->geo.global_los = cfg.global_los;
  p->geo.los_h = cfg.global_los ? 0.0 : p->geo.H;
  for (int i = 0; i < 3; ++i) {
    p->geo.origin[i] = cfg.box_origin[i];
    p->geo.rel[i] = cfg.box_origin[i] - cfg.observer[i];
    p->geo.los_rel[i] = cfg.global_los ? los_unit[i] : p->geo.rel[i];
  }
  *out = p;
  return LPP_OK;
}

lpp_status lpp_plan_destroy(lpp_plan p) {
  if (!p) return LPP_E_INVALID;
  if (p->own_ws && p->ws) (void)hipFree(p->ws);
  if (p->tabs) (void)hipFree(p->tabs);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  for (hipEvent_t e : {p->ev_fork, p->ev_dep[0], p->ev_dep[1], p->ev_done[0], p->ev_done[1]})
    if (e) (void)hipEventDestroy(e);
  if (p->d_batch) (void)hipFree(p->d_batch);
  delete p;
  return LPP_OK;
}

lpp_status lpp_workspace_size(lpp_plan p, int64_t max_gal, int64_t max_ran, size_t* bytes) {
  if (!p || !bytes || max_gal < 1 || max_ran < 1) return LPP_E_INVALID;
  *bytes = layout(p, max_gal, max_ran).total;
  return LPP_OK;
}

lpp_status lpp_set_workspace(lpp_plan p, void* ptr, size_t bytes) {
  if (!p || !ptr || (reinterpret_cast<uintptr_t>(ptr) % kAlign) != 0) return LPP_E_INVALID;
  if (p->own_ws && p->ws) (void)hipFree(p->ws);
  p->ws = ptr;
  p->ws_bytes = bytes;
  p->own_ws = false;
  p->cap_gal = p->cap_ran = 0;
  return LPP_OK;
}

lpp_status lpp_set_stream(lpp_plan p, void* stream) {
  if (!p) return LPP_E_INVALID;
  p->stream = static_cast<hipStream_t>(stream);
  return LPP_OK;
}

lpp_status lpp_result_layout(lpp_plan p, int32_t* n_series, int32_t* n_kbins) {
  if (!p || !n_series || !n_kbins) return LPP_E_INVALID;
  *n_series = static_cast<int32_t>(p->tab.series.size());
  *n_kbins = p->cfg.n_kbins;
  return LPP_OK;
}

const char* lpp_series_name(lpp_plan p, int32_t i) {
  if (!p || i < 0 || i >= static_cast<int32_t>(p->tab.series.size())) return nullptr;
  return p->tab.series[i].c_str();
}

lpp_status lpp_estimate(lpp_plan p, const lpp_catalog* gal, const lpp_catalog* ran, lpp_result* out) {
  if (!p) return LPP_E_INVALID;
  try {
    return p->cfg.precision == LPP_F64 ? run_estimate<double>(p, gal, ran, out) : run_estimate<float>(p, gal, ran, out);
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

lpp_status lpp_estimate_batch(lpp_plan p, int32_t n, const lpp_catalog* gals, const lpp_catalog* rans,
                              lpp_result* outs, lpp_status* per) {
  if (!p || n < 0 || (n > 0 && (!gals || !rans || !outs || !per))) return LPP_E_INVALID;
  try {
    return p->cfg.precision == LPP_F64 ? run_batch<double>(p, n, gals, rans, outs, per)
                                       : run_batch<float>(p, n, gals, rans, outs, per);
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

lpp_status lpp_batch_stats(lpp_plan p, int64_t* captures, int64_t* replays) {
  if (!p || !captures || !replays) return LPP_E_INVALID;
  *captures = p->graph_captures;
  *replays = p->graph_replays;
  return LPP_OK;
}

lpp_status lpp_get_tuning(lpp_plan p, lpp_tuning* out) {
  if (!p || !out) return LPP_E_INVALID;
  *out = resolved_tuning(p);
  return LPP_OK;
}

lpp_status lpp_set_tuning(lpp_plan p, const lpp_tuning* t) {
  if (!p || !t || !tuning_valid(p, *t)) return LPP_E_INVALID;
  p->tune = *t;
  drop_graph(p);
  return LPP_OK;
}

lpp_status lpp_autotune(lpp_plan p, const lpp_catalog* gal, const lpp_catalog* ran, const char* cache_path) {
  if (!p) return LPP_E_INVALID;
  try {
    const lpp_status s = p->cfg.precision == LPP_F64 ? run_autotune<double>(p, gal, ran)
                                                     : run_autotune<float>(p, gal, ran);
    if (s != LPP_OK) return s;
    if (cache_path && !store_tuning_cache(p, cache_path)) return LPP_E_INVALID;
    return LPP_OK;
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

lpp_status lpp_window_multipoles(lpp_plan p, const lpp_catalog* ran, double alpha, int32_t lmax, int32_t n_rbins,
                                 double rmax, double* Q, double* r_eff, int64_t* counts, double* norm_I) {
  if (!p) return LPP_E_INVALID;
  try {
    return p->cfg.precision == LPP_F64
               ? run_window<double>(p, ran, alpha, lmax, n_rbins, rmax, Q, r_eff, counts, norm_I)
               : run_window<float>(p, ran, alpha, lmax, n_rbins, rmax, Q, r_eff, counts, norm_I);
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

lpp_status lpp_deposit_weights(lpp_plan p, const lpp_catalog* cat, double scale, void* mesh) {
  if (!p) return LPP_E_INVALID;
  try {
    return p->cfg.precision == LPP_F64 ? run_deposit<double>(p, cat, scale, mesh)
                                       : run_deposit<float>(p, cat, scale, mesh);
  } catch (...) {
    return LPP_E_NOMEM;
  }
}

lpp_status lpp_set_profiling(lpp_plan p, int32_t on) {
  if (!p || (on != 0 && on != 1)) return LPP_E_INVALID;
  p->prof_on = on != 0;
  return LPP_OK;
}

lpp_status lpp_get_profile(lpp_plan p, double* ms, int64_t* launches, int32_t n) {
  if (!p || !ms || !launches || n < 0) return LPP_E_INVALID;
  for (int i = 0; i < n; ++i) {
    ms[i] = i < LPP_N_STAGES ? p->prof_ms[i] : 0.0;
    launches[i] = i < LPP_N_STAGES ? p->prof_launches[i] : 0;
  }
  return LPP_OK;
}

lpp_status lpp_reset_profile(lpp_plan p) {
  if (!p) return LPP_E_INVALID;
  for (int i = 0; i < LPP_N_STAGES; ++i) {
    p->prof_ms[i] = 0.0;
    p->prof_launches[i] = 0;
  }
  p->ev_used = 0;
  return LPP_OK;
}

lpp_status lpp_fft3d(lpp_plan p, void* mesh) {
  if (!p || !mesh) return LPP_E_INVALID;
  lpp_status s = ensure_tables(p);
  if (s != LPP_OK) return s;
  const hipError_t e = p->cfg.precision == LPP_F64 ? launch_fft3d<double>(mesh, p->cfg.mesh_n, p->d_tw, p->stream)
                                                   : launch_fft3d<float>(mesh, p->cfg.mesh_n, p->d_tw, p->stream);
  if (e != hipSuccess) return hip_status(e);
  return hip_status(hipStreamSynchronize(p->stream));
}

lpp_status lpp_fft3d_zblocked(lpp_plan p, void* mesh) {
  if (!p || !mesh) return LPP_E_INVALID;
  lpp_status s = ensure_tables(p);
  if (s != LPP_OK) return s;
  const FftPrune full{nullptr, nullptr, nullptr, INT_MAX};
  const int N = p->cfg.mesh_n;
  const int lines[3] = {p->tune.fft_rows_x, p->tune.fft_cols_y, p->tune.fft_cols_z};
  hipError_t e = hipSuccess;
  for (int axis = 0; axis < 3 && e == hipSuccess; ++axis)
    e = p->cfg.precision == LPP_F64
            ? launch_fft_axis_zb<double>(mesh, N, p->d_tw, axis, full, p->stream, lines[axis], streaming(p))
            : launch_fft_axis_zb<float>(mesh, N, p->d_tw, axis, full, p->stream, lines[axis], streaming(p));
  if (e != hipSuccess) return hip_status(e);
  return hip_status(hipStreamSynchronize(p->stream));
}

}  // extern "C"
