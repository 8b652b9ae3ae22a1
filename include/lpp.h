/*
 * lpp.h -- C ABI of the MI355X LPP power-spectrum-multipole library (liblpp.so).
 *
 * The library estimates, from a galaxy catalog with shapes and a random
 * catalog, the local-plane-parallel (LPP, endpoint line of sight) multipoles
 * of the power spectra of a projected rank-2 tensor field and of the density
 * field (Kurita & Takada, arXiv:2202.11839, Sec. III.A):
 *
 *   DD_l    density auto, Legendre moments            (eq. lpp_dens_app)
 *   GD_L    shape-density cross, m=2 assoc. Legendre  (eqs. lpp_estimator_cross_Xiij, def_of_Xiij)
 *   PLUS_l  "plus" shape auto P_+ = P_EE + P_BB       (eq. lpp_estimator_auto_+)
 *   MINUS_L "minus" shape auto P_- = P_EE - P_BB,
 *           m=4 assoc. Legendre                       (eqs. lpp_estimator_auto_-, def_of_Xiijkl)
 *   EE_l, BB_l  (P_+ +- sum_L C_lL Re P_-)/2, the Legendre content of the
 *           truncated m=4 series (eq. relation_pm_EB)
 *
 * per k-shell, with the FKP-style normalisation I and the shot noise of the
 * monopoles (subtracted from DD_l0 and PLUS_l0, and reported separately).
 * Real parts are the spectra; imaginary parts are parity-odd diagnostics
 * that vanish for a parity-invariant field (Sec. II.C).
 *
 * Conventions
 *   - Forward transforms carry exp(-i k.x) (Sec. I, conventions).
 *   - Positions are Cartesian comoving coordinates; the observer sits at
 *     config.observer; each object's line of sight is xhat = (x-o)/|x-o|.
 *   - Shapes (g1, g2) are the components of the projected tensor in the
 *     (e_theta, e_phi) basis of the object's own line of sight, gamma =
 *     g1 + i g2 = e_ij(xhat) gamma_ij (Sec. II.B, eq. gamma_def), where
 *     (e_theta, e_phi, xhat) are the columns of the standard rotation
 *     S(xhat) (App. E, eq. def_standard_rotation); phi = 0 at the poles.
 *   - Mesh: node c at box_origin + c*H, H = box_size/mesh_n, periodic;
 *     NGP/CIC/TSC assignment, optional interlacing (second grid shifted by
 *     H/2 on all axes) and compensation by prod_i sinc(pi n_i/N)^p.
 *   - k-shells: bin b holds the modes n != 0 with T_b <= |n|^2 < T_{b+1},
 *     T_b = ceil((b*dn_num/dn_den)^2) (integers; |n| in units of
 *     kf = 2 pi/box_size).  Default width N/(2 n_kbins), i.e. bins up to
 *     the Nyquist frequency.  n_kbins*dn must not exceed N/2.
 *
 * Ownership and errors
 *   - Every function returns an lpp_status and never throws; after any
 *     error the plan remains valid.
 *   - Catalog and result buffers belong to the caller and are never freed
 *     by the library.  Device workspace is either provided by the caller
 *     (lpp_set_workspace; the caller owns it and keeps it alive while the
 *     plan uses it) or, if none is set, allocated by the plan on first use
 *     and released by lpp_plan_destroy.
 *   - Catalogs (host or device) are checked on the device (non-finite
 *     values, objects outside the box or at the observer, zero random
 *     weight) before any mass assignment; the status is returned after the
 *     check synchronises, and nothing else has run.
 *   - Calls on one plan must not overlap; different plans are independent.
 */
#ifndef LPP_H
#define LPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LPP_OK = 0,
  LPP_E_INVALID = 1,      /* bad argument or configuration                        */
  LPP_E_NONFINITE = 2,    /* NaN/Inf in a catalog column                          */
  LPP_E_OUT_OF_BOX = 3,   /* an object outside [origin, origin + box)^3           */
  LPP_E_AT_OBSERVER = 4,  /* an object closer than 1e-6 box to the observer       */
  LPP_E_NO_RANDOMS = 5,   /* the random catalog has zero total weight             */
  LPP_E_WORKSPACE = 6,    /* caller workspace smaller than lpp_workspace_size     */
  LPP_E_NOMEM = 7,        /* device or host allocation failed                     */
  LPP_E_DEVICE = 8,       /* HIP runtime error or no device                       */
  LPP_E_UNSUPPORTED = 9   /* valid request outside what the library supports      */
} lpp_status;

enum { LPP_F32 = 0, LPP_F64 = 1 };
enum { LPP_DD = 1u, LPP_GD = 2u, LPP_PLUS = 4u, LPP_MINUS = 8u, LPP_ALL = 15u };

typedef struct lpp_plan_s* lpp_plan;

typedef struct {
  int32_t mesh_n;          /* N: power of two, 16 <= N <= 1024                     */
  double box_size;         /* side of the cubic box                                */
  double box_origin[3];    /* lower corner of the box                              */
  double observer[3];      /* observer position (origin of the lines of sight)     */
  int32_t assignment;      /* 1 NGP, 2 CIC, 3 TSC                                  */
  int32_t interlacing;     /* 0 or 1                                               */
  int32_t compensate;      /* 0 or 1: divide by the assignment window              */
  int32_t precision;       /* LPP_F32 or LPP_F64: deposit and FFT arithmetic; the
                              shell sums, I and the shot noise are always FP64     */
  int32_t lmax;            /* even, 0..8; DD/PLUS l = 0..lmax, GD L = 2..lmax,
                              MINUS L = 4..lmax                                    */
  uint32_t spectra;        /* bitmask of LPP_DD | LPP_GD | LPP_PLUS | LPP_MINUS    */
  int32_t n_kbins;         /* number of k-shells, 1..256                           */
  int32_t dn_num, dn_den;  /* bin width dn_num/dn_den in units of kf; both 0 for
                              the default N/(2 n_kbins)                            */
  int32_t global_los;      /* 0: each object's own line of sight xhat (the LPP
                              estimator); 1: one line of sight los for every
                              object, the global-plane-parallel estimator of
                              Sec. II.C (shapes then in the basis of los; the
                              observer is not used)                                */
  double los[3];           /* global_los = 1: the line of sight, any length > 0    */
} lpp_config;

typedef struct {
  int64_t n;               /* number of objects, >= 1                              */
  int32_t on_device;       /* 1: pointers are device pointers                      */
  int32_t dtype;           /* LPP_F32 or LPP_F64, for every column                 */
  const void* x;           /* positions, n each                                    */
  const void* y;
  const void* z;
  const void* w;           /* weights; NULL = 1                                    */
  const void* nbar;        /* mean density at the object (randoms: enters I);
                              NULL = sum(w_gal)/box_size^3, a survey that fills
                              the whole box                                       */
  const void* g1;          /* galaxies: shape components; randoms: NULL           */
  const void* g2;
} lpp_catalog;

typedef struct {           /* every array is caller-allocated, sized by lpp_result_layout */
  int64_t* n_modes;        /* [n_kbins] modes per shell (bit-exact)                 */
  double* k_eff;           /* [n_kbins] mean |k| over the shell                     */
  double* k_lo;            /* [n_kbins] shell edges                                 */
  double* k_hi;
  double* re;              /* [n_series][n_kbins] real parts (spectra)              */
  double* im;              /* [n_series][n_kbins] imaginary parts (diagnostics)     */
  double alpha;            /* sum w_gal / sum w_ran                                 */
  double norm_I;           /* alpha sum_ran w^2 nbar                                */
  double shot_dd;          /* (sum w_gal^2 + alpha^2 sum w_ran^2) / I               */
  double shot_plus;        /* sum w_gal^2 |gamma|^2 / I                             */
  double sum_w_gal;
  double sum_w_ran;
} lpp_result;

/* Plan lifetime.  lpp_plan_create validates the configuration and builds the
 * host tables (bin thresholds, harmonic coefficients); it touches no device. */
lpp_status lpp_plan_create(const lpp_config* cfg, lpp_plan* out);
lpp_status lpp_plan_destroy(lpp_plan plan);

/* Device workspace needed for catalogs of up to max_gal / max_ran objects. */
lpp_status lpp_workspace_size(lpp_plan plan, int64_t max_gal, int64_t max_ran, size_t* bytes);
/* Use caller-owned device memory (>= lpp_workspace_size bytes, 256-byte aligned). */
lpp_status lpp_set_workspace(lpp_plan plan, void* device_ptr, size_t bytes);
/* Launch on this HIP stream (hipStream_t; NULL = the default stream). */
lpp_status lpp_set_stream(lpp_plan plan, void* hip_stream);

/* Output layout: number of series and of k-shells. */
lpp_status lpp_result_layout(lpp_plan plan, int32_t* n_series, int32_t* n_kbins);
/* Name of series i ("DD_l0", "GD_L2", "PLUS_l0", "MINUS_L4", "EE_l0", "BB_l0", ...);
 * NULL if i is out of range.  The string lives as long as the plan. */
const char* lpp_series_name(lpp_plan plan, int32_t i);

/* One estimate: catalogs in, multipoles per shell, normalisation and shot
 * noise out (Sec. III.A).  Synchronises the plan's stream before returning. */
lpp_status lpp_estimate(lpp_plan plan, const lpp_catalog* gal, const lpp_catalog* ran, lpp_result* out);

/* n independent estimates (mock catalogs of any sizes) through the same plan
 * (the batch of mocks of Sec. IV, each one estimate of Sec. III.A);
 * per_catalog_status[i] receives each one's status, and the call returns
 * LPP_OK if all succeeded, otherwise the first failure's status.  Every
 * catalog is validated first.  When every catalog is device-resident, the
 * device work of the valid ones is captured into one HIP graph on a capture
 * stream owned by the plan and launched on the plan's stream; a later call
 * with the same catalog pointers and sizes (and the same workspace) replays
 * that graph without capturing again (new contents of the same buffers are
 * fine).  Host-resident batches run catalog by catalog.  Synchronises the
 * plan's stream before returning.  Stage timing does not cover graph work. */
lpp_status lpp_estimate_batch(lpp_plan plan, int32_t n, const lpp_catalog* gals, const lpp_catalog* rans,
                              lpp_result* outs, lpp_status* per_catalog_status);
/* Graphs captured and launched by lpp_estimate_batch over the plan's life. */
lpp_status lpp_batch_stats(lpp_plan plan, int64_t* captures, int64_t* replays);

/* Multipoles of the window's auto-correlation (Sec. III.B, eqs. windowQ and
 * windowQ_ell), with the line of sight of the pair taken at its first point
 * (end point), or the plan's global line of sight when it has one.  The window is alpha * sum_r w_r delta_D(x - x_r) (randoms
 * weighted to the galaxy density; alpha = sum w_gal / sum w_ran of the data),
 * deposited, interlaced and compensated as the plan's density field, and
 * auto-correlated by FFT on the plan's periodic box, which should be at least
 * twice the window's extent along every axis for the separations of interest.
 * Shells of the separation r: n_rbins linear bins [b dr, (b+1) dr),
 * dr = rmax / n_rbins, in integer form T_b <= |n|^2 < T_{b+1} for the
 * minimum-image offset n in cells, T_b = ceil((b u)(b u)), u = dr / H in FP64;
 * r = 0 is excluded.  Outputs (host, caller-allocated):
 *   Q[i * n_rbins + b]  Q_l(r_b) / I for l = 2i, i = 0 .. lmax/2 (lmax even, <= 8),
 *                       I = alpha sum_r w_r^2 nbar_r (nbar missing: alpha sum w_r / box^3),
 *                       so that Q_0 -> 1 as r -> 0;
 *   r_eff[b]            mean separation of the shell;  counts[b]  separations in it;
 *   *norm_I             I.
 * The randoms follow lpp_estimate's rules (shapes ignored).  Uses the plan's
 * workspace (resized like lpp_estimate's); synchronises the plan's stream. */
lpp_status lpp_window_multipoles(lpp_plan plan, const lpp_catalog* ran, double alpha, int32_t lmax, int32_t n_rbins,
                                 double rmax, double* Q, double* r_eff, int64_t* counts, double* norm_I);

/* The same window multipoles by direct pair counting of randoms, the
 * paper's own route (Sec. III.B, eq. windowQ_ell; Sec. IV.C): over the
 * ordered pairs (i, j), i != j, of the catalog `ran` (typically a random
 * subsample of the randoms),
 *   Q[i * n_rbins + b] = (4i+1) alpha^2 sum_{pairs in b} w_i w_j L_{2i}(rhat . dhat) / (V_b norm_I),
 * V_b = (4 pi / 3)((b+1)^3 - b^3) dr^3, dr = rmax / n_rbins, shell b holding
 * (b dr)^2 <= r^2 < ((b+1) dr)^2 with r^2 = dx*dx + dy*dy + dz*dz rounded in
 * FP64 without fused multiply-adds (coincident points are in no shell), and
 * the pair's line of sight dhat the direction from `observer` to the pair's
 * midpoint (los = 1, the paper's "direction toward the pair") or to its
 * first point (los = 0, the end point of the LPP estimator).  alpha weights
 * the given catalog to the galaxy density (for a subsample of m of M
 * randoms of equal weight: the full catalog's alpha times M/m) and norm_I
 * is the estimator's I, so that Q_0 -> 1 as r -> 0.  Outputs as
 * lpp_window_multipoles (host arrays): Q for l = 0, 2, .., lmax (even, <= 8),
 * r_eff[b] the mean separation and counts[b] the number of ordered pairs
 * (exact).  Columns host or device, FP32 or FP64 (summed in FP64); w NULL
 * = 1; no object may sit at the observer; 2 <= n <= 2^26, 1 <= n_rbins <= 256.
 * FP64 throughout, all n^2 pairs (about 1e10 pair terms per second);
 * allocates its own device memory and synchronises `stream`.
 * LPP_E_NONFINITE for a non-finite column value. */
lpp_status lpp_window_pairs(const lpp_catalog* ran, double alpha, double norm_I, const double* observer, int32_t los,
                            int32_t lmax, int32_t n_rbins, double rmax, double* Q, double* r_eff, int64_t* counts,
                            void* stream);

/* Coefficient of Q_{l''} in the window mixing Q^X_{l l'}(r) of eq.
 * def_of_Q_llp (Sec. III.B): (2l+1) sqrt((l-m)!/(l+m)! (l'+m)!/(l'-m)!)
 * (l'' l l'; 0 0 0)(l'' l l'; 0 m -m), m = mX (0 for delta-delta and plus, 2
 * for the cross, 4 for minus); zero when l < m or l' < m.  Host only. */
lpp_status lpp_window_coefficient(int32_t mX, int32_t l, int32_t lp, int32_t lpp, double* out);

/* The plain window-convolved template path (Sec. III.B, eq.
 * window_convolution_X_hankel) of the linear tidal-alignment model, one
 * FFTLog (Hamilton 2000) per Hankel transform, FP64, on the current device.
 * Per parameter point (A, b, f, sigma8, s_N) (params[5 p + 0..4]):
 *   P_lin = (sigma8 / sigma8_fid)^2 P_fid exp(-(k/10)^2), sigma8_fid the
 *   top-hat R = 8 rms of pfid (trapezoid in ln k on the grid);
 *   model multipoles P_+^(0,2,4) = A^2 {2/15, -4/21, 2/35} P_lin,
 *   P_gd^(2,4) = -A {(7b+f)/42, f/105} P_lin;
 *   xi^(l') = H^{-1}_{l'}[P^(l')] (FFTLog bias 1.5), multiplied by
 *   Q^X_{l l'}(r) = sum_{l''} lpp_window_coefficient(mX, l, l', l'') Q_{l''}(r),
 *   P~^(l) = H_l[sum_{l'} Q^X_{l l'} xi^(l')] (bias 1.0 at l = 0, 0.5 above),
 *   interpolated linearly in ln k to k_out; P~_+^(0) += s_N 2 sigma_gamma^2 / nbar.
 * pfid: P_fid at k_n = exp(ln k_min + n d), d = ln(k_max/k_min)/(n_log - 1)
 *   (n_log = 4096; the FFTLog grids are this k grid and r_j = 1/k_{n_log-1-j});
 * Q[i * n_q + j]: Q_{2i}(r_q[j]) / I, i = 0..4 (lpp_window_multipoles),
 *   r_q increasing and > 0; linear in r, with Q(0) = (1, 0, 0, 0, 0) and zero
 *   beyond r_q[n_q-1];
 * out[(p * 5 + o) * n_k + i]: o = 0, 1, 2 for P~_+^(0,2,4), o = 3, 4 for P~_gd^(2,4)
 *   at k_out[i] (k_min <= k_out <= k_max, n_k <= 256).
 * device_io = 0: params and out are host arrays; 1: device arrays (the
 * tables stay host arrays).  stream: a hipStream_t (NULL = default).  The
 * call allocates its own device scratch (about 330 MB) and synchronises the
 * stream before returning.  LPP_E_UNSUPPORTED for another n_log. */
lpp_status lpp_template_plain(const double* pfid, double k_min, double k_max, int32_t n_log, const double* r_q,
                              const double* Q, int32_t n_q, const double* params, int64_t n_pts,
                              const double* k_out, int32_t n_k, double nbar, double sigma_gamma, double* out,
                              int32_t device_io, void* stream);

/* The same plain path for all four families of the estimator (Sec. IV.C,
 * eq. all_convolutions and the leakage equations), with the density auto
 * spectrum of the Kaiser model, P_dd = (b + f mu^2)^2 P_lin, whose multipoles
 * are {b^2 + 2bf/3 + f^2/5, 4bf/3 + 4f^2/7, 8f^2/35} P_lin, and the minus
 * shape spectrum of the same alignment model, P_- = P_+ = (A^2/4)(1-mu^2)^2 P_lin,
 * whose only m=4 moment is P_-^(4) = A^2 P_lin / 420.  Window mixing with
 * mX = 0 for dd and plus, 2 for gd and 4 for minus; everything else as for
 * lpp_template_plain.  Output rows in the estimator's series order:
 *   out[(p * 9 + o) * n_k + i], o = 0, 1, 2: P~_dd^(0,2,4) (P~^(2) is the leakage
 *   moment of an isotropic model), o = 3, 4: P~_gd^(2,4), o = 5, 6, 7: P~_+^(0,2,4)
 *   (with the shot-noise term on l = 0), o = 8: P~_-^(4).
 * Allocates its own device scratch and synchronises the stream. */
lpp_status lpp_template_multipoles(const double* pfid, double k_min, double k_max, int32_t n_log, const double* r_q,
                                   const double* Q, int32_t n_q, const double* params, int64_t n_pts,
                                   const double* k_out, int32_t n_k, double nbar, double sigma_gamma, double* out,
                                   int32_t device_io, void* stream);

/* lpp_template_plain for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, with the device memory of the
 * call (tables, the xi of a chunk of points, host-I/O staging) taken from a
 * static 24 MiB array that the library holds on each device it runs on
 * until the process ends.  Points are processed in chunks that fit the
 * array (about 135 points per pass, so any n_pts is accepted; large batches
 * run slower than through lpp_template_plain, whose chunks are 2,048 points).
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (two streams, two threads) race and must be serialised by
 * the caller; nothing in the array needs to start at zero.  Same errors as
 * lpp_template_plain; LPP_E_DEVICE if the array's address cannot be
 * obtained.  Allocates no device memory; synchronises the stream. */
lpp_status lpp_template_plain_noalloc(const double* pfid, double k_min, double k_max, int32_t n_log,
                                      const double* r_q, const double* Q, int32_t n_q, const double* params,
                                      int64_t n_pts, const double* k_out, int32_t n_k, double nbar,
                                      double sigma_gamma, double* out, int32_t device_io, void* stream);

/* ---- Emulator network (the learned stand-in for lpp_template_plain) ----
 * A fully connected network widths[0] -> ... -> widths[n_layers] with SiLU
 * (x / (1 + exp(-x))) after every layer but the last, trained on the mean
 * squared error with Adam (beta1 0.9, beta2 0.999, eps 1e-8).  Every matrix
 * product runs on the matrix cores with BF16 operands and FP32 accumulation;
 * parameters, gradients and moments are FP32, and a BF16 copy of the
 * parameters (round to nearest even) feeds the products.  In the forward
 * pass each layer input a enters as two BF16 operands, hi = bf16(a) and
 * lo = bf16(a - hi) (two products into one accumulator); the backward
 * products use the hi halves.  Parameter layout
 * (lpp_mlp_get_params): for each layer l, W_l [widths[l+1]][widths[l]]
 * row-major (y = x W^T + b), then b_l.  Initial values: uniform in
 * +-1/sqrt(fan-in) from a splitmix64 stream of `seed`.  All device arrays are
 * FP32, row-major [rows][width], on the current device; calls on one network
 * are stream-ordered and must not overlap.  Not a paper method: the paper has
 * no emulator (the template path it stands in for is Sec. III.B). */
typedef struct lpp_mlp_s* lpp_mlp;
lpp_status lpp_mlp_create(const int32_t* widths, int32_t n_layers, int64_t max_batch, uint64_t seed, lpp_mlp* out);
lpp_status lpp_mlp_destroy(lpp_mlp mlp);
lpp_status lpp_mlp_set_stream(lpp_mlp mlp, void* hip_stream);
lpp_status lpp_mlp_num_params(lpp_mlp mlp, int64_t* n);
/* FP32 parameters and the last step's gradients to host arrays (either may be NULL). */
lpp_status lpp_mlp_get_params(lpp_mlp mlp, float* params_host, float* grads_host);
lpp_status lpp_mlp_set_params(lpp_mlp mlp, const float* params_host);
/* Y[B][widths[n_layers]] = net(X[B][widths[0]]), B <= max_batch (device arrays). */
lpp_status lpp_mlp_forward(lpp_mlp mlp, const float* X, int64_t B, float* Y);
/* One Adam step on the batch (X, targets T) at learning rate lr; the batch
 * loss to *loss_host if not NULL (then the stream is synchronised). */
lpp_status lpp_mlp_train_step(lpp_mlp mlp, const float* X, const float* T, int64_t B, float lr, float* loss_host);
/* epochs over the n rows of (X, T) (device arrays), batches of `batch` rows in
 * a splitmix64-shuffled order per epoch (the last partial batch dropped), the
 * learning rate following a cosine from lr0 to lr1 over the whole fit; each
 * epoch's step is captured once into a HIP graph and replayed.  The last
 * batch loss to *final_loss if not NULL.  Synchronises the stream. */
lpp_status lpp_mlp_fit(lpp_mlp mlp, const float* X, const float* T, int64_t n, int32_t batch, int32_t epochs, float lr0,
                       float lr1, uint64_t seed, float* final_loss);

/* The emulator's encoding of lpp_template_plain's outputs (device arrays;
 * params [n][5] = (A, b, f, sigma8, s_N), templates [n][5][n_k] FP64):
 *   X[n][5]       (theta_i - lo_i) / (hi_i - lo_i) * 2 - 1, ranges = {lo_0, hi_0, ..., lo_4, hi_4} (host);
 *   T[n][5 n_k]   standardised shapes: P~_+^(l) / (A^2 sigma8^2) with the shot noise
 *                 s_N 2 sigma_gamma^2 / nbar taken out of l = 0, P~_gd^(L) / (A sigma8^2),
 *                 minus mean[c], over sd[c] (FP64 column statistics over the n rows, written
 *                 to the device arrays mean, sd [5 n_k]; sd = 1 for a column whose spread is
 *                 below 1e-9 of its mean, i.e. constant up to rounding).
 * LPP_E_INVALID (nothing written) if a range has hi <= lo or a point's prefactor
 * A^2 sigma8^2 or A sigma8^2 is zero or not finite (such a point has no shape).
 * Synchronises the stream; allocates an FP64 scratch of n * 5 n_k values. */
lpp_status lpp_emulator_encode(const double* params, const double* templates, int64_t n, int32_t n_k,
                               const double* ranges, double nbar, double sigma_gamma, float* X, float* T,
                               double* mean, double* sd, void* hip_stream);
/* The inverse map around the network: out[n][5][n_k] (device, FP64) for the
 * parameter points params[n][5] (device), with a network of widths 5 -> ... -> 5 n_k
 * trained on lpp_emulator_encode's (X, T); batches of the network's max_batch.
 * When no layer input is wider than 256 the network runs as one fused launch
 * per batch (activations kept on chip); its outputs are the same bits as the
 * layer-by-layer lpp_mlp_forward's.  LPP_E_INVALID if a range has hi <= lo. */
lpp_status lpp_emulator_predict(lpp_mlp mlp, const double* params, int64_t n, int32_t n_k, const double* ranges,
                                double nbar, double sigma_gamma, const double* mean, const double* sd, double* out);

/* Launch shapes of the plan's kernels (0 = the built-in default).  Every
 * choice gives the same result up to FP32/FP64 rounding order of the shell
 * sums (the transforms and the deposit are unchanged bit for bit). */
typedef struct {
  int32_t fft_rows_x;      /* x pass: lines per workgroup, 8 or 16 (8 z-values of 1 or 2 y) */
  int32_t fft_cols_y;      /* y pass: lines per workgroup, 8 or 16 (8 z-values of 1 or 2 x) */
  int32_t fft_cols_z;      /* z pass: lines per workgroup, 8 or 16 (columns x of one y)     */
  int32_t bin_blocks;      /* workgroups of the shell-sum kernels, 64 .. 8192               */
  int32_t gather_density;  /* density fields per deposit pass, 1 .. 8 (FP64 at N = 1024:
                              1 .. 4)                                                      */
  int32_t gather_shape;    /* shape fields per deposit pass: 1 .. 10 in FP32 up to N = 512,
                              1 .. 4 in FP32 at N = 1024 and in FP64, 1 .. 2 in FP64 at
                              N = 1024                                                     */
  int32_t serial;          /* 1: deposits and transforms on the plan's stream one after the
                              other; 0: the next pass's deposit runs on a second stream of the
                              plan while the current pass is transformed (profiling with
                              lpp_set_profiling always runs them one after the other)      */
  int32_t fft_streaming;   /* 8 + a bit mask of the passes of the 3D transform (1 x, 2 y, 4 z)
                              that use non-temporal loads and stores; 0 = the default
                              (meshes of at most 256 MiB, which stay in the Infinity Cache
                              between passes: z only; larger: x and z, y too when its
                              workgroups read runs of 128 bytes or more: FP32 with 16 y
                              lines, or FP64)                                             */
  int32_t unfused;         /* 1: every shape field takes the z pass as a launch of its own and
                              the shell-sum kernel reads the transformed fields back (also
                              the path for a size whose shells the fused kernel's LDS could
                              not hold, which no supported mesh and shell count reaches);
                              0: the shape fields' z pass runs inside their shell sums     */
} lpp_tuning;
/* Current launch shapes with defaults resolved; set validates each field
 * (LPP_E_INVALID for an unsupported value, the plan unchanged). */
lpp_status lpp_get_tuning(lpp_plan plan, lpp_tuning* out);
lpp_status lpp_set_tuning(lpp_plan plan, const lpp_tuning* t);
/* Time the candidate launch shapes on this catalog pair (one estimate per
 * candidate, one dimension at a time), keep the fastest in the plan, and
 * store them in cache_path (a JSON-lines file, one record per mesh size,
 * precision, assignment and interlacing; NULL = no file).  A plan created
 * while the environment variable LPP_AUTOTUNE_CACHE names such a file starts
 * from its record.  The catalogs follow lpp_estimate's rules. */
lpp_status lpp_autotune(lpp_plan plan, const lpp_catalog* gal, const lpp_catalog* ran, const char* cache_path);

/* Building blocks, exposed for testing and for callers with their own meshes.
 * All meshes are complex, index x + N*(y + N*z), interleaved (re, im), of the
 * plan's precision (float2 or double2), on the device.  (The estimator keeps
 * its own meshes z-blocked, ((z/8 N + y) N + x) 8 + z%8; these entry points
 * take and return the plain order.) */

/* Mass-assign the weights w of a catalog (times `scale`) onto `mesh` (N^3
 * complex; real part = the grid, imaginary part = the interlaced grid if the
 * plan interlaces, else 0).  The mesh is overwritten. */
lpp_status lpp_deposit_weights(lpp_plan plan, const lpp_catalog* cat, double scale, void* mesh);

/* In-place forward 3D DFT (exp(-2 pi i n.c/N)) of an N^3 complex device mesh. */
lpp_status lpp_fft3d(lpp_plan plan, void* mesh);

/* The estimator's own 3D transform on a mesh in its z-blocked order: node or
 * mode (x, y, z) at ((z/8 N + y) N + x) 8 + z%8 (N^3 complex of the plan's
 * precision, in place, exp(-2 pi i n.c/N)), with the x, y and z passes, line
 * counts and non-temporal accesses of lpp_estimate but nothing pruned
 * (every node read, every mode written). */
lpp_status lpp_fft3d_zblocked(lpp_plan plan, void* mesh);

/* Per-stage timing.  When on, the plan records a pair of HIP events on its
 * stream around every kernel group of lpp_estimate and accumulates the
 * elapsed milliseconds and kernel launches per stage (enum below) until
 * lpp_reset_profile.  Off by default; costs two event records per group. */
enum {
  LPP_STAGE_SORT = 0,    /* catalog sort by tile (count, scan, scatter)        */
  LPP_STAGE_DEPOSIT = 1, /* mass assignment kernels                            */
  LPP_STAGE_FFT_X = 2,   /* unit-stride FFT pass                               */
  LPP_STAGE_FFT_YZ = 3,  /* strided FFT passes (y and z, same kernel)          */
  LPP_STAGE_BIN = 4,     /* base construction and shell binning kernels        */
  LPP_STAGE_OTHER = 5,   /* clears and partial-sum reductions                  */
  LPP_N_STAGES = 6
};
lpp_status lpp_set_profiling(lpp_plan plan, int32_t on);
/* ms[i], launches[i] for stages i < n (stages beyond LPP_N_STAGES read 0). */
lpp_status lpp_get_profile(lpp_plan plan, double* ms, int64_t* launches, int32_t n);
lpp_status lpp_reset_profile(lpp_plan plan);

/* Message for a status code (static string). */
const char* lpp_status_string(lpp_status s);

/* Library version string. */
const char* lpp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LPP_H */
