/*
 * xs21 -- excursion-set ionisation, 21 cm brightness temperature and binned
 * power spectrum on AMD Instinct MI355X (gfx950).
 *
 * The method is the likelihood core of 21CMMC (Greig & Mesinger 2015): for a
 * fixed evolved density box and one astrophysical parameter set
 * (zeta, R_mfp, T_vir) it computes
 *
 *   1. delta_R: the box smoothed with a sharp-k top hat for radii stepping down
 *      from the largest filter scale to the cell size (Section 2.1);
 *   2. the ionisation field: a cell is fully ionised when
 *      zeta * f_coll(delta_R) >= 1 at any radius (eq. 1), with
 *      f_coll = erfc((delta_c - delta_R) / sqrt(2 (sigma^2(M_min) - sigma^2(R)))),
 *      otherwise it keeps the partial ionised fraction zeta * f_coll at the
 *      cell radius (Section 2.1), with M_min from T_vir (eq. 3);
 *   3. the brightness temperature dT_b = tb0 x_HI (1 + delta) sqrt((1+z)/10) mK
 *      (eq. 4 with T_S >> T_gamma and without the velocity-gradient factor);
 *   4. its spherically averaged power spectrum in logarithmic k bins
 *      (Section 2.2).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Boxes are N^3 arrays in C order (last axis contiguous), N a power of two in
 * [8, 512].  Lengths are comoving Mpc, masses Msun, temperatures K, dT_b mK,
 * P(k) mK^2 Mpc^3 (per mode |X|^2 L^3 / N^6 with X the unnormalised DFT).
 * k bins: edges e_b = k_f (N/2)^(b/n_bins), b = 0..n_bins, on [k_f, k_Nyquist];
 * DC and modes with |n| > N/2 are dropped; the top edge is closed.
 * Filter: W_R(k) = 1 for |k| <= k_c = (9 pi / 2)^(1/3) / R (volume matching).
 * Radii: the shared ladder of a box is R_i = ladder_top / radius_step^i while
 * R_i > L/N, then L/N.  A walker of mean free path R_mfp uses the radii of the
 * ladder with R <= R_mfp (and always the cell radius).
 *
 * Ownership.  The caller owns every buffer.  All device memory the library
 * uses is one workspace the caller allocates (e.g. a torch tensor) and passes
 * to xs21_prepare; the library keeps only host-side tables and that pointer.
 * Host input boxes are copied by xs21_add_box and may be freed afterwards;
 * device input boxes are copied by xs21_prepare and may be freed after it.
 *
 * Errors.  Every call returns xs21_status; nothing else crosses the ABI.  On
 * error the outputs are unspecified and xs21_last_error() describes the
 * cause (thread-local, valid until the next call on the same thread).  After
 * XS21_EINVAL, XS21_ENOMEM or XS21_EUNSUPPORTED the context stays usable.
 * After XS21_EDEVICE the context is poisoned and every later call on it
 * returns XS21_ESTATE.
 *
 * Threading.  A context belongs to one host thread and one HIP stream.
 */
#ifndef XS21_H
#define XS21_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  XS21_OK = 0,
  XS21_EINVAL = -1,       /* argument out of range, NaN, unknown handle       */
  XS21_ENOMEM = -2,       /* workspace too small / host allocation failed     */
  XS21_EDEVICE = -3,      /* a HIP call failed; the context is poisoned       */
  XS21_EUNSUPPORTED = -4, /* valid request this build does not implement      */
  XS21_ESTATE = -5        /* call out of order, or context poisoned           */
} xs21_status;

typedef enum { XS21_F32 = 0, XS21_F64 = 1, XS21_BF16 = 2 } xs21_dtype;

/* Constants of the method.  xs21_physics_default() fills the values used
 * throughout the paper (Section 1 cosmology) and the synthetic spectrum shape. */
typedef struct {
  double delta_c;     /* linear collapse threshold, 1.686                          */
  double omega_m;     /* 0.27 (Section 1)                                          */
  double omega_l;     /* 0.73                                                      */
  double h;           /* 0.7                                                       */
  double tb0_mK;      /* 27 mK prefactor of eq. (4)                                */
  double pk_amp;      /* A of P(k) = A k (1 + (k/k0)^2)^-2 at z_ref, Mpc^4          */
  double pk_k0;       /* k0, Mpc^-1 (0.05)                                         */
  double z_ref;       /* redshift of pk_amp; D(z) = (1+z_ref)/(1+z) (9)            */
  double radius_step; /* ratio of consecutive radii (1.1)                          */
  double ladder_top;  /* top radius of the shared ladder, Mpc (20)                 */
  double mu;          /* mean molecular weight in eq. (3) (0.6)                    */
  int32_t mmin_form;  /* 0: M_min = 1e8 (T/1e4)^1.5 ((1+z)/10)^-1.5; 1: eq. (3)     */
  int32_t velocity;   /* 1: dT_b includes H / (dv_r/dr + H) of eq. (4), the linear
                         line-of-sight velocity gradient of the box (first axis);
                         0: that factor is 1 (default)                            */
  double dvdr_max;    /* limit on |dv_r/dr| / H in that factor (0.2)               */
} xs21_physics;

/* One astrophysical parameter set (Section 2.1). */
typedef struct {
  double zeta;   /* ionising efficiency, > 0                */
  double r_mfp;  /* mean free path / largest filter, Mpc > 0 */
  double t_vir;  /* minimum virial temperature, K > 0       */
} xs21_walker;

/* One parameter set of the two-population model (Section 4, eq. 9): the
 * efficiency of a halo of virial temperature T is zeta0 (T / t_feed)^beta for
 * T >= t_feed, zeta0 (T / t_feed)^alpha for 1e4 K <= T < t_feed, and 0 below
 * 1e4 K (the atomic-cooling limit, which replaces t_vir as the smallest
 * ionising halo).  Limits: 0 < zeta0 <= 1e6, 1e4 <= t_feed <= 1e9 K,
 * |alpha|, |beta| <= 10 (the paper's prior is [-4/3, 10/3] for both). */
typedef struct {
  double zeta0;   /* normalisation of the efficiency, > 0             */
  double r_mfp;   /* mean free path / largest filter, Mpc > 0        */
  double t_feed;  /* feedback virial temperature, K                  */
  double alpha;   /* power-law index between 1e4 K and t_feed        */
  double beta;    /* power-law index above t_feed                    */
} xs21_walker2;

typedef struct xs21_ctx xs21_ctx;
typedef int32_t xs21_box;

/* ---------------------------------------------------------------- basics */

/* Message of the last failing call on this thread ("" if none). */
const char* xs21_last_error(void);

/* Fills *p with the default constants.  p must not be NULL. */
xs21_status xs21_physics_default(xs21_physics* p);

/* Creates a context bound to HIP device `hip_device` and stream `hip_stream`
 * (a hipStream_t; NULL selects the default stream).  Constants are copied.
 * EINVAL: bad constants; EDEVICE: the device cannot be selected. */
xs21_status xs21_create(xs21_ctx** out, int hip_device, void* hip_stream,
                        const xs21_physics* phys);

/* Releases the host-side state of a context.  NULL is accepted. */
xs21_status xs21_destroy(xs21_ctx* ctx);

/* Blocks until all work queued by the context on its stream has finished. */
xs21_status xs21_sync(xs21_ctx* ctx);

/* ---------------------------------------------------------------- boxes */

/* Registers a density box delta(x) of n^3 cells, side box_mpc, redshift z,
 * with n_bins logarithmic power-spectrum bins.
 * delta: n^3 values of `dtype` (XS21_F32 or XS21_F64) in C order, on the host
 * (on_device = 0, copied now) or on the device (on_device = 1, copied by
 * xs21_prepare).  The box dtype fixes the arithmetic of everything computed
 * on it: F64 boxes run the whole path in double precision, F32 boxes in
 * single precision with FP64 host planning and FP64 bin sums.
 * Must be called before xs21_prepare.
 * EINVAL: n not a power of two in [8, 512], box_mpc <= 0, z <= -1, n_bins
 * outside [1, 64], non-finite values; ESTATE: after xs21_prepare. */
xs21_status xs21_add_box(xs21_ctx* ctx, const void* delta, int on_device, xs21_dtype dtype,
                         int n, double box_mpc, double z, int n_bins, xs21_box* out);

/* Shared radius ladder of a registered box (Section 2.1: decreasing radii
 * from ladder_top down to the cell size L/n).  Writes up to `cap` radii, in
 * decreasing order, to out (may be NULL) and their count to *n_radii. */
xs21_status xs21_box_radii(xs21_ctx* ctx, xs21_box box, double* out, int cap, int* n_radii);

/* k_b (count-weighted mean |k| per bin, Mpc^-1) and mode counts c_b of a box
 * geometry; each array holds n_bins doubles. Either pointer may be NULL. */
xs21_status xs21_box_bins(xs21_ctx* ctx, xs21_box box, double* k_mean, double* counts);

/* ---------------------------------------------------------------- workspace */

/* Bytes of device workspace needed to prepare every registered box with
 * smoothed boxes stored as `storage` (F32 or BF16 for F32 boxes, F64 for F64
 * boxes), evaluate up to `max_walkers` walkers per xs21_eval_batch launch
 * group, and run plain evaluations with up to `max_plain_radii` radii. */
xs21_status xs21_workspace_size(xs21_ctx* ctx, xs21_dtype storage, int max_walkers,
                                int max_plain_radii, size_t* bytes);

/* Computes, on the context stream, the forward FFT of every registered box
 * and every smoothed box delta_R of its shared ladder, and keeps them
 * resident in the workspace (the radius loop of Section 2.1 is independent of
 * the walker, so it runs once per box).  `workspace` is device memory of at
 * least xs21_workspace_size(...) bytes, 256-byte aligned, owned by the caller
 * and left untouched by anyone else until the context is destroyed.
 * ENOMEM: workspace too small; EINVAL: storage not allowed for a box dtype. */
xs21_status xs21_prepare(xs21_ctx* ctx, void* workspace, size_t bytes, xs21_dtype storage,
                         int max_walkers, int max_plain_radii);

/* Recomputes, on the context stream, the forward FFT and every smoothed box
 * of `box` from its resident density (the same work xs21_prepare does for
 * it).  With new_delta != NULL the resident density is first replaced by
 * new_delta (DEVICE, n^3 values of the box dtype, copied).  Asynchronous.
 * ESTATE: not prepared. */
xs21_status xs21_resmooth(xs21_ctx* ctx, xs21_box box, const void* new_delta);

/* ---------------------------------------------------------------- evaluation */

/* Batched evaluation on the resident smoothed boxes: for each walker w and
 * box b, the ionisation field (eq. 1 on the walker's suffix of the shared
 * ladder; partial ionisation at the cell radius), dT_b (eq. 4) and its binned
 * power spectrum.  Asynchronous on the context stream.
 * Outputs are DEVICE arrays: pk[nw][nb][n_bins_max] (P_b, mK^2 Mpc^3; bins past
 * a box's own n_bins are set to 0) and xhi_mean[nw][nb] (volume-weighted mean
 * neutral fraction); n_bins_max is the largest n_bins of the listed boxes.
 * Either output may be NULL.  Walkers are processed in groups of at most
 * max_walkers.  All listed boxes must share the dtype of the first.
 * EINVAL: bad walker values or box handles; ESTATE: not prepared. */
xs21_status xs21_eval_batch(xs21_ctx* ctx, const xs21_box* boxes, int nb,
                            const xs21_walker* walkers, int nw, double* pk, double* xhi_mean);

/* Plain evaluation of one walker on one box: the literal per-walker method.
 * The forward FFT and every smoothed box of the walker's own radius list are
 * recomputed (radii given explicitly, decreasing, last = cell radius; NULL
 * selects R_mfp / radius_step^i down to the cell size).  Synchronous.
 * Outputs are HOST arrays and each may be NULL: x_hi and dtb hold n^3 values
 * of the box dtype; pk, k_mean and counts hold n_bins doubles; xhi_mean one
 * double.  ENOMEM: more radii than max_plain_radii. */
xs21_status xs21_eval(xs21_ctx* ctx, xs21_box box, const xs21_walker* walker,
                      const double* radii, int n_radii, void* x_hi, void* dtb,
                      double* pk, double* k_mean, double* counts, double* xhi_mean);

/* Batched-path fields of one walker on one box, from the resident smoothed
 * boxes: the ionisation kernel of xs21_eval_batch runs over a group of this
 * one walker and writes the per-cell x_HI (Section 2.1, eq. 1 and the partial
 * ionisation at the cell radius) and dT_b (eq. 4) it transforms.  x_hi and
 * dtb are DEVICE arrays of n^3 values of the box dtype, both required.  Uses
 * the evaluation scratch of the workspace.  Asynchronous. */
xs21_status xs21_materialize(xs21_ctx* ctx, xs21_box box, const xs21_walker* walker,
                             void* x_hi, void* dtb);

/* xs21_eval_batch (same arguments, outputs and errors), and in the same
 * launches the x_HI and dT_b boxes of walker `field_walker` (an index into
 * walkers) on boxes[field_box] (an index into boxes): the ionisation launch
 * of that walker's group on that box also stores the per-cell values it
 * transforms.  x_hi and dtb: DEVICE, n^3 values of the box dtype each.  For
 * checking the batched kernel's per-cell output in its production launch
 * shape.  EINVAL: index out of range or a NULL field output. */
xs21_status xs21_eval_batch_fields(xs21_ctx* ctx, const xs21_box* boxes, int nb,
                                   const xs21_walker* walkers, int nw, double* pk,
                                   double* xhi_mean, int field_walker, int field_box,
                                   void* x_hi, void* dtb);

/* xs21_eval_batch for two-population walkers (Section 4, eq. 9).  The
 * criterion of eq. (1) weighs each collapsed halo by its own efficiency:
 * F(delta_R, R) = integral of zeta(M) over the extended Press-Schechter
 * conditional mass function between the 1e4 K halo mass and the mass of the
 * sphere; a cell is fully ionised where F >= 1 at some radius <= r_mfp, else
 * its ionised fraction is F at the cell radius; a sphere at or above delta_c
 * counts as one halo of its own mass.  Per (walker, box) a device pass turns
 * F >= 1 into an interval of delta_R per radius (F rises with delta_R to one
 * maximum, then falls towards delta_c) and tabulates F at the cell radius
 * (FP64 quadrature, relative error below 1e-9; the table's interpolation
 * error is below 1e-7).  Same outputs, layout and errors as
 * xs21_eval_batch. */
xs21_status xs21_eval_batch2(xs21_ctx* ctx, const xs21_box* boxes, int nb,
                             const xs21_walker2* walkers, int nw, double* pk, double* xhi_mean);

/* xs21_materialize for one two-population walker. */
xs21_status xs21_materialize2(xs21_ctx* ctx, xs21_box box, const xs21_walker2* walker,
                              void* x_hi, void* dtb);

/* Copies smoothed box `index` of the shared ladder of `box` into `out` (DEVICE,
 * n^3 values of the box dtype, converted from the storage type). Asynchronous. */
xs21_status xs21_smoothed(xs21_ctx* ctx, xs21_box box, int index, void* out);

/* Binned power spectrum (Section 2.2) of a caller-given real field on the
 * geometry of `box`, through the same FFT and binning kernels as the
 * evaluation.  field: DEVICE, n^3 values of the box dtype.  pk: HOST, n_bins
 * doubles.  Synchronous. */
xs21_status xs21_power_spectrum(xs21_ctx* ctx, xs21_box box, const void* field, double* pk);

/* y[i] = erfc(x[i]) for i < n by the single-precision complementary error
 * function the FP32 ionisation pass uses for the collapsed fraction of
 * Section 2.1 (f_coll = erfc((delta_c - delta_R) / sqrt(2 (S_min - S_R)))):
 * a degree-9 Chebyshev fit of erfc(z) exp(z^2) (Numerical Recipes, 2nd ed.,
 * section 6.2, fractional error below 1.2e-7) with the hardware's approximate
 * reciprocal and exponential.  x, y: DEVICE, n floats each.  Works on any
 * context, prepared or not.  Asynchronous. */
xs21_status xs21_erfc_f32(xs21_ctx* ctx, const float* x, float* y, long n);

/* xs21_power_spectrum for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels, with the spectrum, its Nyquist plane and the
 * partial bin sums in one statically allocated device array of 20 MiB per
 * device (the library holds it until the process ends) instead of the
 * workspace's evaluation scratch.  It allocates nothing and does not
 * synchronise.  field: DEVICE, n^3 values of the box dtype; pk_dev: DEVICE,
 * n_bins doubles (P_b as xs21_power_spectrum returns them).  Asynchronous on
 * the context stream.  EINVAL when the box needs more scratch than 20 MiB
 * (FP32 boxes up to 128^3 fit, FP64 boxes up to 64^3); the message gives both
 * sizes.  Every call on one device shares the array: calls that overlap on
 * one device (several streams or contexts) race and must be ordered by the
 * caller; nothing in the array needs clearing between calls. */
xs21_status xs21_power_spectrum_static(xs21_ctx* ctx, xs21_box box, const void* field, double* pk_dev);

/* Likelihood epilogue (Section 2.5; redshifts combined as in Section 3.4).
 * Sets the mock observation of `box`: delta2_mock[b] is the mock
 * Delta^2_21 (mK^2) on the box's own bins and noise_sigma[b] its
 * observational noise (mK^2; NULL = none).  A bin is fitted when it has modes
 * and its mean |k| (xs21_box_bins) lies in [k_lo, k_hi] Mpc^-1 (0.15 and 1.0
 * in the paper); its variance is noise^2 + (model_err * mock)^2
 * (model_err = 0.25 in the paper), and bins of zero variance are left out.
 * Both arrays are HOST, n_bins doubles, finite; model_err >= 0,
 * 0 <= k_lo <= k_hi.  Synchronous (the table is uploaded before returning). */
xs21_status xs21_set_mock(xs21_ctx* ctx, xs21_box box, const double* delta2_mock, const double* noise_sigma,
                          double model_err, double k_lo, double k_hi);

/* chi2[w] = sum over boxes[0..nb) and their fitted bins b of
 * (Delta^2_w,b - mock_b)^2 / variance_b, with Delta^2_w,b = k_b^3 P_w,b / (2 pi^2)
 * read from pk laid out as xs21_eval_batch writes it for the same box list
 * ([nw][nb][max n_bins], DEVICE).  chi2: DEVICE, nw doubles.  Every listed box
 * needs a mock (XS21_ESTATE otherwise).  Deterministic FP64; asynchronous. */
xs21_status xs21_chi2(xs21_ctx* ctx, const xs21_box* boxes, int nb, const double* pk, int nw, double* chi2);

/* ---------------------------------------------------------------- ensemble sampler */

/* The affine invariant ensemble sampler of Section 2.3 (Goodman & Weare
 * 2010, stretch move, the ensemble moved in two halves) on device-resident
 * walkers, in the paper's coordinates with temperatures as decimal
 * logarithms: dim = 3: rows (zeta, r_mfp, log10 t_vir); dim = 5: rows (zeta0,
 * r_mfp, log10 t_feed, alpha, beta) of the two-population model.  The prior
 * is uniform on the box lo <= x <= hi (first dim entries), which must lie
 * inside the valid parameter domain (zeta, r_mfp > 0; for dim = 5 also the
 * xs21_walker2 limits, 4 <= log10 t_feed <= 9); a is the stretch scale (2 in
 * the paper's sampler). */
typedef struct {
  int dim;
  double lo[5], hi[5];
  double a;
} xs21_sampler;

/* ln p of nw walkers x (DEVICE, [nw][dim] doubles) into lp (DEVICE, nw):
 * -chi^2 / 2 summed over the listed boxes (each needs xs21_set_mock) inside
 * the prior, -inf outside.  Walkers are planned and evaluated on the device
 * by the kernels of xs21_eval_batch / xs21_eval_batch2, in chunks of
 * max_walkers.  Asynchronous on the context stream. */
xs21_status xs21_mcmc_lnprob(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_sampler* s,
                             const double* x, int nw, double* lp);

/* One ensemble step, in place on the device: walkers [0, nw/2) move first,
 * then [nw/2, nw), each against the other half as it stands.  Walker k takes
 * partner j = floor(u0 * nw/2) of the other half, z = ((a - 1) u1 + 1)^2 / a,
 * proposal y = x_j + z (x_k - x_j), and moves (x, lp updated) when
 * ln u2 < (dim - 1) ln z + ln p(y) - lp[k].  u: DEVICE [2][nw/2][3] uniforms
 * in [0, 1) (first index: the half moving).  lp must hold ln p of x (from
 * xs21_mcmc_lnprob or the previous step).  accepted (DEVICE, nw int32, may be
 * NULL): 1 where the walker moved.  nw must be even and >= 4.  Asynchronous. */
xs21_status xs21_mcmc_step(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_sampler* s, double* x,
                           double* lp, int nw, const double* u, int32_t* accepted);

/* ---------------------------------------------------------------- kernel timing */

/* Kernel classes timed by xs21_profile_read. */
typedef enum {
  XS21_K_ROWS_R2C = 0,   /* x pass of a forward transform of a real box        */
  XS21_K_ROWS_C2R = 1,   /* x pass of an inverse transform (writes delta_R)   */
  XS21_K_AXIS_FWD = 2,   /* y or z pass of a forward transform                */
  XS21_K_AXIS_INV = 3,   /* y or z pass of an inverse transform (z: + filter) */
  XS21_K_AXIS_BINS = 4,  /* forward z pass fused with |X|^2 binning           */
  XS21_K_ION = 5,        /* per-cell ionisation + dT_b + forward x pass        */
  XS21_K_FINALIZE = 6,   /* FP64 reduction of bin and x_HI partial sums        */
  XS21_K_OTHER = 7,      /* materialisation and casts                          */
  XS21_K_PLAN = 8,       /* planning on the device (thresholds, tables)        */
  XS21_K_COUNT = 9
} xs21_kernel;

/* enable != 0: from now on every kernel launch of the context is bracketed by
 * HIP events on the context stream and its duration accumulated per class;
 * totals are cleared.  enable == 0: stop recording. */
xs21_status xs21_profile(xs21_ctx* ctx, int enable);

/* Synchronises the context stream, then returns for kernel class `kind` the
 * summed duration (ms), the number of launches, the summed algorithmic bytes
 * (the compulsory HBM reads + writes of each launch's inputs and outputs) and
 * the summed algorithmic vector operations of the per-cell pass
 * (XS21_K_ION only, else 0): per walker-cell one compare per radius the
 * walker filters at, 2.5 log2(N) for its share of the x-axis FFT and 6 for
 * the brightness temperature, packing and unpacking.  Any output pointer may
 * be NULL. */
xs21_status xs21_profile_read(xs21_ctx* ctx, int kind, double* total_ms, long long* launches, double* bytes,
                              double* ops);

/* HBM bandwidth probe: the practical ceiling beside the 8 TB/s peak for the
 * path's memory-bound passes.  kind 0: read every 16-byte vector of the
 * buffer once; 1: write it; 2: copy the first half to the second; 3: read it
 * as 256^3 FP32 half spectra (rows padded to 144 complex values) in strided
 * 128-byte segments over all z planes, the access pattern of the binning
 * pass.  buf: DEVICE, `bytes` >= 1 MiB plus 32 KiB (kind 3: at least one
 * spectrum of 75.5 MB plus 32 KiB), 256-byte aligned, contents overwritten;
 * its last 32 KiB hold the read kernels' block sums.  One untimed launch,
 * then `reps` launches timed with HIP events on the context stream.
 * *gbps: bytes read plus written per second (1e9); *bytes_per_launch (may be
 * NULL): those bytes for one launch.  Synchronous. */
xs21_status xs21_probe_bandwidth(xs21_ctx* ctx, int kind, void* buf, size_t bytes, int reps,
                                 double* gbps, double* bytes_per_launch);

/* ---------------------------------------------------------------- launch shapes */

/* Launch shapes of the batched evaluation for boxes of one grid size (0, or
 * -1 for flag_test, selects the built-in default).  Results do not depend on
 * them except through the order of floating-point sums (the flag test is
 * exact either way). */
typedef struct {
  int32_t ion_blocks;   /* blocks of the ionisation pass, <= 16384 (default 8192, or n^2/2 if fewer) */
  int32_t pipe_blocks;  /* blocks of the pipelined strided passes and smoothing rows (default 2048) */
  int32_t bins_blocks;  /* blocks of one binning launch over a walker group (default 2048) */
  int32_t flag_test;    /* FP32 boxes: 1 sorted-threshold search per radius for the whole walker
                           group (two for two-population walkers: lower and upper interval
                           ends), 0 one compare per walker and radius (two for intervals) */
  int32_t group;        /* walkers per ionisation launch, <= 64 and <= max_walkers (default min of both) */
} xs21_tuning;

/* Sets (t != NULL) or clears (t == NULL) the launch shapes used for boxes of
 * n^3 cells.  EINVAL: n not a power of two in [8, 512], values out of range. */
xs21_status xs21_set_tuning(xs21_ctx* ctx, int n, const xs21_tuning* t);

/* The launch shapes set for n (zeros / -1 where the defaults apply). */
xs21_status xs21_get_tuning(xs21_ctx* ctx, int n, xs21_tuning* t);

/* Chooses launch shapes for the listed boxes (one grid size) by timing
 * xs21_eval_batch of `walkers` on them with HIP events (best of `reps` runs
 * after a warm-up per candidate; coordinate descent from the defaults over
 * the flag test, the ionisation grid, the walker group, the pipelined grid and
 * the binning grid; a candidate must win by more than 1 %), and sets them for
 * that size.  With cache_path != NULL the choice is stored in that JSON file
 * under the key "arch|n=N|dtype|storage|nr=N_R|g=G" (device architecture,
 * grid size, box dtype, smoothed-box storage, ladder length, walker group),
 * and a later call finds it there without timing (*from_cache = 1).  Outputs
 * may be NULL: the chosen shapes, the best batch time (ms; from the cache
 * when cached).  Synchronous; not allowed during graph capture. */
xs21_status xs21_autotune(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_walker* walkers,
                          int nw, int reps, const char* cache_path, xs21_tuning* chosen,
                          double* best_ms, int* from_cache);

/* ---------------------------------------------------------------- launch graphs */

typedef struct xs21_graph xs21_graph;

/* Records the device work of the following calls on the context stream into a
 * launch graph instead of running it (the stream must be a created stream,
 * not the null stream; kernel timing must be off).  Only calls whose work is
 * all on the device may be recorded: xs21_mcmc_lnprob, xs21_mcmc_step,
 * xs21_chi2, xs21_resmooth, xs21_smoothed, xs21_power_spectrum_static,
 * xs21_erfc_f32.  The others return XS21_ESTATE while capturing.  Device
 * buffers named by the recorded calls are read and written again, at the same
 * addresses, every time the graph is launched: e.g. a recorded
 * xs21_mcmc_step advances the chain by one step per launch with the uniforms
 * the caller has placed in `u` by then. */
xs21_status xs21_capture_begin(xs21_ctx* ctx);

/* Ends the recording and instantiates the graph (*out). */
xs21_status xs21_capture_end(xs21_ctx* ctx, xs21_graph** out);

/* Launches a recorded graph on the context stream.  Asynchronous. */
xs21_status xs21_graph_launch(xs21_ctx* ctx, const xs21_graph* g);

/* Releases a graph.  NULL is accepted. */
xs21_status xs21_graph_destroy(xs21_graph* g);

/* ---------------------------------------------------------------- host planning */
/* Pure host functions (no device, no context): the FP64 scalar planning the
 * kernels consume, exposed so it can be checked on its own. */

/* Radius ladder R_i = r_top / step^i while R_i > r_cell, then r_cell. */
xs21_status xs21_plan_ladder(double r_top, double r_cell, double step, double* out, int cap,
                             int* n_radii);

/* sigma^2(R, z) of the sharp-k window on the linear spectrum of `phys`. */
xs21_status xs21_plan_sigma2(const xs21_physics* phys, double radius, double z, double* out);

/* Per-radius flag thresholds of one walker at redshift z over `radii`
 * (decreasing, last = cell radius).  thr[j]: a cell is fully ionised at
 * radius j when delta_R >= thr[j] (the exact rewrite of zeta f_coll >= 1 via
 * the inverse of erfc); +inf where no cell can be (sigma^2(M_min) <=
 * sigma^2(R_j) or zeta <= 1/2).  dsig2[j] = sigma^2(M_min) - sigma^2(R_j).
 * *first: index of the first radius <= r_mfp.  *m_min: M_min in Msun.
 * Any output pointer may be NULL. */
xs21_status xs21_plan_walker(const xs21_physics* phys, double z, const double* radii,
                             int n_radii, const xs21_walker* walker, double* thr,
                             double* dsig2, int* first, double* m_min);

/* Bin index of every integer |n|^2 in [0, 3 (n/2)^2] (-1 = dropped). out
 * holds 3 (n/2)^2 + 1 entries. */
xs21_status xs21_plan_bins(int n, int n_bins, int8_t* out);

#ifdef __cplusplus
}
#endif
#endif /* XS21_H */
