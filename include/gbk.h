/*
 * gbk.h -- C ABI of the MI355X (gfx950) library libgbk.so: batched likelihood
 * evaluation of the thin-disc intensity-cube model of Bekiaris, Glazebrook,
 * Fluke & Abraham (2016), "Kinematic modelling of disc galaxies using
 * graphics processing units", and the optimisers that call it.
 *
 * One evaluation = model cube (Sec. 2.1 eqs. 1-8, Sec. 2.2.2) -> convolution
 * with the PSF and LSF (eq. 9, Sec. 2.2.3) -> down-sampling by the
 * upsampling factor (Sec. 2.2.4) -> moment maps (Sec. 2.2.5) -> masked
 * goodness of fit (eq. 11, Sec. 2.2.6).
 *
 * Conventions (fixed for every entry point):
 *  - angles in degrees, lengths in data pixels, velocities in km/s;
 *  - data pixel (i, j) is centred at (x, y) = (i, j), x along the fastest
 *    axis of every map; maps are row-major [ny][nx];
 *  - data channel k has velocity v0_kms + (k - crpix) * dv_kms; with
 *    upsampling u the model grid is u times finer along x, y and velocity,
 *    fine pixel m sitting at (m + 1/2)/u - 1/2 in data units;
 *  - the PSF is a circular Gaussian of the given FWHM (data pixels), the LSF
 *    a Gaussian of the given sigma (km/s); each axis is sampled at integer
 *    fine-grid offsets -h..h, h = ceil(R * sigma), and normalised to unit
 *    sum; 0 switches an axis off;
 *  - the model is evaluated on the data window plus a halo of h fine pixels
 *    (channels) on each side and every convolution is "valid";
 *  - line profile: I(r) times a unit-area Gaussian of width sigma_model
 *    sampled at channel centres, I(r) = I0 exp(-min(r/r0, 60));
 *  - m0 = dv * sum C, m1 = sum C v / sum C, m2 = sqrt(sum C (v - m1)^2 / sum C)
 *    over the data channels; sum C == 0 gives (0, Vsys, 0);
 *  - chi2 = sum over mask != 0 of (m1 - v_obs)^2 / E_v^2 + W (m2 - s_obs)^2 / E_s^2.
 *
 * Parameter rows are 12 doubles (GK_NP), in the slot order of the enum below.
 * A row outside the model's domain (non-finite value, inclination outside
 * (0, 90), sigma <= 0, r0 <= 0, rt <= 0, I0 <= 0, or for the Epinat curve
 * g <= 0 or a < 0) evaluates to NaN maps and chi2 = +inf.
 *
 * Memory: `params` may be host or device memory (told apart with
 * hipPointerGetAttributes); outputs named "device" must be device memory
 * owned by the caller.  Observations are copied into library-owned device
 * memory.  Work is enqueued on the caller's HIP stream (NULL = the null
 * stream) and the call returns without waiting, except where stated.
 * Calls on one model from several host threads, or overlapping calls on
 * different streams, race on the model's scratch memory: serialise them.
 * No C++ exception crosses this interface; on failure the entry points
 * return a negative gk_status and gk_last_error() describes it.
 */
#ifndef GBK_H
#define GBK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gk_model gk_model; /* opaque, created and freed by the library */

typedef enum {
    GK_OK = 0,
    GK_PARTIAL = 1,     /* some host-given rows are out of domain (their chi2 = +inf, maps NaN) */
    GK_EINVAL = -1,     /* invalid argument: descriptor, observation, pointer kind, size */
    GK_ENOMEM = -2,     /* device or host allocation failed */
    GK_EDEVICE = -3,    /* HIP runtime error */
    GK_ENOTCONV = -4,   /* an optimiser stopped at its iteration cap */
    GK_ESTATE = -5      /* call out of order (e.g. chi2 before an observation is set) */
} gk_status;

/* Parameter slots (Sec. 2.1): kinematic centre, position angle, inclination,
 * systemic velocity, rotation-curve velocity and turn-over radius, intrinsic
 * dispersion (Sec. 2.1.4), exponential-disc scale length and central
 * brightness (eq. 5), Epinat outer and inner slopes a, g (eq. 7). */
enum { GK_XO = 0, GK_YO, GK_PA, GK_INC, GK_VSYS, GK_VT, GK_RT, GK_SIG, GK_R0, GK_I0, GK_A, GK_G,
       GK_NP };

/* Rotation curves: arctan (eq. 6), Epinat (eq. 7), exponential rise
 * Vt (1 - exp(-r/rt)). */
enum { GK_RC_ARCTAN = 0, GK_RC_EPINAT = 1, GK_RC_BOISSIER = 2 };

typedef struct {
    int32_t nx, ny, nz;          /* data grid, each >= 1 */
    int32_t upsample;            /* u >= 1 (Sec. 2.2.2, eq. 10) */
    double dv_kms;               /* channel width, > 0 */
    double v0_kms, crpix;        /* v_k = v0 + (k - crpix) dv */
    double psf_fwhm_pix;         /* >= 0; 0 = no PSF */
    double lsf_sigma_kms;        /* >= 0; 0 = no LSF */
    double kernel_radius_sigma;  /* R > 0 (4 is the usual choice) */
    int32_t rc;                  /* GK_RC_* */
    int32_t conv_mode;           /* GK_CONV_*: how the spatial PSF convolution runs */
    int32_t strategy;            /* GK_STRATEGY_*: 0 (zero-initialised) = the cube strategy */
} gk_model_desc;

/* Spatial PSF convolution: AUTO takes the direct LDS-tiled passes while the
 * PSF half-width fits them (at most 16 fine pixels for the register-blocked
 * u = 1 kernel, the LDS budget otherwise) and the FFT path beyond; DIRECT
 * and FFT force one (DIRECT fails for a PSF too wide for LDS).  The FFT path
 * convolves along x, then along y, with radix-2 FFTs of the next power of
 * two >= the padded extent (eq. 10) in FP64; its results equal the direct
 * path's up to rounding of order log2(P) * 1e-16 of the largest plane value. */
enum { GK_CONV_AUTO = 0, GK_CONV_DIRECT = 1, GK_CONV_FFT = 2 };

/* Modelling strategy (Sec. 2.2).  GK_STRATEGY_CUBE is the chain described at
 * the top of this header.  GK_STRATEGY_VFIELD is the velocity-field strategy
 * of Sec. 2.2.1: the model of eq. 8 is evaluated at every data pixel centre
 * (x, y) = (i, j), and the cube, convolution, down-sampling and moment steps
 * are skipped, so the evaluation goes straight to eq. 11.  Its maps are
 * [3][ny][nx] = surface brightness I(r) (eq. 5), line-of-sight velocity
 * (eq. 8) and the intrinsic dispersion sigma (the dispersion map of a disc
 * without beam smearing), FP64 inside and stored as FP32; its residuals and
 * chi-square are those of eq. 11 with these maps in place of m1 and m2 (an
 * observation set with W = 0 compares the velocity field alone).  It needs
 * upsample = 1 and no PSF or LSF; nz, dv_kms, v0_kms, crpix,
 * kernel_radius_sigma and conv_mode are not used.  Parameter rows and their
 * domain are the same as for the cube strategy.  The evaluation calls, the
 * fitters (LM, nested sampling, nested grids), graphs and profiling (kernel
 * index 1 = the velocity-field kernel; no voxel count) accept such models;
 * surveys whose models all use this strategy, and gk_mc_errors accept such
 * models; gk_surrogate_create, gk_autotune, gk_set_conv_config and
 * gk_model_conv_path return GK_EINVAL for them. */
enum { GK_STRATEGY_CUBE = 0, GK_STRATEGY_VFIELD = 1 };

/* Creates a model for one instrument grid on HIP device `device`.
 * Limits of the cube strategy: upsample 1..8; at most 65534 fine channels with
 * the LSF halo (nz * upsample + 2 h_lsf); the fine grid with the PSF halo
 * (nx * upsample + 2 h_psf by ny * upsample + 2 h_psf) under 2^28 spaxels,
 * i.e. one FP64 plane of it under 2^31 bytes (the kernels address a plane
 * with 32-bit byte offsets).
 * Errors: GK_EINVAL (bad descriptor or a limit exceeded), GK_ENOMEM, GK_EDEVICE. */
gk_status gk_create_model(const gk_model_desc *desc, int device, gk_model **out);

/* Frees the model and its device memory; waits for its pending work.  NULL is a no-op. */
gk_status gk_destroy_model(gk_model *model);

/* Sets the observed maps (Sec. 2.2, Sec. 2.2.6): velocity, dispersion and
 * their errors, [ny][nx] float host arrays, a [ny][nx] byte mask (nonzero =
 * use the pixel) and the dispersion weight W >= 0 of eq. 11.  The data are
 * copied; the call blocks until the copy is done.  `sig`/`esig` may be NULL
 * only when W == 0.  Errors: GK_EINVAL if an unmasked pixel has a non-finite
 * value or an error <= 0 (E_s only checked when W > 0). */
gk_status gk_set_observation(gk_model *model, const float *vel, const float *sig,
                             const float *evel, const float *esig, const uint8_t *mask,
                             double W);

/* Number of unmasked pixels of the current observation (host value). */
gk_status gk_observation_count(const gk_model *model, int64_t *n_valid);

/* Evaluates B parameter rows `params` [B][GK_NP] (host or device) into the
 * device array `maps` [B][3][ny][nx] float: m0, m1, m2 of each row
 * (Sec. 2.2.2-2.2.5).  Returns GK_PARTIAL when host-given rows are out of
 * domain; rows given in device memory are checked on the device only (their
 * maps become NaN, the status stays GK_OK).  B == 0 is a no-op. */
gk_status gk_evaluate_batch(gk_model *model, const double *params, int32_t B, float *maps,
                            void *hip_stream);

/* Masked chi-square (eq. 11) of B rows against the current observation:
 * chi2 [B] double and, if not NULL, n_valid [B] int64 (unmasked pixels
 * counted; 0 for an out-of-domain row), both device arrays.  The sums are
 * double precision and reduced in a fixed order, so repeated calls give
 * bit-identical results.  Errors: GK_ESTATE without an observation. */
gk_status gk_chi2_batch(gk_model *model, const double *params, int32_t B, double *chi2,
                        int64_t *n_valid, void *hip_stream);

/* Weighted residual maps for least squares (Sec. 2.3.1): resid [B][2][ny][nx]
 * double device array, (m1 - v_obs)/E_v and sqrt(W) (m2 - s_obs)/E_s on
 * unmasked pixels and 0 elsewhere; the sum of squares of a row is its chi2.
 * Out-of-domain rows are filled with NaN.  Errors: GK_ESTATE without an
 * observation. */
gk_status gk_residual_batch(gk_model *model, const double *params, int32_t B, double *resid,
                            void *hip_stream);

/* Allocation-free chi-square, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * gk_chi2_batch, but the per-row scratch (row constants, T_j planes,
 * chi-square tile partials, FFT x-pass planes) lives in one fixed device
 * array of GK_NOALLOC_SCRATCH_BYTES per GPU, part of the library's device
 * code and held by every GPU the call has run on until the process ends;
 * batches larger than it holds run in chunks on the caller's stream.  The call
 * makes no hipMalloc, hipFree, pinned staging or graph (its first call on a
 * GPU looks the array's address up once).  params, chi2 and n_valid
 * (nullable) must be device memory.  All calls on one GPU share its array, so
 * calls that overlap on one GPU (other streams or threads without ordering
 * between them) race and give undefined results; the array keeps the last
 * call's contents, none of which the next call reads.  Errors: GK_EINVAL for
 * host rows or outputs, or a model one of whose rows needs more scratch than
 * the array holds (about 5.5 M halo-extended fine spaxels); GK_ESTATE without
 * an observation. */
#define GK_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
gk_status gk_chi2_batch_noalloc(gk_model *model, const double *params, int32_t B,
                                double *chi2, int64_t *n_valid, void *hip_stream);

/* Measurement hooks for the benchmark (not needed for correct results).
 * flags: GK_PROF_TIMING brackets every kernel launch of the following calls
 * with HIP events on the caller's stream; GK_PROF_COUNT makes the line-profile
 * kernel count, per row, the fine voxels inside each spaxel's line support
 * (channels within sqrt(40 / kappa) of the line centre, i.e. where the
 * Gaussian of Sec. 2.2.2 exceeds 2^-40 of its peak), which is the work the
 * evaluation has to do.  Counting adds atomics, so it is meant for an
 * untimed pass.  gk_read_profile waits for the recorded work, returns the
 * totals since the last read and clears them.  Kernel index: 0 = per-row
 * constants, 1 = line profiles, 2 = PSF passes + moments + chi-square terms,
 * 3 = chi-square reduction. */
enum { GK_PROF_TIMING = 1, GK_PROF_COUNT = 2 };
typedef struct {
    double kernel_ms[4];        /* summed kernel durations */
    int64_t launches[4];        /* launches timed */
    int64_t support_voxels;     /* counted line-support voxels (GK_PROF_COUNT) */
    int64_t rows;               /* rows evaluated while profiling */
} gk_profile_stats;
gk_status gk_set_profiling(gk_model *model, int flags);
gk_status gk_read_profile(gk_model *model, gk_profile_stats *out);

/* ---- Levenberg-Marquardt (Sec. 2.3.1) ----------------------------------
 * Damped Gauss-Newton on the residuals of gk_residual_batch with box
 * constraints.  Jacobian column a of a free slot: (r(p+) - r(p-)) / (p+ - p-),
 * p+- = p_a +- fd_step clipped to [lo_a, hi_a] (the paper uses an absolute
 * step of about 0.1, Sec. 4).  A = J^T J and g = J^T r are formed in FP64;
 * the step (A + lambda diag A) d = -g is solved by Cholesky in FP64, trial =
 * clip(p + d).  A trial that lowers chi2 is accepted (lambda /= 10),
 * otherwise lambda *= 10.  Free slots whose Jacobian column is identically
 * zero (e.g. I0, which only scales the cube) are frozen.  Each iteration is
 * one batched launch of 1 + 2 n_free rows: the trial point and the Jacobian
 * rows around it (used if the trial is accepted).  gk_fit_lm runs the whole
 * iteration on the device (the step rule in one GPU thread, no host round
 * trip), eight iterations per HIP graph replay in the graph launch mode; the
 * survey LM keeps the rule on the host; both give the same result. */
typedef struct {
    int32_t max_iter;   /* trials; default 200 */
    int32_t reserved;   /* must be 0 */
    double fd_step;     /* absolute finite-difference step in ABI units; default 0.1 */
    double lambda0;     /* initial damping; default 1e-3 */
    double ftol;        /* stop when the relative chi2 decrease <= ftol; default 1e-10 */
    double xtol;        /* stop when max |d_a| / (|p_a| + 1e-10) <= xtol; default 1e-10 */
} gk_lm_opts;

enum { GK_LM_FTOL = 1, GK_LM_XTOL = 2, GK_LM_LAMBDA = 3, GK_LM_MAXITER = 4 };

typedef struct {
    double chi2;              /* at the returned parameters */
    int64_t n_valid;          /* unmasked pixels */
    int32_t iterations;       /* trials made */
    int32_t reason;           /* GK_LM_* */
    int64_t n_evals;          /* parameter rows evaluated */
    double errors[GK_NP];     /* sqrt(diag((J^T J)^-1)) of free slots, 0 elsewhere */
} gk_lm_result;

/* Fills opts with the defaults above. */
gk_status gk_lm_default_opts(gk_lm_opts *opts);

/* Fits p_inout [GK_NP] (host, start values in, optimum out) with the slots
 * where free_mask[k] != 0 free inside [lo_k, hi_k] (host arrays; NULL bounds
 * mean unbounded).  Blocks until done; runs on a stream of the model's own.
 * Needs an observation (GK_ESTATE otherwise).  Returns GK_OK, or GK_ENOTCONV
 * when max_iter was reached (the result is still filled), or an error; a
 * start outside the model's domain is GK_EINVAL.  opts may be NULL. */
gk_status gk_fit_lm(gk_model *model, double *p_inout, const uint8_t *free_mask, const double *lo,
                    const double *hi, const gk_lm_opts *opts, gk_lm_result *result);

/* ---- Nested sampling (Sec. 2.3.2) -----------------------------------------
 * Nested sampling (Skilling 2004) over a uniform prior box with an
 * ellipsoidal bound (Mukherjee et al. 2006; several ellipsoids as in
 * MultiNest, Feroz et al. 2009).  N live points; L = exp(-chi2/2).  Each round
 * bounds the live points by an ellipsoid (covariance scaled to enclose them
 * all, volume enlarged by `enlarge`), split recursively in two by 2-means
 * while the two children's volumes sum to under half the parent's (each child
 * keeping >= 2 (d + 1) points, at most max_ell ellipsoids, none smaller than
 * the prior volume n_e X_k / N of its points), rebuilt after every N/20
 * retired points from the live points at the start of a round and used from
 * the next round on (an older bound still encloses the shrinking constrained
 * region); draws a batch of candidates
 * uniformly over the union inside the box, evaluates them in one launch, and
 * consumes them in draw order: a candidate whose L
 * exceeds the current lowest live L replaces that point, which is retired with
 * prior-volume weight X_{k-1} - X_k, X_k = exp(-k/N).  Stops when
 * log(Z + L_max X_k) - log Z < tol, then adds the live points with weight X_k/N.
 * Batch: `batch` candidates per round, or, with batch_max > batch, as many
 * as should give about accept_target (default N/10) acceptances at the
 * acceptance rate of the last two rounds, within [batch, batch_max] (fewer,
 * larger launches when the
 * bound fits the constrained region poorly; the candidates of a round are
 * still drawn from a bound that encloses the region, so the sampler's
 * statistics are those of the fixed batch).
 * Random numbers: Philox4x32-10 (Salmon et al. 2011) keyed by `seed`. */
typedef struct {
    int32_t n_live;      /* default 400 */
    int32_t batch;       /* candidates per launch; default n_live */
    int64_t max_iter;    /* retired points; default 1e6 */
    double enlarge;      /* ellipsoid volume factor; default 1.25 (= 1/e with e = 0.8) */
    double tol;          /* evidence tolerance; default 0.5 */
    uint64_t seed;       /* default 1 */
    int32_t max_ell;     /* ellipsoids of the bound, 1..8; default 8 (1: one ellipsoid) */
    int32_t batch_max;   /* adaptive batch ceiling (>= batch; 0: fixed batch); default 0 */
    int32_t accept_target; /* acceptances per round the adaptive batch aims at (>= 0;
                              0: N/10); default 0 */
    /* gk_fit_nested_screened only: a round of n candidates skips the screen
     * (every candidate gets the plain chi2) unless (1 - f) n > screen_cost n +
     * screen_rows, f = the pass fraction of the last screened round; every
     * 8th round is screened regardless.  screen_cost = cost of a surrogate
     * row in plain rows, screen_rows = the screen's fixed cost per round in
     * plain rows; default 0 and 0 (every round screened). */
    double screen_cost;
    int32_t screen_rows;
    /* 1: mode separation (MultiNest's, simplified; Sec. 2.3.2).  When the
     * ellipsoids of a mode's decomposition fall into groups that do not
     * intersect, the mode splits into one mode per group (its live points and
     * prior volume shared out in proportion to their points), and each mode
     * then runs as a nested sampler of its own: a candidate drawn from a
     * mode's ellipsoids (uniform over that mode's union, modes picked by
     * volume) replaces that mode's lowest live point if its L is higher, and
     * the mode's volume shrinks by exp(-1/n_m).  A mode stops receiving
     * candidates once its remaining evidence L_max X_m is below
     * (e^tol - 1) Z / (number of modes); the run ends when every mode has
     * stopped.  Local evidence of a mode = its own retired and final live
     * points plus its ancestors' evidence shared out by live points at each
     * split.  At most GK_NS_MAX_MODES modes.  Meant for posteriors known to
     * have separated modes: a connected but curved contour can also split,
     * and its pieces may then count the same region twice.  0 (default): one
     * mode. */
    int32_t separate_modes;
    /* > 0: stop after this much wall time (checked after each round), as if
     * max_iter had been reached (GK_ENOTCONV, results from the points so
     * far); 0 (default): no limit */
    double max_wall_s;
} gk_ns_opts;

/* Per-mode results (gk_ns_result.modes). */
#define GK_NS_MAX_MODES 8
typedef struct {
    double logz, logz_err;     /* local evidence and sqrt(H_m / n_m) */
    double info_h;             /* information of the mode's own points (nats) */
    int64_t n_live;            /* live points of the mode */
    int64_t n_samples;         /* posterior points of the mode (its own, weight > 0) */
    double mean[GK_NP], sd[GK_NP];                 /* over the mode's own points */
    double median[GK_NP], q16[GK_NP], q84[GK_NP];
} gk_ns_mode;

typedef struct {
    double logz, logz_err;     /* log evidence and sqrt(H / N) */
    double info_h;             /* information H (nats) */
    double max_logl;           /* best log-likelihood seen */
    int64_t n_iter;            /* retired points */
    int64_t n_evals;           /* likelihood evaluations */
    int64_t n_launches;        /* batched launches */
    double best[GK_NP];        /* best point */
    double mean[GK_NP], sd[GK_NP];            /* posterior mean and standard deviation */
    double median[GK_NP], q16[GK_NP], q84[GK_NP];  /* posterior quantiles */
    /* surrogate screening (gk_fit_nested_screened; 0 otherwise) */
    int64_t n_screened;        /* candidates judged by the surrogate */
    int64_t n_rejected;        /* of those, discarded without a plain evaluation */
    int64_t n_audited;         /* discarded ones evaluated anyway (audit draws) */
    int64_t n_audit_miss;      /* audited ones that the plain chi2 would have accepted */
    double t_wall_s;           /* wall time of the call (model fits; 0 for gk_nested_sample) */
    double t_wait_s;           /* of which blocked waiting for the device */
    int32_t n_modes;           /* final modes (1 without mode separation) */
    int32_t reserved_modes;
    gk_ns_mode modes[GK_NS_MAX_MODES];  /* the first n_modes are filled */
} gk_ns_result;

gk_status gk_ns_default_opts(gk_ns_opts *opts);

/* Samples the posterior of the model's parameters against the current
 * observation.  Slots with free_mask[k] != 0 have the uniform prior
 * [lo_k, hi_k]; the others are fixed at fixed[k] (host arrays).  Blocks.
 * Posterior arrays of fixed slots hold the fixed value.  If samples is not
 * NULL, up to cap weighted posterior samples are written as rows of GK_NP + 1
 * doubles (the parameters, then the normalised weight) and their count to
 * *n_samples.  GK_ENOTCONV when max_iter was reached (result still filled). */
gk_status gk_fit_nested(gk_model *model, const double *lo, const double *hi,
                        const uint8_t *free_mask, const double *fixed, const gk_ns_opts *opts,
                        gk_ns_result *result, double *samples, int64_t cap, int64_t *n_samples);

/* Batch log-likelihood for gk_nested_sample: theta [n][dim] -> logl [n];
 * returns 0 on success (non-zero aborts the run with GK_EINVAL). */
typedef int (*gk_loglike_fn)(const double *theta, int32_t n, int32_t dim, double *logl, void *user);

/* The same sampler over any batch likelihood of dim <= GK_NP parameters with
 * the uniform prior [lo, hi]; result arrays use their first dim entries. */
gk_status gk_nested_sample(int32_t dim, const double *lo, const double *hi, gk_loglike_fn fn,
                           void *user, const gk_ns_opts *opts, gk_ns_result *result,
                           double *samples, int64_t cap, int64_t *n_samples);

/* Philox4x32-10 block function (for reproducibility checks): out = philox(ctr, key). */
gk_status gk_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ---- Nested grids (Sec. 2.3.3) -------------------------------------------
 * Brute-force search on a regular grid of n nodes per free slot (end points
 * included) spanning the current box; the node of least chi2 (ties: lowest
 * linear node index, first free slot varying slowest) centres the next box,
 * which is that node +- one grid spacing clipped to the initial box.  Each
 * level's n^d nodes are generated on the device and evaluated in batched
 * launches; the argmin is reduced on the device.  Stops after max_levels or
 * when every free slot's spacing is below accuracy[k]. */
typedef struct {
    double best[GK_NP];       /* best node of the last level */
    double chi2;              /* its chi2 */
    int64_t best_index;       /* its linear node index within the last level */
    int32_t levels;           /* levels run */
    int32_t reserved;
    int64_t n_evals;          /* rows evaluated */
    double spacing[GK_NP];    /* grid spacing of the last level per slot */
} gk_grid_result;

/* Free slots: free_mask[k] != 0 searched in [lo_k, hi_k]; others fixed at
 * fixed[k].  n_per_dim >= 2; n_per_dim^(free slots) <= 2^31 nodes per level.
 * accuracy may be NULL (then only max_levels stops).  Blocks. */
gk_status gk_fit_grid(gk_model *model, const double *lo, const double *hi,
                      const uint8_t *free_mask, const double *fixed, int32_t n_per_dim,
                      int32_t max_levels, const double *accuracy, gk_grid_result *result);

/* The same search with n_per_slot[k] >= 2 nodes along each free slot k
 * (n_per_slot [GK_NP], entries of fixed slots ignored), as the paper's grids
 * of different resolution per parameter (Sec. 4: 7, 11, 11, 5, 5, 5 nodes for
 * PA, r_t, V_t, sigma, a, g).  Node index = mixed-radix number of the free
 * slots' node indices, first free slot most significant; the product of the
 * counts <= 2^31.  gk_fit_grid is this call with every count n_per_dim. */
gk_status gk_fit_grid_nd(gk_model *model, const double *lo, const double *hi,
                         const uint8_t *free_mask, const double *fixed, const int32_t *n_per_slot,
                         int32_t max_levels, const double *accuracy, gk_grid_result *result);

/* ---- Surveys: ragged batches over many models -----------------------------
 * A survey groups models (galaxies with their own grids, PSFs and
 * observations) on one device.  A batch lists (model, parameter row) pairs of
 * any mix of models; every row is evaluated in the same launch chain, each
 * kernel locating its (row, tile) in the ragged work list. */
typedef struct gk_survey gk_survey;

/* models [n] must stay alive (and on one device) while the survey is used;
 * their observations are read at each call.  All models of a survey use one
 * strategy; cube models must run the direct convolution path.
 * Errors: GK_EINVAL. */
gk_status gk_create_survey(gk_model *const *models, int32_t n, gk_survey **out);
gk_status gk_destroy_survey(gk_survey *survey);

/* chi2 [B] (device) of rows params [B][GK_NP] (host or device) of models
 * model_idx [B] (host).  Every model needs an observation (GK_ESTATE). */
gk_status gk_survey_chi2(gk_survey *survey, const int32_t *model_idx, const double *params,
                         int32_t B, double *chi2, void *hip_stream);

/* Levenberg-Marquardt (the rule of gk_fit_lm) of every galaxy of the survey
 * at once: each iteration evaluates all unconverged galaxies' trial points and
 * Jacobian rows in one ragged launch chain and forms their normal equations in
 * one kernel; converged galaxies drop out.  p_inout [n][GK_NP], lo/hi
 * [n][GK_NP] (NULL = unbounded), free_mask [GK_NP] shared, results [n].
 * Blocks.  GK_ENOTCONV if some galaxy reached max_iter. */
gk_status gk_fit_lm_survey(gk_survey *survey, double *p_inout, const uint8_t *free_mask,
                           const double *lo, const double *hi, const gk_lm_opts *opts,
                           gk_lm_result *results);

/* Nested grids (gk_fit_grid_nd) of every galaxy of the survey at once: lo, hi
 * and fixed are [n][GK_NP] (galaxy g's box and fixed values), free_mask,
 * n_per_slot and accuracy [GK_NP] are shared (accuracy may be NULL).  Each
 * level evaluates the nodes of every galaxy still refining in ragged
 * launches of up to 2^20 rows (galaxy-major, each galaxy's nodes in index
 * order) and reduces each galaxy's least-chi2 node on the device; a galaxy
 * whose every spacing is below accuracy stops.  results [n]; each equals what
 * gk_fit_grid_nd gives for that galaxy's model alone (same chi-square,
 * same ties).  Blocks. */
gk_status gk_fit_grid_survey(gk_survey *survey, const double *lo, const double *hi,
                             const uint8_t *free_mask, const double *fixed,
                             const int32_t *n_per_slot, int32_t max_levels, const double *accuracy,
                             gk_grid_result *results);

/* ---- Learned surrogate of the moment maps (not part of the paper) ----------
 * A multilayer perceptron maps a parameter row to the velocity and dispersion
 * maps of one instrument (the grid, PSF and LSF of the model it is created
 * from).  Inputs: slots x0 y0 PA i Vsys Vt rt sigma r0 I0, each scaled from
 * the box [lo, hi] to [-1, 1] (0 where lo == hi), PA as (cos PA, sin PA),
 * zero-padded to 32.  `layers` hidden layers of width `hidden` with the exact
 * GELU z Phi(z); a linear output layer of 2 nx ny values: m1 / 300 then
 * m2 / 100 (km/s), row-major.  Weights and activations BF16, products on the
 * matrix cores with FP32 accumulation, FP32 master weights.
 * Training minimises sum mask (y - t)^2 / sum mask with Adam (beta 0.9 /
 * 0.999, eps 1e-8), where t are the plain evaluation's maps of rows drawn
 * uniformly in the box on the device (Philox4x32-10 keyed by `seed`) and
 * mask marks spaxels whose flux is at least 1% of the row's peak.
 * Initial weights: He normal for hidden layers, 1/sqrt(fan-in) for the
 * output layer, zero biases.  The surrogate keeps a pointer to the model:
 * the model must outlive it, and calls on one surrogate must not overlap. */
typedef struct gk_surrogate gk_surrogate;

typedef struct {
    int32_t hidden;     /* width, multiple of 32; default 1024 */
    int32_t layers;     /* hidden layers; default 4 */
    int32_t batch;      /* rows per training step and per inference chunk, multiple of 32; default 512 */
    int32_t reserved;
    double lr;          /* Adam step size at the start of each training call; default 1e-3 */
    double lr_final;    /* ... decayed by a half cosine to this at its end; default 1e-5 */
    uint64_t seed;      /* weight initialisation and training draws; default 1 */
} gk_surrogate_opts;

gk_status gk_surrogate_default_opts(gk_surrogate_opts *opts);

/* lo/hi [GK_NP] (host): the box of the training draws and of the input
 * scaling; it must lie in the parameter domain.  The model needs upsample 1
 * and nx * ny a multiple of 16.  Errors: GK_EINVAL, GK_ENOMEM, GK_EDEVICE. */
gk_status gk_surrogate_create(gk_model *instrument, const double *lo, const double *hi,
                              const gk_surrogate_opts *opts, gk_surrogate **out);
gk_status gk_surrogate_destroy(gk_surrogate *s);

/* Runs `steps` Adam steps of `batch` fresh draws each; losses [steps] (host,
 * may be NULL) receives each step's loss before its update.  Blocks. */
gk_status gk_surrogate_train(gk_surrogate *s, int64_t steps, float *losses);

/* Number of floats in the weight vector: for each layer (the output layer
 * last) W [out][in] row-major, then b [out]; the first layer has in = 32. */
int64_t gk_surrogate_weight_count(const gk_surrogate *s);
/* Host copies of the master weights; set_weights also resets Adam.  Block. */
gk_status gk_surrogate_get_weights(gk_surrogate *s, float *w, int64_t n);
gk_status gk_surrogate_set_weights(gk_surrogate *s, const float *w, int64_t n);

/* Saves the surrogate to a file: options, box and instrument description
 * (the fields of gk_model_desc that define the grid, PSF, LSF and rotation
 * curve) and the FP32 master weights, little-endian, after the 8-byte tag
 * "GKSURR01".  Load creates a surrogate for `instrument` from such a file and
 * sets its weights (fresh Adam state); the instrument must match the saved
 * description.  Both block.  Errors: GK_EINVAL (unreadable or truncated file,
 * wrong tag, instrument mismatch), GK_ENOMEM, GK_EDEVICE. */
gk_status gk_surrogate_save(gk_surrogate *s, const char *path);
gk_status gk_surrogate_load(gk_model *instrument, const char *path, gk_surrogate **out);

/* Loss and its gradient (host, weight-vector layout) on the rows params
 * [B][GK_NP] (host or device; B a multiple of 32), targets from the plain
 * evaluation; no update.  Blocks. */
gk_status gk_surrogate_gradients(gk_surrogate *s, const double *params, int32_t B, float *grads,
                                 double *loss);

/* One Adam step on the caller's rows params [B][GK_NP] (host or device; B a
 * multiple of 32, at most 65536) with step size lr > 0: targets and mask from
 * the plain evaluation, the loss gradient as in gk_surrogate_gradients, then
 * m = 0.9 m + 0.1 g, v = 0.999 v + 0.001 g^2 and
 * w -= lr (m / (1 - 0.9^t)) / (sqrt(v / (1 - 0.999^t)) + 1e-8) on every master
 * weight and bias (FP32), t counting the steps since the weights were set.
 * gk_surrogate_train's step t of a call of n steps is this step on the rows
 * drawn for it (row b, slot s: lo_s + u (hi_s - lo_s) rounded once (a fused
 * multiply-add; lo_s where hi_s <= lo_s), u = (r_s + 1/2) 2^-32
 * with r the 12 words of Philox4x32-10 blocks j = 0, 1, 2 at counter
 * (b, t_total, t_total >> 32, j), key (seed, (seed >> 32) ^ 0x73757272), t_total
 * = the steps since the weights were set) with step size
 * lr_final + (lr - lr_final) (1 + cos(pi t / (n - 1))) / 2.  *loss (may be
 * NULL) receives the loss before the update.  Blocks. */
gk_status gk_surrogate_step(gk_surrogate *s, const double *params, int32_t B, double lr,
                            double *loss);

/* maps [B][2][ny][nx] (device, km/s: m1 then m2) predicted for params
 * [B][GK_NP] (host or device), enqueued on hip_stream. */
gk_status gk_surrogate_predict(gk_surrogate *s, const double *params, int32_t B, float *maps,
                               void *hip_stream);

/* chi2 [B] (device) of the predicted maps against the observation of `model`
 * (eq. 11 with the model's mask, errors and W); +INF for rows outside the
 * parameter domain.  The model must have the surrogate's instrument. */
gk_status gk_surrogate_chi2(gk_surrogate *s, gk_model *model, const double *params, int32_t B,
                            double *chi2, void *hip_stream);

/* Nested sampling as gk_fit_nested, with every round's candidates screened by
 * the surrogate.  With chi2_floor the plain chi2 of the lowest live point at
 * the start of the round and `shift` the largest surrogate-minus-plain chi2
 * among the latest 4 max(n_live, batch, batch_max) plainly evaluated
 * candidates whose plain chi2 was within 4 max(margin, 1) of the floor of
 * their round (the errors the screen must bound are those of acceptable
 * candidates; until 64 such candidates exist: among the latest
 * max(n_live, batch) plainly evaluated candidates, 0 before the first), a
 * candidate whose surrogate chi2 exceeds chi2_floor + shift + margin is
 * discarded, except that a Philox draw (counter: candidate, round)
 * keeps it with probability audit (the audit sample measures the screen);
 * every other candidate gets the plain chi2, which alone decides acceptance,
 * posterior and evidence.
 * With a useless surrogate the screen passes everything and the run is the
 * plain one.  margin >= 0, 0 <= audit <= 1.  Blocks. */
gk_status gk_fit_nested_screened(gk_model *model, gk_surrogate *s, const double *lo,
                                 const double *hi, const uint8_t *free_mask, const double *fixed,
                                 const gk_ns_opts *opts, double margin, double audit,
                                 gk_ns_result *result, double *samples, int64_t cap,
                                 int64_t *n_samples);

/* ---- Monte-Carlo parameter errors (Sec. 4.2, Sec. 4.3) --------------------
 * Refits n_sim simulated observations of the model's instrument, each with
 * the LM of gk_fit_lm_survey (same options and box, started from `best`), and
 * returns every fit and the sample standard deviation over the simulations.
 * The simulations are built on the device from the model's observation:
 *  GK_MC_SHUFFLE (the GHASP errors, Sec. 4.2): residual field of `best`
 *    re-dealt over the unmasked pixels: with the unmasked pixels numbered
 *    0..n_valid-1 in row-major order, pixel k of simulation s gets
 *    V_best(k) + (V_obs - V_best)(perm[s][k]), and likewise sigma when the
 *    observation's W > 0; perm [n_sim][n_valid] (host) holds one
 *    permutation of 0..n_valid-1 per simulation (checked);
 *  GK_MC_PERTURB (the DYNAMO errors, Sec. 4.3): every unmasked pixel moves
 *    by its error times a standard normal draw, V_obs + E_v noise[s][0] and,
 *    when W > 0, sigma_obs + E_s noise[s][1]; noise [n_sim][2][ny][nx] (host).
 * Masked pixels, errors, mask and W stay those of the observation; the
 * random draws are inputs, so results are reproducible.  best [12], lo, hi
 * [12] (NULL = unbounded), free_mask [12] and opts as for gk_fit_lm.
 * fits [n_sim][12] (host) gets each simulation's fit, sd [12] the standard
 * deviation (divisor n_sim - 1) of each free slot over the simulations, 0 for
 * fixed ones; *n_capped (may be NULL) the fits that stopped at max_iter.
 * Simulations run in groups as surveys of clones of the model (its
 * observation memory each), with the LM residuals of a group kept under
 * 4 GiB.  Cube models must run the direct convolution path.  Blocks.
 * Errors: GK_EINVAL (arguments, a row of perm that is not a permutation),
 * GK_ESTATE (no observation), GK_ENOMEM, GK_EDEVICE. */
enum { GK_MC_SHUFFLE = 0, GK_MC_PERTURB = 1 };
gk_status gk_mc_errors(gk_model *model, const double *best, const uint8_t *free_mask,
                       const double *lo, const double *hi, const gk_lm_opts *opts, int32_t mode,
                       int32_t n_sim, const int32_t *perm, const float *noise, double *fits,
                       double *sd, int32_t *n_capped);

/* ---- Gaussian line fitting of a cube (Sec. 2.2.5, Sec. 5.2) ---------------
 * The alternative to moment maps: every spectrum of a data cube is fitted by
 * A exp(-(v - mu)^2 / (2 s^2)) at the channel velocities
 * v_k = v0_kms + (k - crpix) dv_kms, minimising the sum of squared residuals.
 * Start: the moments of the spectrum clipped at zero (area S0 dv, centre,
 * width; A = area / (s sqrt(2 pi))); S0 <= 0 or zero width means no line.
 * Box: A >= 0, mu inside the band, s in [dv / 4, nz dv].  Steps: damped
 * Gauss-Newton with the analytic Jacobian, (M + lambda diag M) d = -g by
 * Cholesky (d = 0 if M is not positive definite), trial clipped to the box,
 * accepted if chi2 drops (lambda /= 10; stop when the relative chi2 decrease
 * <= ftol or the largest relative step <= xtol), else lambda *= 10 (stop above
 * 1e10); at most max_iter trials.  All FP64, one lane per spectrum.
 * cube: device float [nz][nspec] (channel-major: a [nz][ny][nx] cube is
 * nspec = nx ny).  maps: device float [3][nspec] = line flux A s sqrt(2 pi)
 * (0 without a line), centre mu and width s (NaN without a line).  status
 * (device int32 [nspec], may be NULL): 0 no line, 1 converged, 2 damping
 * limit, 3 iteration cap; iterations (device int32 [nspec], may be NULL): the
 * trials made.  Enqueued on hip_stream. */
typedef struct {
    int32_t max_iter;   /* default 100 */
    int32_t reserved;   /* must be 0 */
    double lambda0;     /* default 1e-3 */
    double ftol, xtol;  /* defaults 1e-12 */
} gk_line_opts;
gk_status gk_line_default_opts(gk_line_opts *opts);
gk_status gk_fit_lines(const float *cube, int32_t nz, int64_t nspec, double v0_kms, double dv_kms,
                       double crpix, const gk_line_opts *opts, float *maps, int32_t *status,
                       int32_t *iterations, void *hip_stream);

/* BF16 GEMM of the surrogate: C [M][N] (f32, row stride ldc) = sum_k A(m, k)
 * B(n, k), A(m, k) = trans_a ? A[k lda + m] : A[m lda + k], B likewise; BF16
 * operands as uint16 bit patterns; all device memory; K a multiple of 32,
 * lda and ldb multiples of 8, operands 16-byte aligned.  Enqueued on hip_stream. */
gk_status gk_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                       const uint16_t *A, int32_t lda, const uint16_t *B, int32_t ldb, float *C,
                       int32_t ldc, void *hip_stream);

/* Shape of the fine model cube with its halo and the halos themselves:
 * dims = {nx_ext, ny_ext, nz_ext, h_psf, h_lsf}. */
gk_status gk_model_dims(const gk_model *model, int32_t dims[5]);

/* Launch mode of the evaluation calls (gk_evaluate_batch, gk_chi2_batch,
 * gk_residual_batch and the fitters' batched evaluations) whose rows are in
 * device memory and whose stream is not the null stream.  GK_LAUNCH_GRAPH
 * (the default): the second call with the same rows pointer, batch size,
 * output pointers and stream records the call's launch chain (every chunk's
 * kernels) in a HIP graph, and later such calls replay it; the rows' values
 * may change between calls (the kernels read them when they run).  A graph
 * is dropped when the model's scratch grows or its observation is set, and
 * at most 8 are kept (oldest dropped first).  GK_LAUNCH_EAGER launches every
 * kernel each time.  Profiling (gk_set_profiling) always launches eagerly.
 * Results are identical in both modes. */
enum { GK_LAUNCH_EAGER = 0, GK_LAUNCH_GRAPH = 1 };
gk_status gk_set_launch_mode(gk_model *model, int32_t mode);
/* graph replays made by the model so far */
gk_status gk_graph_launches(const gk_model *model, int64_t *count);

/* ---- Launch-shape autotuner ------------------------------------------------
 * Times every spatial-convolution configuration the model can run -- the FFT
 * path and direct data tiles of 32x32, 64x32 (the register-blocked u = 1
 * kernel when it applies), 32x16, 16x16, 32x8, 16x8, 8x8 and 64x16 -- on
 * `batch` synthetic rows (a disc centred in the window; chi2 if the model
 * has an observation, maps otherwise), best of three launches each after a
 * warm-up, and keeps the fastest.  A model created with GK_CONV_DIRECT or
 * GK_CONV_FFT only tries that path.  Frees the row scratch; blocks. */
typedef struct {
    int32_t conv_mode;      /* chosen: GK_CONV_DIRECT or GK_CONV_FFT */
    int32_t tile_x, tile_y; /* chosen data tile of the direct path (0 for FFT) */
    int32_t n_candidates;   /* configurations timed */
    double ms_best;         /* its time per batch */
    double ms[16];          /* per candidate in the order above, -1 if it did not fit */
} gk_tune_result;
gk_status gk_autotune(gk_model *model, int32_t batch, gk_tune_result *result);

/* Forces a configuration (GK_CONV_DIRECT with a data tile from the list
 * above, or GK_CONV_FFT with tile 0 x 0).  GK_EINVAL if it does not fit. */
gk_status gk_set_conv_config(gk_model *model, int32_t conv_mode, int32_t tile_x, int32_t tile_y);

/* The spatial convolution path the model runs: GK_CONV_DIRECT or GK_CONV_FFT. */
gk_status gk_model_conv_path(const gk_model *model, int32_t *conv_mode);

/* Message of the last failed call on this host thread ("" if none). */
const char *gk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GBK_H */
