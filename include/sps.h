/*
 * sps.h - C ABI of the MI355X (gfx950) batched stellar-population forward model.
 *
 * The library evaluates, for a batch of B parameter vectors theta[B, P] (the
 * live points of a nested sampler), the forward model of the paper "Ceridwen:
 * Fast and Flexible GPU-Accelerated Stellar Population Inference":
 *   SFH x enrichment weights W_ma (Sec. 2.2, App. B), contraction with the SSP
 *   grid (eq. 1), nebular lines (Sec. 2.3, App. C), two-component dust
 *   (Sec. 2.4, eq. D2), observer-frame conversion (Sec. 2.6), projection onto
 *   photometry (App. E) or a spectrum (App. F), and the diagonal Gaussian
 *   log-likelihood with the noise floor (eq. 6, eq. G1),
 * plus its exact gradient and a continuous-batching request server.
 *
 * Conventions
 *   - Every call returns sps_status: SPS_OK (0), SPS_PENDING (1) or a negative
 *     error.  sps_last_error() returns a thread-local message for the last error
 *     of the calling thread.  No call throws across the ABI.
 *   - Host arrays passed to *_load / *_create / sps_submit are copied; the
 *     caller keeps ownership and may free them after the call returns.
 *   - theta, model, logl and grad pointers of the hot calls are device pointers
 *     on the library's device, owned by the caller, contiguous, row-major.
 *   - Hot calls (sps_forward, sps_logl, sps_logl_grad) validate arguments
 *     synchronously, enqueue their kernels on the caller's HIP stream and return
 *     without synchronising; they never allocate.  A device fault surfaces as
 *     SPS_E_HIP on a later call.  Calls that share one sps_obs use its
 *     workspace: serialise them on one stream.
 */
#ifndef SPS_H
#define SPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sps_status;
enum {
  SPS_OK = 0,
  SPS_PENDING = 1,
  SPS_E_INVAL = -1,     /* bad argument (NULL, non-finite, out of range, bare R) */
  SPS_E_SHAPE = -2,     /* size mismatch, B > max_batch, unsupported size */
  SPS_E_NOMEM = -3,     /* device or host allocation failed (load/create only) */
  SPS_E_BUDGET = -4,    /* request can never fit the server's HBM budget */
  SPS_E_HIP = -5,       /* HIP runtime error (message names the call) */
  SPS_E_STATE = -6,     /* object in the wrong state (destroyed, shut down) */
  SPS_E_TIMEOUT = -7,   /* sps_wait timed out */
  SPS_E_CANCELLED = -8, /* request was cancelled */
  SPS_E_NOTFOUND = -9   /* unknown ticket */
};

/* Arithmetic of the library contraction (eq. 1).  The luminosity distance and
 * the chi-squared accumulation are always FP64.
 *   SPS_FP64   : everything in FP64 (parity instance).
 *   SPS_FP32   : FP32 MFMA contraction, FP32 epilogue and projection.
 *   SPS_BF16/SPS_FP16 : library stored as 2^e (H + R) per row with 16-bit hi H
 *     and 16-bit residual R, weights as 2^e (W_h + W_l) per point; MFMA passes
 *     W_h.H + W_h.R + W_l.H accumulated in FP32 (one refinement pass over the
 *     residual terms).
 *   *_1PASS    : W_h.H only.   *_HR : W_h.H + W_h.R only.
 *   *_WL       : W_h.H + W_l.H (the library residual dropped: two passes). */
typedef enum {
  SPS_FP64 = 0,
  SPS_FP32 = 1,
  SPS_BF16 = 2,
  SPS_FP16 = 3,
  SPS_BF16_1PASS = 4,
  SPS_FP16_1PASS = 5,
  SPS_BF16_HR = 6,
  SPS_FP16_HR = 7,
  SPS_BF16_WL = 8,
  SPS_FP16_WL = 9
} sps_precision;

typedef struct sps_library sps_library;
typedef struct sps_obs sps_obs;
typedef struct sps_server sps_server;

/* ------------------------------------------------------------------------- */
/* Library: SSP grid + model configuration (Sec. 2.1-2.6)                     */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_age, n_z, n_afe, n_wave;
  const double *ages;   /* [n_age] yr, strictly increasing, > 0 */
  const double *logz;   /* [n_z] log10(Z/Zsun), strictly increasing */
  const double *afe;    /* [n_afe] [alpha/Fe] nodes; may be NULL when n_afe == 1 */
  const double *wave;   /* [n_wave] rest wavelength, Angstrom, strictly increasing */
  const double *flux;   /* [n_afe][n_z][n_age][n_wave] Lsun/A per Msun formed, >= 0 */
  double t_young;       /* birth-cloud edge in yr: ages < t_young see tau_BC (Sec. 2.4) */
  /* star-formation history (Sec. 2.2, App. B): n_sfh lookback bins with edges
   * 0, then log-uniform from T1 to t_univ(z); n_zh enrichment nodes (0 =
   * constant-metallicity mode using theta[logzsol]). */
  int32_t n_sfh;
  double T1;
  int32_t n_zh;
  double H0, Om;        /* flat LambdaCDM (Sec. 2.6): km/s/Mpc, Omega_m */
  const double *dust_a; /* [n_wave] diffuse-law shape a(lambda); NULL = zeros */
  const double *dust_d; /* [n_wave] bump shape d(lambda); NULL = zeros */
  /* nebular lines (App. C); n_line = 0: no lines.  Without n_line_tau the line
   * table's age axis is exactly the SSP ages younger than t_young. */
  int32_t n_line, n_zg, n_u;
  const double *line_wave;  /* [n_line] rest Angstrom */
  const double *line_table; /* [n_line][n_line_tau or n_young][n_zg][n_u] log10(L_line/Q), erg */
  const double *zg_nodes;   /* [n_zg] gas log10(Z/Zsun) */
  const double *u_nodes;    /* [n_u] log10 U */
  uint32_t precisions;  /* bitmask of (1u << sps_precision) copies to build;
                           FP32 is always built */
  int32_t device;       /* HIP device ordinal */
  /* Full nebular grid evaluation (Sec. 2.3.1, App. C), optional (zero / NULL: off).
   * The line table may carry an age axis of its own (n_line_tau > 0, line_tau[] in yr,
   * strictly increasing); the nebular continuum cube cont_table holds log10(L_nu/Q)
   * (L_nu in erg/s/Hz, Q in photons/s) on its own (age, log Z_gas, log U) axes, tabulated
   * on the library's wavelengths.  Each cube is interpolated trilinearly (linearly in
   * age) and scaled by Q_ma (eq. C1); nebular emission goes to the SSP ages inside every
   * cube's age range, which must be birth-cloud ages (at most 128 of them with a
   * continuum, whose cube has at most 128 (Z_gas, U) nodes: else SPS_E_SHAPE).
   * SPS_E_INVAL when an axis is not increasing, a table is not finite or no SSP age,
   * or one older than t_young, falls in the range. */
  int32_t n_line_tau;
  const double *line_tau;   /* [n_line_tau] yr */
  int32_t n_cont_tau, n_cont_zg, n_cont_u;
  const double *cont_tau;   /* [n_cont_tau] yr */
  const double *cont_zg;    /* [n_cont_zg] gas log10(Z/Zsun) */
  const double *cont_u;     /* [n_cont_u] log10 U */
  const double *cont_table; /* [n_cont_tau][n_cont_zg][n_cont_u][n_wave] log10(L_nu/Q) */
  /* Ionising-photon escape (Sec. 2.3.2, App. D.1): sps_escape.  With a geometry, theta
   * gains a last column frac_obrun = f_ob (clamped to [0, 1]); nebular emission is
   * scaled by the covered fraction and a fraction f_ob of the nebular ages' ionising
   * continuum is restored: SPS_ESCAPE_RUNAWAY_BC puts the young light (stars, nebular
   * continuum and lines) through (1 - f_ob) e^{-tau_BC} + f_ob and lets the restored
   * ionising continuum bypass the birth cloud (eq. runaway_mix); SPS_ESCAPE_PICKET lets
   * f_ob of the young stars, ionising continuum included, escape free of both dust
   * components and attenuates the covered rest (and its nebular emission) by both. */
  int32_t escape;
  /* SFH to age weights (App. B): SPS_SFH_STEP (bin masses, linear-time cell overlap) or
   * SPS_SFH_LINEAR (theta's SFH values are the SFR at the lookback edges T_0 .. T_{n-1},
   * the last repeated at T_n, Msun/yr per unit of 10^logmass; piecewise-linear SFR
   * integrated against the linear-in-ln(age) tent of each SSP age node, eq. tent_integral,
   * clipped at zero and rescaled to each bin's trapezoid mass). */
  int32_t sfh_scheme;
  /* IGM transmission (Sec. 2.6), a bit mask: 0 off; SPS_IGM_MADAU the Madau (1995)
   * Lyman-series and Lyman-limit optical depth scaled by a theta column igm_factor (after
   * frac_obrun), applied at lambda (1 + z) to the observer-frame model and to each line;
   * with it, optionally, SPS_IGM_DAMPING the damping wing of a partly neutral IGM between
   * z = 6 and the source (Miralda-Escude 1998, Totani et al. 2006; neutral fraction in a
   * theta column x_hi; tau_GP(z) = 3.88e5 ((1 + z) / 7)^1.5; the Gunn-Peterson depth
   * blueward of the source's Lyman alpha inside that range) and SPS_IGM_DLA a damped
   * Lyman-alpha absorber (Tepper-Garcia 2006 Voigt profile, b = 10 km/s) of column
   * 10^log_nhi cm^-2 at z_dla (two theta columns).  Other values: SPS_E_INVAL. */
  int32_t igm;
  /* Free stellar velocity dispersion (Sec. 2.5, App. F): > 0 adds a theta column
   * sigma_gal (km/s, after igm_factor) admitted in [0, sigma_gal_max] (a point outside
   * gets a NaN model and logL); 0 = no column.  Every observation's continuum is then
   * broadened in the Fourier stage: the rest-frame nodes the projection reads (the
   * pixels' range plus the banded kernel's and sigma_gal_max's reach, or the filter
   * nodes' range plus sigma_gal_max's reach), padded with their edge values to a
   * power-of-two transform of at most 8192 points, are multiplied by
   * exp(-2 pi^2 sigma_gal^2 nu^2), nu conjugate to c ln(lambda); before the IGM and the
   * instrument's kernel.  Needs a wavelength grid uniform in ln(lambda) (else
   * SPS_E_INVAL).  The fixed sigma_gal_kms of a spectrum stays folded into its kernel. */
  double sigma_gal_max;
} sps_library_desc;

typedef enum { SPS_SFH_STEP = 0, SPS_SFH_LINEAR = 1 } sps_sfh_scheme;
enum { SPS_IGM_MADAU = 1, SPS_IGM_DAMPING = 2, SPS_IGM_DLA = 4 };

typedef enum { SPS_ESCAPE_NONE = 0, SPS_ESCAPE_RUNAWAY_BC = 1, SPS_ESCAPE_PICKET = 2 } sps_escape;

typedef struct {
  int32_t K, K_pad, K_young_pad, N, N_pad, n_young, n_line;
  int64_t device_bytes; /* device memory held by the library */
} sps_library_info;

/* Copies the grid to the device, packs it in young-first K order (young SSP
 * rows, then the line-profile rows, then, with an escape geometry, the raw ionising
 * continuum of the nebular ages, then old rows, each padded), removes the ionising
 * continuum of nebular-covered ages from their SSP rows (Fig. A1), computes Q_ma
 * (eq. C1), resamples the nebular cubes onto the SSP ages and builds the requested
 * precision copies (per-row 2^e scaling and 16-bit hi/residual split), plus an N-major
 * FP32 copy for the adjoint.
 * Errors: SPS_E_INVAL (bad values), SPS_E_SHAPE, SPS_E_NOMEM, SPS_E_HIP. */
sps_status sps_library_load(const sps_library_desc *desc, sps_library **out);
sps_status sps_library_info_get(const sps_library *lib, sps_library_info *out);
void sps_library_destroy(sps_library *lib);

/* Column layout of theta[B, P] (FP64, row-major), shared by every observation:
 * 14 scalar columns (in this order: logmass, zred, tau_bc, alpha_bc, tau_diff,
 * delta, logzsol, gas_logz, gas_logu, afe, log_err_scale, log_f_calib,
 * log_f_data, log_jitter), then sfh[n_sfh] bin masses (Msun formed per unit of
 * 10^logmass; node SFRs under SPS_SFH_LINEAR), then zh[n_zh] enrichment nodes, then,
 * for a library with an escape geometry, frac_obrun, then, with the IGM, igm_factor,
 * x_hi with its damping wing, log_nhi and z_dla with its damped absorber, then, with a
 * free velocity dispersion, sigma_gal (each -1 when absent).  Unused columns are
 * ignored. */
typedef struct {
  int32_t P, n_scalar, sfh, n_sfh, zh, n_zh;
  int32_t logmass, zred, tau_bc, alpha_bc, tau_diff, delta, logzsol, gas_logz, gas_logu, afe;
  int32_t log_err_scale, log_f_calib, log_f_data, log_jitter;
  int32_t frac_obrun, igm_factor, sigma_gal;
  int32_t x_hi, log_nhi, z_dla;
} sps_layout;
sps_status sps_theta_layout(const sps_library *lib, sps_layout *out);

/* ------------------------------------------------------------------------- */
/* Observations (Sec. 3): photometry (App. E) or a spectrum (App. F)          */
/* ------------------------------------------------------------------------- */
enum { SPS_OBS_PHOT = 0, SPS_OBS_SPEC = 1, SPS_OBS_LINES = 2 };
/* calibration polynomial of a spectrum (Sec. 3.2, App. H.3) */
enum { SPS_CALIB_NONE = 0, SPS_CALIB_MARGINAL = 1, SPS_CALIB_OPTIMISE = 2 };
/* LSF unit conventions of eq. F2.  SPS_LSF_BARE_R is rejected (SPS_E_INVAL):
 * a resolving power must state whether it is lambda/FWHM or lambda/sigma. */
enum {
  SPS_LSF_R_FWHM = 0, SPS_LSF_R_SIGMA = 1, SPS_LSF_FWHM_AA = 2, SPS_LSF_SIGMA_AA = 3,
  SPS_LSF_SIGMA_KMS = 4, SPS_LSF_FWHM_KMS = 5, SPS_LSF_BARE_R = 6
};
/* noise-floor switches of eq. G1 (parameters read from theta in ln space) */
enum { SPS_NOISE_ERR_SCALE = 1, SPS_NOISE_F_CALIB = 2, SPS_NOISE_F_DATA = 4, SPS_NOISE_JITTER = 8 };
/* warning flags returned by sps_obs_create */
enum { SPS_WARN_LSF_FINER_THAN_LIBRARY = 1 };

typedef struct {
  int32_t kind;               /* SPS_OBS_PHOT, SPS_OBS_SPEC or SPS_OBS_LINES */
  /* photometry: n_band filter curves concatenated; filter_len[b] nodes each,
   * observer-frame Angstrom, strictly increasing within a curve */
  int32_t n_band;
  const int32_t *filter_len;
  const double *filter_wave;
  const double *filter_trans;
  /* spectrum: detector pixel centres (observer Angstrom, increasing) */
  int32_t n_pix;
  const double *pix_wave;
  int32_t lsf_mode;           /* SPS_LSF_* */
  double lsf_value;           /* constant R / width, used when lsf_curve == NULL */
  const double *lsf_curve;    /* [n_pix] or NULL */
  double z_ref;               /* reference redshift of the fixed kernel (eq. F4) */
  double sigma_gal_kms;       /* fixed stellar dispersion folded into the kernel */
  double sigma_gas_kms;       /* gas dispersion of the line profiles (eq. F6) */
  /* data [n_data] with n_data = n_band or n_pix: maggies (F_nu / 3631 Jy) */
  const double *data;
  const double *sigma;
  const uint8_t *mask;        /* NULL = all included; ANDed with finite(data),
                                 finite(sigma), sigma > 0 (App. H.1) */
  uint32_t noise_flags;       /* SPS_NOISE_* */
  int32_t max_batch;          /* workspace is sized for B <= max_batch */
  /* spectrum: spectrophotometric calibration polynomial (Sec. 3.2, App. H.3).  The model
   * mu (1 + sum_m c_m T_m(x)), T_m Chebyshev polynomials on the pixel wavelengths mapped
   * onto [-1, 1] (first pixel -1, last +1), c ~ N(0, diag(calib_prior^2)):
   * SPS_CALIB_MARGINAL integrates the coefficients out (eq. app_polymarg),
   * SPS_CALIB_OPTIMISE evaluates the likelihood at their regularised best fit; the noise
   * model is that of the uncalibrated model, and the model returned is mu.  Order in
   * [0, 7]; calib_prior [calib_order + 1] widths > 0.  No gradient (SPS_E_INVAL). */
  int32_t calib_mode;
  int32_t calib_order;
  const double *calib_prior;
  /* emission-line catalogue (SPS_OBS_LINES, Sec. 3.3, App. I): n_band entries, entry k
   * the sum of line_len[k] of the library's lines, their indices concatenated in
   * line_index (an unresolved blend); data and sigma are integrated fluxes in erg/s/cm^2;
   * upper[k] != 0 marks an upper limit (one-sided chi-squared, eq. app_line_chi2_UL),
   * NULL none.  logL = -chi^2 / 2 over the inclusion mask (App. I.2). */
  const int32_t *line_len;
  const int32_t *line_index;
  const uint8_t *upper;
  /* spectrum: analytic marginalisation of the line fluxes (Sec. 4.1, App. I.3,
   * eq. app_line_marg).  The library lines whose observed wavelength lies within the pixel
   * range are free amplitudes alpha with unit-flux profiles A on the pixels:
   * SPS_LINEMARG_GAUSS gives each the prior N(F_l, (line_prior_frac F_l)^2) around its grid
   * flux F_l (flat for the lines flagged in line_flat [n_line], NULL none; Gaussian lines
   * with F_l = 0 stay fixed at 0), SPS_LINEMARG_FLAT a flat prior to all.  logL becomes
   * lnL_diag(r) + b^T P^-1 b / 2 - ln|P| / 2 - sum ln s_l + (m_flat / 2) ln 2 pi with
   * r = d - mu - A alpha_0, b = A^T W r, P = A^T W A + diag(s^-2) (W at the grid model); the
   * model returned is the grid model.  At most 128 library lines in any rest-frame interval
   * as wide as the pixel range (else SPS_E_SHAPE); spectra of at most 8192 pixels; not with a
   * calibration polynomial; no gradient, no allocation-free call (SPS_E_INVAL). */
  int32_t line_marg;
  double line_prior_frac;
  const uint8_t *line_flat;
} sps_obs_desc;

enum { SPS_LINEMARG_NONE = 0, SPS_LINEMARG_GAUSS = 1, SPS_LINEMARG_FLAT = 2 };

/* Builds the observation's fixed operators (filter rows of eq. E1, kernel
 * widths of eq. F4, line-width table) and its workspace.  *warnings (may be
 * NULL) receives SPS_WARN_* flags.  Errors: SPS_E_INVAL, SPS_E_SHAPE,
 * SPS_E_NOMEM, SPS_E_HIP. */
sps_status sps_obs_create(const sps_library *lib, const sps_obs_desc *desc, sps_obs **out,
                          uint32_t *warnings);
/* Replaces data/sigma/mask of an existing observation (same n_data). */
sps_status sps_obs_set_data(sps_obs *obs, const double *data, const double *sigma,
                            const uint8_t *mask);
int32_t sps_obs_n_data(const sps_obs *obs);
void sps_obs_destroy(sps_obs *obs);

/* ------------------------------------------------------------------------- */
/* Hot calls                                                                  */
/* ------------------------------------------------------------------------- */
/* model_dev [B, n_data] FP64: photometry in maggies, spectra in maggies per
 * pixel (F_nu / 3631 Jy).  Errors: SPS_E_INVAL, SPS_E_SHAPE (B < 1 or
 * B > max_batch), SPS_E_HIP. */
sps_status sps_forward(const sps_library *lib, sps_obs *obs, const double *theta_dev, int32_t B,
                       int32_t precision, double *model_dev, void *hip_stream);
/* logl_dev [B] FP64: eq. (6) with eq. G1 over the inclusion mask; a spectrum with a
 * calibration polynomial adds its marginal or optimised term (Sec. 3.2, App. H.3), a line
 * catalogue takes -chi^2/2 with one-sided upper limits (App. I.2).
 * model_dev may be NULL; when given it also receives the model (for a calibrated
 * spectrum, the model before calibration). */
sps_status sps_logl(const sps_library *lib, sps_obs *obs, const double *theta_dev, int32_t B,
                    int32_t precision, double *logl_dev, double *model_dev, void *hip_stream);
/* logl_dev [B] and grad_dev [B, P] = d logL / d theta (FP64; columns the
 * model does not use are zero).  Hand-written reverse pass.  Supported for
 * SPS_FP64 and SPS_FP32, for libraries without a nebular continuum cube, an
 * escape geometry, a line table on an age axis of its own, the linear SFH scheme, the
 * IGM or a free sigma_gal, and for photometry and spectra without a calibration
 * polynomial or marginalised line fluxes (a line catalogue, a calibrated spectrum or one
 * with marginalised line fluxes: SPS_E_INVAL). */
sps_status sps_logl_grad(const sps_library *lib, sps_obs *obs, const double *theta_dev, int32_t B,
                         int32_t precision, double *logl_dev, double *grad_dev, void *hip_stream);
/* Joint analytic marginalisation of the line fluxes over a spectrum, a line catalogue and
 * a photometric observation of the same object (Sec. 4.1, App. I.3: eq. app_line_marg
 * summed over the observations).  spec: a spectrum created with line_marg set (its prior
 * mode, fraction and flat flags apply); cat: an SPS_OBS_LINES catalogue, or NULL; phot: an
 * SPS_OBS_PHOT observation, or NULL; all of the same library.  The fitted lines are the
 * spectrum's (observed wavelength within its pixel range) and the lines of the catalogue's
 * detected, included entries, less Gaussian-prior lines with no grid flux.  A catalogue
 * detection is linear in the fitted lines of its blend and enters b and P with weight
 * sigma^-2 and lnL_diag as -chi^2 / 2; an upper limit keeps its one-sided chi-squared at the
 * grid model (it is not Gaussian in the fluxes).  A band is linear in every fitted line
 * through the line's band response (its profile on the model grid through the dust, the
 * observer frame, the IGM and the filter, per unit of its observed flux), with the weight
 * and the normalised Gaussian term of eq. 6 with the noise floor at its grid model; the
 * lines not fitted stay at their grid fluxes.  logl_dev [B] FP64 receives the joint logL of
 * all the observations given.  Stream, ownership and allocation as sps_logl (each
 * observation's workspace is used).  Errors: SPS_E_INVAL (NULL spec or theta, kinds, another
 * library, photometry with a free sigma_gal), SPS_E_SHAPE (a catalogue of more than 256
 * entries; more than 128 lines fitted jointly, bounded by the spectrum's window count plus
 * the catalogue's distinct lines; a photometric observation with fewer than about 43
 * filter nodes per band; B beyond a workspace), SPS_E_HIP. */
sps_status sps_logl_lines_joint(const sps_library *lib, sps_obs *spec, sps_obs *cat, sps_obs *phot,
                                const double *theta_dev, int32_t B, int32_t precision, double *logl_dev,
                                void *hip_stream);

/* Allocation-free variant of sps_logl, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and stream semantics as sps_logl; the per-call scratch of the
 * forward path (batch keys, weight rows, K-tile bits, per-point rows, the attenuated
 * rest-frame spectrum, line luminosities) lives in one static device array of
 * SPS_STATIC_SCRATCH_BYTES per GPU, held until the process ends, instead of the
 * observation's workspace, so the observation may be created with max_batch = 1.  The
 * call allocates nothing and never synchronises.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (on different streams, or from different
 * threads without ordering) race.  Errors: SPS_E_SHAPE when B points at this precision
 * need more scratch than the array holds (64 MiB: on a 2496 x 6016 library with 128
 * lines, up to B = 1792 at FP32 or 16 bit and B = 896 at FP64); SPS_E_INVAL for a
 * spectrum with a calibration polynomial or marginalised line fluxes; otherwise as
 * sps_logl. */
#define SPS_STATIC_SCRATCH_BYTES (64ull << 20)
sps_status sps_logl_static(const sps_library *lib, const sps_obs *obs, const double *theta_dev, int32_t B,
                           int32_t precision, double *logl_dev, double *model_dev, void *hip_stream);

/* Timing of the library-contraction kernel.  When enabled, every hot call on
 * this observation hands a pair of HIP events to the contraction kernel's own
 * dispatch on the caller's stream (hipExtLaunchKernel), which stamps the
 * kernel's start and end without a marker between kernels;
 * sps_obs_contract_timing synchronises those events and returns the summed
 * milliseconds, the number of launches and the executed K-tile count (for
 * executed-flop accounting), then resets the counters. */
sps_status sps_obs_enable_timing(sps_obs *obs, int32_t enable);
sps_status sps_obs_contract_timing(sps_obs *obs, double *ms_total, int64_t *launches,
                                   int64_t *executed_k_tiles, int64_t *dense_k_tiles);

const char *sps_last_error(void);
const char *sps_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPS_H */
