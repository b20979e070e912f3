// Internal definitions shared by the host runtime (api.cpp) and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sps {

// ---------------------------------------------------------------- constants (cgs)
constexpr double kC_cms = 2.99792458e10;
constexpr double kC_kms = 2.99792458e5;
constexpr double kHplanck = 6.62607015e-27;
constexpr double kLsun = 3.839e33;            // FSPS value (Sec. 2.6)
constexpr double kPc_cm = 3.0856775814913673e18;
constexpr double kMpc_cm = 1e6 * kPc_cm;
constexpr double kMpc_km = kMpc_cm / 1e5;
constexpr double kYr_s = 3.15576e7;
constexpr double kFnuAB = 3.631e-20;          // 3631 Jy (App. E)
constexpr double kAng_cm = 1e-8;
constexpr double kLamV = 5500.0;              // attenuation reference (Sec. 2.4)
constexpr double kLamLyman = 912.0;           // eq. C1 upper limit
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- tiling
constexpr int kKAlign = 64;     // K segments (young, old) padded to this
constexpr int kNAlign = 128;    // wavelength axis padded to this
constexpr int kMAlign = 128;    // batch rows padded to this (contraction M tile)
constexpr int kKTile = 32;      // K tile of the occupancy bitmask (FP32 / FP64 kernels)
constexpr int kMaxKPad = 32768; // largest padded K (weight rows) a library may have
constexpr int kMaxKTiles32 = kMaxKPad / kKTile;
// Library row sources (packing): s >= 0 SSP flat index (ia * n_z + m) * n_age + a; -1 - l
// line l's profile; kIonSrc - s the raw ionising continuum (below 912 A) of SSP s; INT_MIN
// padding.
constexpr int kIonSrc = -(1 << 24);
// Longest transform of the Fourier stage of a free sigma_gal (two FP64 complex rows of it
// fill 128 KB of LDS)
constexpr int kVdispMaxFFT = 8192;

// theta scalar columns (see include/sps.h)
enum ThetaCol {
  TH_LOGMASS = 0, TH_ZRED, TH_TAU_BC, TH_ALPHA_BC, TH_TAU_DIFF, TH_DELTA, TH_LOGZSOL,
  TH_GAS_LOGZ, TH_GAS_LOGU, TH_AFE, TH_LOG_ERR_SCALE, TH_LOG_F_CALIB, TH_LOG_F_DATA,
  TH_LOG_JITTER, TH_NSCALAR
};

// Device-resident library (all pointers are device pointers).
struct DevLib {
  int n_age, n_z, n_afe, N, N_pad, K, K_pad, K_young_pad, n_young, n_line, n_zg, n_u;
  // Nebular emission (App. C) and ionising-photon escape (Sec. 2.3.2).  Ages [neb_a0,
  // neb_a1) (birth-cloud ages) take nebular emission; has_neb: lines or continuum on.
  // escape: 0 none, 1 runaway_bc, 2 picket; th_fob: theta column of f_ob.  With an escape
  // geometry the raw ionising continuum of the nebular ages has K rows [ion_k0, ion_k0 +
  // n_ion) between the young segment and the old rows, which start at K_old0; ion_nlim is
  // the first model pixel at or above 912 A (the ionising rows are zero from there on).
  int neb_a0, neb_a1, has_neb, escape, th_fob, ion_k0, n_ion, K_old0, ion_nlim, line_k0;
  // Nebular continuum: cube axes (n_cz, n_cu) and, per nebular age, the log2 cube minus a
  // per-pixel reference, [neb age][n_cz][n_cu][N_pad], with 10^ref * c / lambda^2 / Lsun *
  // kWqScale per pixel (cont_sc); FP64 copies in log10 units for the FP64 path.
  int has_cont, n_cz, n_cu;
  int sfh_scheme;                    // 0 step, 1 linear (tent integral; ages close prep_tab)
  int igm, th_igm;                   // IGM bit mask (1 Madau, 2 damping wing, 4 damped absorber),
  int th_xhi, th_nhi;                //   theta columns of igm_factor, x_HI, logN_HI (z_dla next)
  int vdisp, th_sgal;                // free stellar velocity dispersion and its theta column
  double vd_max;                     // largest admitted sigma_gal [km/s]
  const double *cz, *cu;
  const float *cont_f, *cont_sc_f;
  const double *cont_d, *cont_sc_d;
  int n_sfh, n_zh, P, n_gl;
  int log_uniform;                   // wave grid uniform in ln(lambda) (direct indexing)
  int zmajor;                        // K order: 0 age-major, 1 metallicity-major (see kpos_of)
  double T1, H0, Om, t_young;
  double lnw0, inv_dlnw, dlnw;       // ln(lambda_0), 1/dln(lambda) and dln(lambda) when log_uniform
  const double *cell_lo, *cell_hi;   // [n_age] linear-time Voronoi cells
  const double *logz, *afe;          // nodes
  const double *Q;                   // [n_afe][n_z][n_young] photons/s/Msun
  const double *line_table;          // [n_zg][n_u][n_line][n_young] (-1000 outside the nebular ages)
  const float *line_table_f;         // the same in FP32 (FP32 and 16-bit paths)
  const double *zg, *un;             // nebular table axes
  const double *line_wave;           // [n_line] rest A
  const double *line_a, *line_d;     // dust shape tables at the line wavelengths
  const double *wave_d, *lnwave_d;   // [N_pad] rest wavelength (padding: +inf-ish)
  const float *wave_f;
  const double *lnlv_d;              // [N_pad] ln(lambda/5500)
  const float *lnlv_f;
  const double *dust_a_d, *dust_d_d; // [N_pad]
  const float *dust_a_f, *dust_d_f;
  const double *lam2_d;              // [N_pad] lambda^2 (A^2)
  const double *LT64;                // [N_pad][K_pad] FP64, K contiguous
  const float *LT32;                 // [N_pad][K_pad] FP32
  const float *L32n;                 // [K_pad][N_pad] FP32, N contiguous (adjoint)
  const uint16_t *Hb, *Rb;           // [N_pad][K_pad] bf16 hi / residual
  const uint16_t *Hh, *Rh;           // [N_pad][K_pad] fp16 hi / residual
  const int *kexp;                   // [K_pad] row exponent e_k of the 16-bit copies
  const int16_t *kexp16;             // the same as 16-bit integers (weight builder)
  const double *gl_u, *gl_w;         // [n_gl] composite Gauss-Legendre on [0,1]
  // The weight builder's node tables in one block, in the order of its LDS layout:
  // logz[n_z], afe[n_afe] (0 when n_afe = 1), cell_lo[n_age], cell_hi[n_age],
  // zg[n_zg], un[n_u], Q[n_afe][n_z][n_young] (nebular emission only), ages[n_age] (linear SFH
// scheme only), padded to an even count.
  const double *prep_tab;
};

// Nebular continuum: photon-weighted masses sum_m W Q are carried in units of 2^150
// photons/s (FP32 range), the factor folded into cont_sc.
constexpr double kWqScale = 1.4272476927059599e45;   // 2^150

// Length in doubles of DevLib::prep_tab.
__host__ __device__ inline int prep_tab_len(const DevLib &lib) {
  const int nq = lib.has_neb ? lib.n_afe * lib.n_z * lib.n_young : 0;
  const int n = lib.n_z + lib.n_afe + 2 * lib.n_age + lib.n_zg + lib.n_u + nq + (lib.sfh_scheme ? lib.n_age : 0);
  return n + (n & 1);
}

// Observation descriptor in device memory.
struct DevObs {
  int kind, n_data, n_band, n_fnodes, noise_flags, lsf_mode, has_curve, pad;
  const int *band_off;               // [n_band+1]
  const double *fw;                  // [n_fnodes] filter node wavelengths (observer A)
  const double *fwln;                // [n_fnodes] their natural logarithms
  const double *fr_d;                // R_j lambda_j dlambda_j / zero point  (eq. E1)
  const float *fr_f;
  const double *pix, *lnpix;         // [n_pix]
  const double *ksig;                // [n_pix] continuum kernel dispersion in ln(lambda)
  const double *lsf_vals;            // [n_pix] LSF parameter curve (eq. F2 units) or NULL
  double sigma_gas_kms, lsf_value;   // gas dispersion; constant LSF parameter
  double fwln_min, fwln_max;         // ln of the shortest and longest filter node
  double ksig_max;                   // largest continuum kernel dispersion (spectra)
  double lnpix_lo, lnpix_hi;         // ln of the first and last pixel (spectra)
  const double *data, *sigma;        // [n_data]
  const uint8_t *mask;               // [n_data] final inclusion mask
  const double *ivar;                // [n_data] 1/sigma^2, 0 where masked
  double lnorm;                      // -1/2 sum ln(2 pi sigma^2) over the included data
  // spectrum calibration polynomial: mode (0 off, 1 marginal, 2 optimise), order, x = pixel
  // wavelength * calib_xs + calib_x0 on [-1, 1], prior inverse variances, sum of ln s_m
  int calib_mode, calib_order;
  double calib_xs, calib_x0, calib_lnsd;
  double calib_ivar[8];
  // line catalogue: entry k sums lines lidx[loff[k] .. loff[k+1]); upper[k]: upper limit
  const int *loff, *lidx;
  const uint8_t *upper;
  // Fourier stage of a free sigma_gal: window margin in nodes, transform length (a power
  // of two) and its log2, ln of the observed range's ends, the grid's dln(lambda), and the
  // twiddles e^{-2 pi i k / n}, k < n / 2, as (cos, sin) pairs
  int vd_M, vd_nfft, vd_log2, vd_pad;
  double vd_lnlo, vd_lnhi, vd_dlnl;
  const double *vd_tw;
  // analytic marginalisation of the line fluxes of a spectrum: mode (0 off, 1 Gaussian prior
  // of width lm_frac F_l, flat where lm_flat[l]; 2 flat), per-line flat flags or NULL
  int lm_mode, lm_pad;
  double lm_frac;
  const uint8_t *lm_flat;
};
// Lines a spectrum's marginalisation fits at most (its dense normal matrix lives in LDS:
// 129 KB of the workgroup's 150 KB)
constexpr int kLineMargMax = 128;

// Per-point quantities, stored at the point's sorted row.
struct PointRow {
  double z, t_univ, dl, dc, scale_fnu, mass10, wscale;
  double tau_bc, alpha_bc, tau_diff, delta;
  // escape geometry: the young light crosses the birth cloud with transmission
  // bc_p e^{-tau_BC} + bc_q; nebular emission is scaled by neb_s; fob = f_ob
  double bc_p, bc_q, neb_s, fob;
  // nebular continuum: the point's cell (nc_j) and fractions (nc_t) on the cube's
  // (log Z_gas, log U) axes
  double nc_t[2];
  int nc_j[2];
  int b;        // original batch index
  int obs;      // observation slot
  int kind;     // observation kind
  int seg0;     // log-uniform grid: first rest-frame pixel the projection reads (photometry:
  int seg_n;    //   phot_span; spectra: spec_span) and the number of pixels from there
  int cov0;     // pixels [cov0, cov0 + cov_n) of F that must be computed: the span above, or
  int cov_n;    //   with a free sigma_gal the Fourier stage's window (vdisp_window), which holds it
};

// Window [j0, j0 + n) of the Fourier stage of a free sigma_gal (Sec. 2.5, App. F) at
// redshift z: from floor(u(lambda_lo)) - M to floor(u(lambda_hi)) + 1 + M, clamped to the
// grid, u(lambda) = (ln lambda - ln(1 + z) - ln lambda_0) / dln(lambda); empty for a
// non-finite redshift or a range off the grid.
__device__ __forceinline__ void vdisp_window(const DevLib &lib, double lnlo, double lnhi, int M, double dlnl,
                                             double z, int &j0, int &n) {
  const double lnopz = log1p(z);
  const double u0 = (lnlo - lnopz - lib.lnw0) / dlnl, u1 = (lnhi - lnopz - lib.lnw0) / dlnl;
  j0 = 0;
  n = 0;
  if (!(isfinite(u0) && isfinite(u1))) return;
  const double a = fmax(floor(u0) - M, 0.0), b = fmin(floor(u1) + 2.0 + M, (double)lib.N);
  if (b > a) {
    j0 = (int)a;
    n = (int)b - j0;
  }
}

// Fractional log index of the rest wavelength of an observed filter node, on a
// log-uniform grid: ln(lambda_obs) / dln(lambda) + ui0, ui0 = -(ln(1+z) + ln lambda_0) /
// dln(lambda).  One fused multiply-add, so that every caller rounds it the same way.
__device__ __forceinline__ double phot_u(const DevLib &lib, double fwln, double ui0) {
  return __fma_rn(fwln, lib.inv_dlnw, ui0);
}
__device__ __forceinline__ double phot_ui0(const DevLib &lib, double z) {
  return -(log1p(z) + lib.lnw0) * lib.inv_dlnw;
}
// Rest-frame pixels [seg0, seg0 + seg_n) that the filter nodes of an observation at
// redshift z interpolate between: from the bracketing interval of the shortest node to
// that of the longest, clamped to the grid.
__device__ __forceinline__ void phot_span(const DevLib &lib, double fwln_min, double fwln_max, double z, int &seg0,
                                          int &seg_n) {
  const double ui0 = phot_ui0(lib, z);
  const double u0 = phot_u(lib, fwln_min, ui0), u1 = phot_u(lib, fwln_max, ui0);
  if (!(isfinite(u0) && isfinite(u1))) {   // non-finite redshift: no pixels
    seg0 = 0;
    seg_n = 0;
    return;
  }
  const double top = (double)(lib.N - 2);
  seg0 = (int)fmin(fmax(floor(u0), 0.0), top);
  seg_n = (int)fmin(fmax(floor(u1), 0.0), top) + 2 - seg0;
}

// Nodes by which a spectrum's span reaches past its pixels' rest range on each side: five
// of the widest LSF row's dispersions (the rows' cut) and two nodes.
__host__ __device__ inline double spec_span_ext(double ksig_max, double inv_dlnw) {
  return 5.0 * ksig_max * inv_dlnw + 2.0;
}

// Rest-frame pixels [seg0, seg0 + seg_n) that the banded LSF rows of a spectrum at redshift
// z read on a log-uniform grid: the pixels' rest range widened by spec_span_ext, clamped to
// the grid (none for a non-finite redshift).
__device__ __forceinline__ void spec_span(const DevLib &lib, double lnpix_lo, double lnpix_hi, double ksig_max, double z,
                                          int &seg0, int &seg_n) {
  const double lnopz = log1p(z);
  const double ext = spec_span_ext(ksig_max, lib.inv_dlnw);
  const double ua = (lnpix_lo - lnopz - lib.lnw0) * lib.inv_dlnw - ext;
  const double ub = (lnpix_hi - lnopz - lib.lnw0) * lib.inv_dlnw + ext;
  if (!(isfinite(ua) && isfinite(ub))) {
    seg0 = 0;
    seg_n = 0;
    return;
  }
  const double top = (double)(lib.N - 1);
  seg0 = (int)fmin(fmax(floor(ua), 0.0), top);
  seg_n = (int)fmin(fmax(ceil(ub), 0.0), top) + 1 - seg0;
}

// ---------------------------------------------------------------- contraction tiles
// Forward launches on a log-uniform grid skip the (M tile, N tile) pairs whose 64 model
// pixels no row of the M tile reads (its span, PointRow seg0/seg_n).  k_tile_list writes
// the others as a list: count at list[0], then (mt << 16) | nt, in N-tile-major order
// (16-bit kernel: the XCDs split the library columns) or M-tile-major order (FP32 kernel:
// an XCD keeps its weight rows in L2).  Block b goes to XCD b mod 8, and XCD x takes the
// x-th eighth of the list, so the blocks that do work are dealt evenly; blocks past the
// list return at once (returns false).
constexpr int kSpanTile = 64;          // model pixels per contraction N tile
constexpr int kTileListMaxM = 1024;    // M tiles a tile list can hold
// Ints of the tile-list buffer for up to Bp rows: the count, the pairs, then each 64-row
// M tile's span in N tiles (lo, hi)
__host__ __device__ inline size_t tile_list_ints(size_t Bp, int N_pad) {
  const size_t m64 = (Bp + 63) / 64;
  return 1 + m64 * (size_t)(N_pad / kSpanTile) + 2 * m64;
}
__device__ __forceinline__ bool span_block_tile(const int *__restrict__ list, int &mt, int &nt) {
  const int count = list[0];
  const int per = (count + 7) >> 3;
  const int x = blockIdx.x & 7, l = blockIdx.x >> 3;
  const int logical = x * per + l;
  if (l >= per || logical >= count) return false;
  const int v = list[1 + logical];
  mt = v >> 16;
  nt = v & 0xffff;
  return true;
}

// Block -> (M tile, N tile) for the library contractions.  The hardware deals
// consecutive blocks round-robin to the 8 XCDs; XCD x takes the consecutive tiles
// [x*nblk/8, (x+1)*nblk/8) of the order (N tile, then M tile), so the XCDs split the
// library columns and each holds a share of every M tile (M tiles differ in their
// active K-tile counts).  The M tiles of an N tile are rotated so that the blocks
// l, l+32, l+64, ... of an XCD (32 CUs), which tend to share a CU, come from M tiles
// spread over the batch; blocks_per_cu is the occupancy the kernel is built for.
__device__ __forceinline__ void balanced_tile(int n_mt, int n_nt, int blocks_per_cu, int &mt, int &nt) {
  const int nblk = gridDim.x, bid = blockIdx.x;
  if ((nblk & 7) != 0) {
    mt = bid / n_nt;
    nt = bid - mt * n_nt;
    return;
  }
  const int per = nblk >> 3, l = bid >> 3;
  const int logical = (bid & 7) * per + l;
  const int n = logical / n_mt, mm = logical - n * n_mt;
  const int grp = n_mt < 32 ? 32 / n_mt : 1;                       // N tiles between blocks l and l+32
  const int rot = n_mt > blocks_per_cu ? n_mt / blocks_per_cu : 1;
  mt = (mm + rot * (n / grp)) % n_mt;
  nt = n;
}

// K-tile ranges a contraction launch leaves out, in 32-wide tiles: [lo0, hi0) and
// [lo1, hi1) (empty ranges: nothing left out).  The escape-geometry passes use them to
// split the K order between the attenuated and the dust-free parts.
struct TileSkip {
  int lo0, hi0, lo1, hi1;
};

// Active K-tile list of the M tile whose rows start at m0: OR of the rows' occupancy
// bits (one bit per 32-wide K tile, mask_words words per row), less the skipped ranges,
// grouped into tiles of 32*tf; the young tiles come first in the K order, so the list
// starts with them.  Run by the whole block; s_tl receives the tile ids in order, s_or
// is 64 words of scratch, s_n two ints.  Returns the list length and the count of young
// tiles.
__device__ __forceinline__ void block_tile_list(const uint32_t *__restrict__ rowmask, int mask_words, int m0, int MT,
                                                int tf, int n_tiles32, int young_tiles32, int *s_tl, uint32_t *s_or,
                                                int *s_n, int &n_act, int &n_young, TileSkip skip = TileSkip{0, 0, 0, 0}) {
  const int tid = threadIdx.x;
  if (tid < 64) s_or[tid] = 0u;
  __syncthreads();
  const uint32_t *rm = rowmask + (size_t)m0 * mask_words;
  for (int idx = tid; idx < MT * mask_words; idx += blockDim.x) {
    const uint32_t v = rm[idx];
    if (v) atomicOr(&s_or[idx % mask_words], v);
  }
  __syncthreads();
  if (tid < 64) {   // one wave: ballot over 64 tiles at a time, positions by prefix popcount
    const int n_tiles = (n_tiles32 + tf - 1) / tf, y_tiles = young_tiles32 / tf;
    int count = 0, ycount = 0;
    for (int base = 0; base < n_tiles; base += 64) {
      const int t = base + tid;
      bool on = false;
      if (t < n_tiles)
        for (int q = 0; q < tf; ++q) {
          const int t32 = t * tf + q;
          const bool skipped = (t32 >= skip.lo0 && t32 < skip.hi0) || (t32 >= skip.lo1 && t32 < skip.hi1);
          if (t32 < n_tiles32 && !skipped) on |= ((s_or[t32 >> 5] >> (t32 & 31)) & 1u) != 0u;
        }
      const unsigned long long bal = __ballot(on);
      if (on) s_tl[count + __popcll(bal & ((1ull << tid) - 1ull))] = t;
      count += __popcll(bal);
      const unsigned long long yb = __ballot(on && t < y_tiles);
      ycount += __popcll(yb);
    }
    if (tid == 0) {
      s_n[0] = count;
      s_n[1] = ycount;
    }
  }
  __syncthreads();
  n_act = s_n[0];
  n_young = s_n[1];
}

// The skipped K ranges of a contraction launch over an N tile (above_lyman: the tile
// starts at or above 912 A):
// pass 0 (the attenuated sum) leaves out the ionising rows under the picket fence, and
// above the Lyman limit (where they are zero) under either geometry; pass 1 (the picket
// fence's dust-free part) keeps only the young stellar rows and the ionising rows.
__host__ __device__ inline TileSkip escape_skip(const DevLib &lib, int pass, bool above_lyman) {
  TileSkip s{0, 0, 0, 0};
  if (!lib.escape) return s;
  const int i0 = lib.ion_k0 / kKTile, i1 = lib.K_old0 / kKTile;
  if (pass == 0) {
    if (lib.escape == 2 || above_lyman) {
      s.lo0 = i0;
      s.hi0 = i1;
    }
  } else {
    s.lo0 = lib.line_k0 / kKTile;   // the line rows (tile-aligned under the picket fence)
    s.hi0 = i0;
    s.lo1 = above_lyman ? i0 : i1;
    s.hi1 = lib.K_pad / kKTile;
  }
  return s;
}

// ---------------------------------------------------------------- device helpers
// index j with x[j] <= v < x[j+1], limited to [0, n-2]
template <typename T>
__device__ __forceinline__ int bracket(const T *x, int n, T v) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// first index j with x[j] >= v (n if none)
template <typename T>
__device__ __forceinline__ int lower_bound_dev(const T *x, int n, T v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (x[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// K position of SSP node (alpha ia, metallicity m, age a) in the young-first order:
// young ages (a < n_young) first, then the line rows, then old ages, each segment
// padded; inside a segment age-major (a, m, ia) or metallicity-major (m, ia, a).
__device__ __forceinline__ int kpos_of(const DevLib &lib, int ia, int m, int a) {
  const int nz = lib.n_z, nf = lib.n_afe, ny = lib.n_young;
  if (a < ny) return lib.zmajor ? (m * nf + ia) * ny + a : (a * nz + m) * nf + ia;
  const int no = lib.n_age - ny, ao = a - ny;
  return lib.K_old0 + (lib.zmajor ? (m * nf + ia) * no + ao : (ao * nz + m) * nf + ia);
}

// k with wave[k] <= lr < wave[k+1] (lr inside the grid), limited to [0, N-2]
__device__ __forceinline__ int wave_bracket(const DevLib &lib, double lr) {
  if (lib.log_uniform) {
    int k = (int)floor((log(lr) - lib.lnw0) * lib.inv_dlnw);
    k = min(max(k, 0), lib.N - 2);
    while (k > 0 && lib.wave_d[k] > lr) --k;
    while (k < lib.N - 2 && lib.wave_d[k + 1] <= lr) ++k;
    return k;
  }
  return bracket(lib.wave_d, lib.N, lr);
}

// as wave_bracket with ln(lr) supplied by the caller
__device__ __forceinline__ int wave_bracket_ln(const DevLib &lib, double lr, double lnlr) {
  if (lib.log_uniform) {
    int k = (int)floor((lnlr - lib.lnw0) * lib.inv_dlnw);
    k = min(max(k, 0), lib.N - 2);
    while (k > 0 && lib.wave_d[k] > lr) --k;
    while (k < lib.N - 2 && lib.wave_d[k + 1] <= lr) ++k;
    return k;
  }
  return bracket(lib.wave_d, lib.N, lr);
}

// same in ln(lambda): k with lnwave[k] <= x < lnwave[k+1]
__device__ __forceinline__ int lnwave_bracket(const DevLib &lib, double x) {
  if (lib.log_uniform) {
    int k = (int)floor((x - lib.lnw0) * lib.inv_dlnw);
    k = min(max(k, 0), lib.N - 2);
    while (k > 0 && lib.lnwave_d[k] > x) --k;
    while (k < lib.N - 2 && lib.lnwave_d[k + 1] <= x) ++k;
    return k;
  }
  return bracket(lib.lnwave_d, lib.N, x);
}

// first j with lnwave[j] >= x
__device__ __forceinline__ int lnwave_lower_bound(const DevLib &lib, double x) {
  if (lib.log_uniform) {
    int j = (int)ceil((x - lib.lnw0) * lib.inv_dlnw);
    j = min(max(j, 0), lib.N);
    while (j > 0 && lib.lnwave_d[j - 1] >= x) --j;
    while (j < lib.N && lib.lnwave_d[j] < x) ++j;
    return j;
  }
  return lower_bound_dev(lib.lnwave_d, lib.N, x);
}

// bracketing node j and fraction t of x on a 1-D grid, clamped (metallicity split of App. B)
__device__ __forceinline__ void grid_split_dev(const double *nodes, int n, double x, int &j, double &t,
                                               bool &inside) {
  double xc = x;
  inside = true;
  if (xc < nodes[0]) { xc = nodes[0]; inside = false; }
  if (xc > nodes[n - 1]) { xc = nodes[n - 1]; inside = false; }
  int jj = 0;
  while (jj + 1 < n - 1 && nodes[jj + 1] <= xc) ++jj;
  j = jj;
  t = (xc - nodes[jj]) / (nodes[jj + 1] - nodes[jj]);
}

// IGM (Sec. 2.6): the Madau (1995) optical depth of the Lyman-series forest (Ly alpha to
// Ly delta, A_j (lambda/lambda_j)^3.46 where lambda_j < lambda < lambda_j (1 + z)) and of
// Lyman-limit systems below the source's limit, at observed wavelength lam (A).
template <typename T>
__device__ __forceinline__ T igm_tau(T lam, T z) {
  const T xe = (T)1 + z;
  T tau = (T)0;
  auto series = [&](T lj, T aj) {   // Lyman alpha .. delta
    if (lam > lj && lam < lj * xe) tau += aj * exp((T)3.46 * log(lam / lj));
  };
  series((T)1215.67, (T)3.6e-3);
  series((T)1025.72, (T)1.7e-3);
  series((T)972.54, (T)1.2e-3);
  series((T)949.74, (T)9.3e-4);
  const T xc = lam / (T)911.75;
  if (xc > (T)1 && xc < xe) {
    const T lc = log(xc), le = log(xe);
    auto pw = [](T l, T e) { return exp(e * l); };
    tau += (T)0.25 * xc * xc * xc * (pw(le, (T)0.46) - pw(lc, (T)0.46)) +
           (T)9.4 * pw(lc, (T)1.5) * (pw(le, (T)0.18) - pw(lc, (T)0.18)) -
           (T)0.7 * xc * xc * xc * (pw(lc, (T)-1.32) - pw(le, (T)-1.32)) - (T)0.023 * (pw(le, (T)1.68) - pw(lc, (T)1.68));
  }
  return tau;
}

// Damping wing of a partly neutral IGM (Miralda-Escude 1998, Totani et al. 2006): neutral
// fraction x between z = 6 and the source at z.  Redward of the source's Lyman alpha the
// scattering wing integrated through the region, x tau_GP(z) (R_alpha / pi) ((1 + z_o) /
// (1 + z))^1.5 [I(x_u) - I(x_l)] with I the antiderivative of t^4.5 / (1 - t)^2, x_u = (1 +
// z) / (1 + z_o), x_l = 7 / (1 + z_o); blueward, inside the region, the Gunn-Peterson
// depth x tau_GP(z_o); tau_GP(z) = 3.88e5 ((1 + z) / 7)^1.5.
__device__ __forceinline__ double igm_damping_I(double t) {
  const double s = sqrt(t);
  return t * t * t * t * s / (1.0 - t) + (9.0 / 7.0) * t * t * t * s + 1.8 * t * t * s + 3.0 * t * s + 9.0 * s -
         4.5 * log((1.0 + s) / (1.0 - s));
}
__device__ __forceinline__ double igm_damping_tau(double lam, double z, double x) {
  const double zl = 6.0, opz_o = lam / 1215.67, opz = 1.0 + z;
  if (!(z > zl) || x == 0.0) return 0.0;
  const double gp = 3.88e5 / (7.0 * 2.6457513110645906);   // tau_GP / (1 + z)^1.5
  if (opz_o > opz) {
    const double r_alpha = 6.265e8 * 1215.67e-8 / (4.0 * kPi * kC_cms);
    return x * gp * opz_o * sqrt(opz_o) * (r_alpha / kPi) *
           (igm_damping_I(opz / opz_o) - igm_damping_I((1.0 + zl) / opz_o));
  }
  if (opz_o > 1.0 + zl) return x * gp * opz_o * sqrt(opz_o);
  return 0.0;
}
// Damped Lyman-alpha absorber (Tepper-Garcia 2006): column 10^lnh cm^-2 at zd, Doppler
// parameter 10 km/s; N (pi e^2 / m_e c) f H(a, x) / (sqrt(pi) dnu_D), x = (nu - nu_alpha) /
// dnu_D in the absorber's frame, H by Tepper-Garcia's approximation (for x^2 < 1e-4 its
// limit H0 - a (2 - 4 x^2 + 5/3 x^4) / sqrt(pi), free of the cancellation).
__device__ __forceinline__ double igm_dla_tau(double lam, double zd, double lnh) {
  const double lam_a = 1215.67e-8, dnu_d = 10.0e5 / lam_a;
  const double a = 6.265e8 / (4.0 * kPi * dnu_d);
  const double x = (kC_cms * (1.0 + zd) / (lam * 1e-8) - kC_cms / lam_a) / dnu_d;
  const double u = x * x, h0 = exp(-u);
  const double corr = u < 1e-4 ? 2.0 - 4.0 * u + (5.0 / 3.0) * u * u
                               : (h0 * h0 * (4.0 * u * u + 7.0 * u + 4.0 + 1.5 / u) - 1.5 / u - 1.0) / u;
  const double H = h0 - a * corr * 0.56418958354775628;   // 1 / sqrt(pi)
  // pi e^2 / (m_e c) f_alpha / sqrt(pi), cgs
  const double k = kPi * 4.80320471e-10 * 4.80320471e-10 / (9.1093837015e-28 * kC_cms) * 0.4164 * 0.56418958354775628;
  return exp10(lnh) * k * H / dnu_d;
}

// IGM transmission of a point (theta row th) at observed wavelength lam: 1 without the IGM;
// the Madau depth (blueward of Ly alpha) scaled by igm_factor, plus the damping wing and
// the absorber where the library has them.
__device__ __forceinline__ double igm_T(const DevLib &lib, const double *th, double z, double lam) {
  if (!lib.igm) return 1.0;
  double tau = lam < 1215.67 * (1.0 + z) ? th[lib.th_igm] * igm_tau<double>(lam, z) : 0.0;
  if (lib.igm & 2) tau += igm_damping_tau(lam, z, th[lib.th_xhi]);
  if (lib.igm & 4) tau += igm_dla_tau(lam, th[lib.th_nhi + 1], th[lib.th_nhi]);
  return tau == 0.0 ? 1.0 : exp(-tau);
}


}  // namespace sps

// ---------------------------------------------------------------- host launchers
namespace sps {
struct Workspace;
}
