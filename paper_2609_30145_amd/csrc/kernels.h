// Host-side launchers of the gfx950 kernels (one declaration per kernel family).
#pragma once
#include "common.h"

namespace sps {

struct PrepLaunch {
  const double *theta;
  int P, B, B_pad;
  const double *keys;        // batch-ordering keys from launch_keys
  const int *ranks;          // each point's row in the key order, from launch_keys, or NULL
  const DevObs *obs_table;
  const int *point_obs;
  void *W, *Wlo;
  uint32_t *rowmask;
  int mask_words;
  PointRow *rows;
  double *Lline;
  double *WQ;                // [B_pad][nebular ages] photon-weighted masses (continuum), or NULL
  const int *kpos;
  int line_k0;
  int mode;   // 0 f64, 1 f32, 2 bf16, 3 f16
};

size_t prep_smem_bytes(const DevLib &lib, int mode);   // mode as PrepLaunch::mode
// batch-ordering keys (the weight builder ranks the points by them)
// batch-ordering keys and, when ranks is not NULL, each point's rank among them (ties by
// index; the weight builder ranks its own point otherwise)
constexpr int kSmallMtBatch = 256;     // 16-bit contraction: 64-row M tiles up to this padded batch
// forward launches of at most kDenseMaxBpad padded rows whose whole grid fits kDenseMaxBlocks
// blocks (one per CU) skip the tile list: the extra tiles run on otherwise idle CUs, and
// the list kernel's serial latency is saved
constexpr int kDenseMaxBpad = 128, kDenseMaxBlocks = 256;
constexpr int kSelfKeyMaxB = 512;      // batches up to this size: each weight-builder workgroup forms the keys
constexpr int kRankKernelMinB = 2048;   // batches from this size rank in a kernel of their own
hipError_t launch_keys(const DevLib &lib, const double *theta, int P, int B, double *keys, int *ranks,
                       hipStream_t s);
// weights, per-row K-tile occupancy bits and per-point rows, each point at its rank
hipError_t launch_prep(const DevLib &lib, const PrepLaunch &pl, hipStream_t s);

struct ContractLaunch {
  const void *W, *Wlo;       // weights (hi/lo planes for 16-bit)
  int B_pad;
  const uint32_t *rowmask;   // [B_pad][mask_words] K-tile occupancy bits per row (32-wide tiles)
  int mask_words;
  unsigned long long *counter;   // executed K tiles are added here (timing), or NULL
  const PointRow *rows;
  void *F;                   // [B_pad][N_pad] attenuated rest-frame spectrum (float or double)
  void *Yatt;                // optional [B_pad][N_pad]: young part after both attenuations
  int precision;             // sps_precision value
  hipEvent_t ev_start, ev_stop;   // timing: events that take the kernel's own start and end, or NULL
  const int *list;           // span-limited launch: the tile list (launch_tile_list), or NULL: every tile
  int pass;                  // 0: the attenuated sum; 1: the picket fence's dust-free part, added to F
};
// The tile list of a span-limited forward launch: the (M tile, N tile) pairs whose pixels
// some row of the M tile reads (common.h: span_block_tile); list holds 1 + (B_pad/MT) *
// n_nt ints.  N-tile-major for the 16-bit kernel, M-tile-major for FP32.
hipError_t launch_tile_list(const PointRow *rows, int B_pad, int MT, int n_nt, bool nt_major, int *list,
                            hipStream_t s);
// M tile used by the contraction of a precision (the occupancy list granularity)
// (16-bit: 64 rows for batches of at most kSmallMtBatch padded rows, where 128-row tiles
// would leave CUs idle and load the padding rows' weights; 128 otherwise)
int contract_mtile(int precision, int B_pad);
int contract_ktile_factor(int precision);   // K tile in units of kKTile
hipError_t launch_contract(const DevLib &lib, const ContractLaunch &cl, hipStream_t s);

struct ProjectLaunch {
  const DevObs *obs_table;
  const PointRow *rows;
  const void *F;             // float or double [B_pad][N_pad]
  int f64;
  const double *theta;
  int P, B;
  const double *Lline;       // [B_pad][n_line]
  double *model;             // [B][n_data] or NULL
  double *logl;              // [B] or NULL
  double *gvec;              // [B_pad][n_data_max] dlogL/dm (adjoint) or NULL
  double *gnoise;            // [B][4] dlogL/d(noise params) or NULL
  double *msorted;           // [B_pad][ld_g] model at sorted rows or NULL
  int ld_model;              // row stride of model
  int ld_g;
};
hipError_t launch_project(const DevLib &lib, const ProjectLaunch &pl, hipStream_t s);

// spectrum calibration polynomial (App. H.3): the correction to logL from the model at the
// sorted rows (written by the projection), per point
// analytic marginalisation of a spectrum's line fluxes (App. I.3): one workgroup per row,
// after the projection (which leaves the grid model at the sorted rows)
struct LineMargLaunch {
  const DevObs *obs_table;
  const PointRow *rows;
  const double *theta;
  const double *Lline;       // [B_pad][n_line] line luminosities from the weight builder
  const double *msorted;     // [B_pad][ld] grid model at the sorted rows
  int ld;
  double *scr;               // [B_pad][ld_scr] per-row scratch: residuals, weights (ld_scr >= 2 n_pix), then the profiles
  int ld_scr, B_pad;
  double *logl;              // [B] or NULL: overwritten with the marginal likelihood
  // joint marginalisation with a line catalogue of the same points (its rows in the same
  // sorted order): its observation (device) and its model at the sorted rows, or NULL
  const DevObs *cat;
  const double *cat_model;
  int cat_ld;
  // and with a photometric observation of the same points: its observation, its model at
  // the sorted rows, a per-row scratch [B_pad][phot_ld_scr] (band responses, residuals,
  // weights: >= n_band (NM + 2) doubles) and the library's compact FP64 line profiles
  const DevObs *phot;
  const double *phot_model;
  int phot_ld;
  double *phot_scr;
  int phot_ld_scr;
  const double *lprof;
  const int *lprof_k0, *lprof_len;
  int lprof_w;
};
hipError_t launch_linemarg(const DevLib &lib, const LineMargLaunch &lm, hipStream_t s);

struct CalibLaunch {
  const DevObs *obs_table;
  const PointRow *rows;
  const double *theta;
  const double *msorted;     // [B_pad][ld] model at the sorted rows
  int ld, B_pad;
  double *sums;              // [B_pad][ld_sums] per-row sums (S_0..S_14, b_0..b_7), ld_sums >= 23
  int ld_sums;
  double *logl;              // [B] or NULL
};
hipError_t launch_calib(const DevLib &lib, const CalibLaunch &cl, hipStream_t s);

// nebular continuum added to F (App. C); a no-op for a library without a continuum cube
struct NebLaunch {
  const double *theta;
  const PointRow *rows;
  const double *WQ;          // [B_pad][nebular ages] from the weight builder
  void *F;
  const int *list;           // the contraction's tile list, or NULL: every tile
  int B_pad, MT, f64;
};
hipError_t launch_nebular(const DevLib &lib, const NebLaunch &nl, hipStream_t s);

// Fourier stage of a free sigma_gal (Sec. 2.5, App. F): every row's window of F (PointRow
// cov0 / cov_n) broadened in place, one workgroup per pair of sorted rows
struct VdispLaunch {
  const DevObs *obs;         // the observation (device): twiddles and the grid step
  const double *theta;       // [B, P] caller's order
  const PointRow *rows;
  void *F;                   // [B_pad][N_pad] FP32, or FP64 when f64
  int B_pad, nfft, log2n, f64;
};
hipError_t launch_vdisp(const DevLib &lib, const VdispLaunch &vl, hipStream_t s);

// library packing
struct PackLaunch {
  const double *flux;        // [n_afe][n_z][n_age][N] raw
  const double *lineprof;    // [n_line][N] per-A line profiles on the model grid
  const int *ksrc;           // [K_pad]: >= 0 SSP flat index (ia*n_z + m)*n_age + a; -1-l line l; INT_MIN pad
  int neb_mask;              // remove lambda < 912 A from nebular-covered ages
  double *LT64;
  float *LT32, *L32n;
  uint16_t *Hb, *Rb, *Hh, *Rh;
  int *kexp;
  int16_t *kexp16;
  double *Q;                 // [n_afe][n_z][n_young]
  const double *wave;        // [N]
};
hipError_t launch_pack(const DevLib &lib, const PackLaunch &pk, hipStream_t s);

}  // namespace sps
