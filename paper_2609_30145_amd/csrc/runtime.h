// Host-side objects behind the C ABI handles.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <map>
#include <vector>

#include "../../include/sps.h"
#include "common.h"

namespace sps {

sps_status fail(sps_status code, const char *fmt, ...);

// Owns a set of device allocations.
// A host-side first-fit sub-allocator over one device allocation: alloc and free make no
// HIP call (so they never wait on running kernels); blocks are 256-byte aligned.  Used by
// one thread at a time.
struct DeviceArena {
  char *base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_blocks;   // offset -> length
  ~DeviceArena();
  bool init(size_t n);
  void *alloc(size_t n);
  void free(void *p, size_t n);
};

struct DeviceBuffers {
  std::vector<void *> ptrs;
  std::vector<size_t> sizes;
  int64_t bytes = 0;
  DeviceArena *arena = nullptr;   // set: blocks come from (and return to) the arena
  ~DeviceBuffers();
  void release();
  void *alloc(size_t n);
  void *upload(const void *h, size_t n);
};

// Per-observation workspace, sized once for max_batch rows.
struct Workspace {
  DeviceBuffers mem;
  int max_batch = 0, B_pad_max = 0, mask_words = 0;
  double *keys = nullptr;       // batch-ordering keys [B_pad]
  int *ranks = nullptr;          // each point's row in the key order [B_pad]
  void *W = nullptr;             // B_pad * K_pad * 8 bytes
  uint32_t *rowmask = nullptr;
  PointRow *rows = nullptr;
  void *F = nullptr, *Yatt = nullptr;   // B_pad * N_pad * 8 bytes each
  int *tiles = nullptr;          // the contraction's tile list (k_tile_list): 1 + (B_pad/64) * (N_pad/64) ints,
                                 // then each M tile's span in N tiles (2 * B_pad/64 ints)
  bool f_spans = false;          // the last forward pass formed F (and Yatt) only over the rows' spans
  double *Lline = nullptr;
  double *WQ = nullptr;          // nebular continuum: photon-weighted masses [B_pad][nebular ages]
  double *gvec = nullptr, *gnoise = nullptr;
  double *gbuf = nullptr;        // adjoint per-point sums [B_pad][16]
  double *mbuf = nullptr;        // model at sorted rows [B_pad][n_data] (gradient pass)
  double *scr = nullptr;         // adjoint per-node / per-pixel scratch [B_pad][ld_scr]; calibration sums
  int ld_scr = 0;
  double *dLl = nullptr;         // adjoint d logL / d L_line [B_pad][n_line]
  void *G = nullptr;             // adjoint [B_pad][N_pad] float/double
  void *dW = nullptr;            // adjoint [2][B_pad_max][K_pad] double (two wavelength halves)
  unsigned long long *counter = nullptr;
  sps_status create(const sps_library *L, int max_batch, int n_data, int n_fnodes, bool forward_only = false);
};

// Host copy of an observation's fixed operators and data.
struct ObsHost {
  int kind = 0, n_data = 0, noise_flags = 0, lsf_mode = 0;
  std::vector<int> band_off;
  std::vector<double> fw, fwln, fr;
  std::vector<float> fr_f;
  std::vector<double> pix, lnpix, ksig, lsf_vals;
  double lsf_value = 0, sigma_gas = 0;
  std::vector<double> data, sigma;
  std::vector<uint8_t> mask;
  // constant-noise form of the likelihood: 1/sigma^2 (0 where masked) and
  // -1/2 sum ln(2 pi sigma^2) over the included data
  std::vector<double> ivar;
  double lnorm = 0;
  int calib_mode = 0, calib_order = 0;
  std::vector<double> calib_prior;
  double calib_xs = 0, calib_x0 = 0;
  std::vector<int> loff, lidx;       // line catalogue blends
  std::vector<uint8_t> upper;
  int vd_M = 0, vd_nfft = 0, vd_log2 = 0;   // Fourier stage of a free sigma_gal
  double vd_lnlo = 0, vd_lnhi = 0, vd_dlnl = 0;
  std::vector<double> vd_tw;
  int lm_mode = 0;                   // line-flux marginalisation (spectra)
  int lm_most = 0;                   //   most library lines in a rest interval as wide as the pixels
  double lm_frac = 0;
  std::vector<uint8_t> lm_flat;
};

sps_status build_obs_operators(const sps_library *L, const sps_obs_desc *d, ObsHost &h, uint32_t *warnings);
sps_status set_obs_data(ObsHost &h, const double *data, const double *sigma, const uint8_t *mask);

}  // namespace sps

struct sps_library {
  int device = 0;                  // -1: host-only (layout and operators, no device copies)
  double logz_lo = 0, logz_hi = 0, afe_lo = 0, afe_hi = 0;
  std::vector<double> wave_h;      // host copy of the wavelength grid
  std::vector<double> line_wave_h; // host copy of the line wavelengths (rest Angstrom)
  int n_age = 0, n_z = 0, n_afe = 0, N = 0, n_young = 0, n_line = 0, n_sfh = 0, n_zh = 0;
  int line_k0 = 0;
  bool line_tau_axis = false;      // the line table came on an age axis of its own
  uint32_t precisions = 0;
  sps::DevLib dev;
  int *kpos_d = nullptr;
  // the line profiles on the model grid in FP64, compactly: line l's nonzero nodes start at
  // lprof_k0[l], lprof_len[l] <= lprof_w of them (joint line marginalisation with photometry)
  const double *lprof_d = nullptr;
  const int *lprof_k0_d = nullptr, *lprof_len_d = nullptr;
  int lprof_w = 0;
  sps::DeviceBuffers mem;
  void host_wave(std::vector<double> &w) const;   // copies wave[N] from the device
};

struct sps_obs {
  const sps_library *lib = nullptr;
  sps::ObsHost host;
  sps::DevObs dobs;
  sps::DevObs *dev_obs = nullptr;
  sps::DeviceBuffers opmem;        // operators and data
  sps::Workspace ws;
  // contraction timing
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  size_t ev_next = 0, ev_pending = 0;
  double ms_total = 0;
  int64_t launches = 0, dense_tiles = 0, dense_per_launch = 0;
  ~sps_obs();
  sps_status upload_operators();
  sps_status upload_data();
  sps_status enable_timing(bool on);
  hipError_t timing_events(int n_mtiles, int n_ktiles, hipEvent_t *start, hipEvent_t *stop);
  sps_status read_timing(double *ms, int64_t *launches, int64_t *exec_tiles, int64_t *dense_tiles);
};

namespace sps {
sps_status run_forward(const sps_library *L, sps_obs *o, const double *theta, int B, int prec, double *logl,
                       double *model, bool want_grad_buffers, hipStream_t s);
sps_status run_adjoint(const sps_library *L, sps_obs *o, const double *theta, int B, int prec, double *grad,
                       hipStream_t s);
// The forward launch sequence on an explicit workspace and observation table
// (point_obs: observation slot per point, NULL = slot 0).  `one` is the host side of the
// observation when every point has the same one (NULL on the serving path, which mixes
// observations): line catalogues, calibration polynomials and a free sigma_gal need it.
// keep_sorted_model: the model at the sorted rows stays in w.mbuf; joint: the catalogue of
// a joint line marginalisation (its cat, cat_model, cat_ld fields), or NULL.
struct LineMargLaunch;
constexpr int kLineCatMaxHost = 256;   // catalogue entries of a joint marginalisation
sps_status launch_forward(const sps_library *L, Workspace &w, const DevObs *obs_table, const int *point_obs,
                          const double *theta, int B, int prec, double *logl, double *model, int ld_model,
                          bool grad, int ld_g, const ObsHost *one, sps_obs *timing_obs, hipStream_t s,
                          bool keep_sorted_model = false, const LineMargLaunch *joint = nullptr);
bool precision_built(const sps_library *L, int p);
// Device address of the allocation-free entry point's static scratch on `device`, looked
// up once per device (called by sps_library_load).
sps_status static_scratch_init(int device);
// Device copies of an observation's operators and data (used by sps_obs and the server).
sps_status upload_obs(const ObsHost &h, DevObs &o, DeviceBuffers &mem, hipStream_t s);
int64_t obs_device_bytes(const ObsHost &h);
}  // namespace sps
