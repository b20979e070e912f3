// Observation operators, workspaces and contraction timing.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"

using namespace sps;

void sps_library::host_wave(std::vector<double> &w) const { w = wave_h; }

sps_status Workspace::create(const sps_library *L, int mb, int n_data, int n_fnodes, bool forward_only) {
  const DevLib &g = L->dev;
  max_batch = mb;
  B_pad_max = (mb + kMAlign - 1) / kMAlign * kMAlign;
  const size_t Bp = B_pad_max;
  mask_words = (g.K_pad / kKTile + 31) / 32;
  bool ok = true;
  auto al = [&](size_t n) {
    void *p = mem.alloc(n);
    ok = ok && p;
    return p;
  };
  keys = (double *)al(Bp * 8);
  ranks = (int *)al(Bp * 4);
  W = al(Bp * g.K_pad * 8);
  rowmask = (uint32_t *)al(Bp * mask_words * 4);
  rows = (PointRow *)al(Bp * sizeof(PointRow));
  F = al(Bp * g.N_pad * 8);
  tiles = (int *)al(tile_list_ints(Bp, g.N_pad) * 4);
  const size_t gb = forward_only ? 1 : Bp;   // gradient-pass buffers
  Yatt = al(gb * g.N_pad * 8);
  Lline = (double *)al(Bp * (size_t)std::max(1, g.n_line) * 8);
  if (g.has_cont) WQ = (double *)al(Bp * (size_t)(g.neb_a1 - g.neb_a0) * 8);
  gvec = (double *)al(gb * (size_t)std::max(1, n_data) * 8);
  gnoise = (double *)al(gb * 4 * 8);
  gbuf = (double *)al(gb * 16 * 8);
  mbuf = (double *)al(gb * (size_t)std::max(1, n_data) * 8);
  ld_scr = std::max(std::max(3 * n_fnodes, 8 * n_data), 24);   // also the calibration sums
  scr = (double *)al(gb * (size_t)std::max(1, ld_scr) * 8);
  dLl = (double *)al(gb * (size_t)std::max(1, g.n_line) * 8);
  G = al(gb * g.N_pad * 8 * 2);
  dW = al(gb * g.K_pad * 8 * 2);   // FP32 gradient: two wavelength halves
  counter = (unsigned long long *)al(8);
  if (!ok) return fail(SPS_E_NOMEM, "workspace allocation failed (max_batch=%d)", mb);
  if (hipMemset(counter, 0, 8) != hipSuccess) return fail(SPS_E_HIP, "hipMemset failed");
  return SPS_OK;
}

sps_obs::~sps_obs() {
  for (auto e : ev_start) (void)hipEventDestroy(e);
  for (auto e : ev_stop) (void)hipEventDestroy(e);
}

namespace sps {

static size_t r256(size_t n) { return (n + 255) / 256 * 256; }

int64_t obs_device_bytes(const ObsHost &h) {
  size_t b = 0;
  if (h.kind == SPS_OBS_PHOT) {
    b += r256(h.band_off.size() * 4) + 3 * r256(h.fw.size() * 8) + r256(h.fw.size() * 4);
  } else {
    b += 3 * r256(h.pix.size() * 8) + (h.lsf_vals.empty() ? 0 : r256(h.lsf_vals.size() * 8));
  }
  b += 3 * r256((size_t)h.n_data * 8) + r256((size_t)h.n_data) + r256(h.vd_tw.size() * 8) + r256(h.lm_flat.size());
  return (int64_t)b;
}

// Uploads operators and data of an observation into `mem` (asynchronously on `s`;
// the host vectors must stay alive until `s` has drained).
sps_status upload_obs(const ObsHost &host, DevObs &o, DeviceBuffers &mem, hipStream_t s) {
  memset(&o, 0, sizeof o);
  o.kind = host.kind;
  o.n_data = host.n_data;
  o.noise_flags = host.noise_flags;
  bool ok = true;
  auto put = [&](const void *h, size_t n) -> void * {
    void *p = mem.alloc(n);
    if (!p) {
      ok = false;
      return nullptr;
    }
    if (h && hipMemcpyAsync(p, h, n, hipMemcpyHostToDevice, s) != hipSuccess) ok = false;
    return p;
  };
  if (host.kind == SPS_OBS_PHOT) {
    o.n_band = host.n_data;
    o.n_fnodes = (int)host.fw.size();
    o.band_off = (const int *)put(host.band_off.data(), host.band_off.size() * 4);
    o.fw = (const double *)put(host.fw.data(), host.fw.size() * 8);
    o.fwln = (const double *)put(host.fwln.data(), host.fwln.size() * 8);
    o.fr_d = (const double *)put(host.fr.data(), host.fr.size() * 8);
    o.fr_f = (const float *)put(host.fr_f.data(), host.fr_f.size() * 4);
    o.fwln_min = o.fwln_max = host.fwln.empty() ? 0.0 : host.fwln[0];
    for (double v : host.fwln) {
      o.fwln_min = std::min(o.fwln_min, v);
      o.fwln_max = std::max(o.fwln_max, v);
    }
  } else if (host.kind == SPS_OBS_SPEC) {
    o.pix = (const double *)put(host.pix.data(), host.pix.size() * 8);
    o.lnpix = (const double *)put(host.lnpix.data(), host.lnpix.size() * 8);
    o.ksig = (const double *)put(host.ksig.data(), host.ksig.size() * 8);
    o.lsf_mode = host.lsf_mode;
    o.lsf_value = host.lsf_value;
    o.has_curve = host.lsf_vals.empty() ? 0 : 1;
    if (o.has_curve) o.lsf_vals = (const double *)put(host.lsf_vals.data(), host.lsf_vals.size() * 8);
    o.sigma_gas_kms = host.sigma_gas;
    o.ksig_max = 0.0;
    for (double v : host.ksig) o.ksig_max = std::max(o.ksig_max, v);
    o.lnpix_lo = host.lnpix.empty() ? 0.0 : host.lnpix.front();
    o.lnpix_hi = host.lnpix.empty() ? 0.0 : host.lnpix.back();
    o.calib_mode = host.calib_mode;
    o.calib_order = host.calib_order;
    o.calib_xs = host.calib_xs;
    o.calib_x0 = host.calib_x0;
    o.calib_lnsd = 0.0;
    for (int m = 0; m < 8; ++m) o.calib_ivar[m] = 0.0;
    for (size_t m = 0; m < host.calib_prior.size() && m < 8; ++m) {
      o.calib_ivar[m] = 1.0 / (host.calib_prior[m] * host.calib_prior[m]);
      o.calib_lnsd += std::log(host.calib_prior[m]);
    }
  }
  if (host.kind == SPS_OBS_LINES) {
    o.loff = (const int *)put(host.loff.data(), host.loff.size() * 4);
    o.lidx = (const int *)put(host.lidx.data(), std::max<size_t>(1, host.lidx.size()) * 4);
    o.upper = (const uint8_t *)put(host.upper.data(), host.upper.size());
  }
  if (host.lm_mode) {
    o.lm_mode = host.lm_mode;
    o.lm_frac = host.lm_frac;
    if (!host.lm_flat.empty()) o.lm_flat = (const uint8_t *)put(host.lm_flat.data(), host.lm_flat.size());
  }
  if (host.vd_nfft > 0) {
    o.vd_M = host.vd_M;
    o.vd_nfft = host.vd_nfft;
    o.vd_log2 = host.vd_log2;
    o.vd_lnlo = host.vd_lnlo;
    o.vd_lnhi = host.vd_lnhi;
    o.vd_dlnl = host.vd_dlnl;
    o.vd_tw = (const double *)put(host.vd_tw.data(), host.vd_tw.size() * 8);
  }
  o.data = (const double *)put(host.data.data(), (size_t)host.n_data * 8);
  o.sigma = (const double *)put(host.sigma.data(), (size_t)host.n_data * 8);
  o.mask = (const uint8_t *)put(host.mask.data(), (size_t)host.n_data);
  o.ivar = (const double *)put(host.ivar.data(), (size_t)host.n_data * 8);
  o.lnorm = host.lnorm;
  if (!ok) return fail(SPS_E_NOMEM, "observation upload failed");
  return SPS_OK;
}

}  // namespace sps

sps_status sps_obs::upload_operators() {
  sps_status st = upload_obs(host, dobs, opmem, nullptr);
  if (st != SPS_OK) return st;
  dev_obs = (DevObs *)opmem.alloc(sizeof(DevObs));
  if (!dev_obs) return fail(SPS_E_NOMEM, "observation upload failed");
  if (hipMemcpy(dev_obs, &dobs, sizeof(DevObs), hipMemcpyHostToDevice) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return fail(SPS_E_HIP, "observation upload failed");
  return SPS_OK;
}

sps_status sps_obs::upload_data() {
  const size_t n = host.n_data;
  hipError_t e = hipMemcpy((void *)dobs.data, host.data.data(), n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((void *)dobs.sigma, host.sigma.data(), n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((void *)dobs.mask, host.mask.data(), n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((void *)dobs.ivar, host.ivar.data(), n * 8, hipMemcpyHostToDevice);
  dobs.lnorm = host.lnorm;
  if (e == hipSuccess) e = hipMemcpy(dev_obs, &dobs, sizeof(DevObs), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(SPS_E_HIP, "observation data upload failed: %s", hipGetErrorString(e));
  return SPS_OK;
}

// ---------------------------------------------------------------- timing
static constexpr size_t kEvents = 64;

sps_status sps_obs::enable_timing(bool on) {
  if (on && ev_start.empty()) {
    ev_start.resize(kEvents);
    ev_stop.resize(kEvents);
    // timing-only events: no system-scope fence at record, so that recording them costs
    // no cache writeback and invalidation between the kernels they bracket
    for (size_t i = 0; i < kEvents; ++i) {
      if (hipEventCreateWithFlags(&ev_start[i], hipEventDisableSystemFence) != hipSuccess ||
          hipEventCreateWithFlags(&ev_stop[i], hipEventDisableSystemFence) != hipSuccess)
        return fail(SPS_E_HIP, "hipEventCreateWithFlags failed");
    }
  }
  timing = on;
  ev_next = ev_pending = 0;
  ms_total = 0;
  launches = dense_tiles = 0;
  if (hipMemset(ws.counter, 0, 8) != hipSuccess) return fail(SPS_E_HIP, "hipMemset failed");
  return SPS_OK;
}

// The pair of events for the next timed contraction launch: the launch hands them to the
// kernel's dispatch, which stamps its own start and end (no marker between kernels).
hipError_t sps_obs::timing_events(int n_mtiles, int n_ktiles, hipEvent_t *start, hipEvent_t *stop) {
  *start = *stop = nullptr;
  if (!timing) return hipSuccess;
  const size_t i = ev_next % kEvents;
  if (ev_pending >= kEvents) {   // reuse the oldest pair: fold its time in first
    float ms = 0;
    hipError_t e = hipEventSynchronize(ev_stop[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev_start[i], ev_stop[i]);
    if (e != hipSuccess) return e;
    ms_total += ms;
    --ev_pending;
  }
  dense_tiles += (int64_t)n_mtiles * n_ktiles;   // (M tile, N tile) pairs times K tiles
  *start = ev_start[i];
  *stop = ev_stop[i];
  ++ev_next;
  ++ev_pending;
  ++launches;
  return hipSuccess;
}

sps_status sps_obs::read_timing(double *ms, int64_t *nl, int64_t *exec_tiles, int64_t *dense) {
  if (!timing) return fail(SPS_E_STATE, "timing is not enabled on this observation");
  while (ev_pending > 0) {
    const size_t i = (ev_next - ev_pending) % kEvents;
    float t = 0;
    hipError_t e = hipEventSynchronize(ev_stop[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev_start[i], ev_stop[i]);
    if (e != hipSuccess) return fail(SPS_E_HIP, "event timing failed: %s", hipGetErrorString(e));
    ms_total += t;
    --ev_pending;
  }
  unsigned long long c = 0;
  if (hipMemcpy(&c, ws.counter, 8, hipMemcpyDeviceToHost) != hipSuccess) return fail(SPS_E_HIP, "counter read failed");
  if (ms) *ms = ms_total;
  if (nl) *nl = launches;
  if (exec_tiles) *exec_tiles = (int64_t)c;
  if (dense) *dense = dense_tiles;
  ms_total = 0;
  launches = dense_tiles = 0;
  ev_next = ev_pending = 0;
  if (hipMemset(ws.counter, 0, 8) != hipSuccess) return fail(SPS_E_HIP, "hipMemset failed");
  return SPS_OK;
}
