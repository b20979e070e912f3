// Shared definitions of the request server (host scheduler, device kernels, mock executor).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "common.h"

namespace sps {

// One active request in a tick's batch.
struct DevReq {
  double *theta_cur;   // [B][P] current live points (device, or host for the mock)
  double *logl_cur;    // [B]
  uint64_t seed;
  int off, B, stage, slot;
};

// Box that proposals are kept inside (the stand-in sampler's prior support).
struct ProposalBox {
  double logmass_lo, logmass_hi, z_lo, z_hi, tau_hi, delta_lo, delta_hi;
  double logz_lo, logz_hi, afe_lo, afe_hi;
  double step;         // proposal scale
};

// SplitMix64 output function (Steele, Lea & Flood 2014) used as a counter-based hash.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Standard normal deviate for (seed, stage, point, parameter) by Box-Muller.
__host__ __device__ inline double counter_normal(uint64_t seed, uint64_t stage, uint64_t point, uint64_t param) {
  const uint64_t key = mix64(seed ^ mix64(stage * 0x632be59bd9b4e019ull ^ mix64(point * 0x8cb92ba72f3d8dd7ull ^ param)));
  const uint64_t a = mix64(key), b = mix64(key ^ 0xd6e8feb86659fd93ull);
  const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__host__ __device__ inline double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Gaussian random-walk proposal of one live point inside the box; bin masses are
// perturbed multiplicatively and renormalised to one.
__host__ __device__ inline void propose_point(const double *src, double *dst, int P, int n_sfh, const ProposalBox &bx,
                                              uint64_t seed, uint64_t stage, uint64_t i) {
  for (int c = 0; c < P; ++c) dst[c] = src[c];
  const double s = bx.step;
  auto nrm = [&](int c) { return counter_normal(seed, stage, i, (uint64_t)c); };
  dst[TH_LOGMASS] = clampd(src[TH_LOGMASS] + s * nrm(TH_LOGMASS), bx.logmass_lo, bx.logmass_hi);
  dst[TH_ZRED] = clampd(src[TH_ZRED] + 0.2 * s * nrm(TH_ZRED), bx.z_lo, bx.z_hi);
  dst[TH_TAU_BC] = clampd(src[TH_TAU_BC] + s * nrm(TH_TAU_BC), 0.0, bx.tau_hi);
  dst[TH_TAU_DIFF] = clampd(src[TH_TAU_DIFF] + s * nrm(TH_TAU_DIFF), 0.0, bx.tau_hi);
  dst[TH_DELTA] = clampd(src[TH_DELTA] + s * nrm(TH_DELTA), bx.delta_lo, bx.delta_hi);
  dst[TH_LOGZSOL] = clampd(src[TH_LOGZSOL] + s * nrm(TH_LOGZSOL), bx.logz_lo, bx.logz_hi);
  dst[TH_AFE] = clampd(src[TH_AFE] + 0.5 * s * nrm(TH_AFE), bx.afe_lo, bx.afe_hi);
  double tot = 0.0;
  for (int k = 0; k < n_sfh; ++k) {
    const double m = src[TH_NSCALAR + k] * exp(s * nrm(TH_NSCALAR + k));
    dst[TH_NSCALAR + k] = m;
    tot += m;
  }
  for (int k = 0; k < n_sfh; ++k) dst[TH_NSCALAR + k] /= tot;
}

hipError_t launch_propose(const DevReq *reqs, int n_req, int P, int n_sfh, const ProposalBox &box,
                          double *theta_all, int *point_obs, int n_total, hipStream_t s);
// thr: [n_req] device scratch for the per-request thresholds
hipError_t launch_update(const DevReq *reqs, int n_req, int P, const double *theta_all, const double *logl_all,
                         double *thr, int n_total, hipStream_t s);

}  // namespace sps
