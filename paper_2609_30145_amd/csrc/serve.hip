// Device side of the request server: stand-in sampler proposals and updates for every
// active request, laid out in one batch (request r owns points [off_r, off_r + B_r)).
#include "serve.h"

namespace sps {

// ---------------------------------------------------------------- proposals
// One wave per point, lanes over the parameters: the same Gaussian random-walk proposal
// as propose_point (counter-based deviates per parameter), with the bin masses'
// normalising sum taken by a wave butterfly (a fixed order).
__global__ void __launch_bounds__(256) k_propose(const DevReq *__restrict__ reqs, int n_req, int P, int n_sfh,
                                                 ProposalBox box, double *__restrict__ theta_all,
                                                 int *__restrict__ point_obs, int n_total) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= n_total) return;   // uniform over the wave
  int lo = 0, hi = n_req - 1;   // last request with off <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].off <= p) lo = mid; else hi = mid - 1;
  }
  const DevReq rq = reqs[lo];
  const int i = p - rq.off;
  const double *src = rq.theta_cur + (size_t)i * P;
  double *dst = theta_all + (size_t)p * P;
  if (lane == 0) point_obs[p] = rq.slot;
  if (rq.stage == 0) {
    for (int c = lane; c < P; c += 64) dst[c] = src[c];
    return;
  }
  const double sstep = box.step;
  const uint64_t seed = rq.seed, stage = (uint64_t)rq.stage, pt = (uint64_t)i;
  double part = 0.0;
  for (int c = lane; c < P; c += 64) {
    double v = src[c];
    if (c >= TH_NSCALAR && c < TH_NSCALAR + n_sfh) {
      v *= exp(sstep * counter_normal(seed, stage, pt, (uint64_t)c));
      part += v;
    } else if (c == TH_LOGMASS) {
      v = clampd(v + sstep * counter_normal(seed, stage, pt, c), box.logmass_lo, box.logmass_hi);
    } else if (c == TH_ZRED) {
      v = clampd(v + 0.2 * sstep * counter_normal(seed, stage, pt, c), box.z_lo, box.z_hi);
    } else if (c == TH_TAU_BC || c == TH_TAU_DIFF) {
      v = clampd(v + sstep * counter_normal(seed, stage, pt, c), 0.0, box.tau_hi);
    } else if (c == TH_DELTA) {
      v = clampd(v + sstep * counter_normal(seed, stage, pt, c), box.delta_lo, box.delta_hi);
    } else if (c == TH_LOGZSOL) {
      v = clampd(v + sstep * counter_normal(seed, stage, pt, c), box.logz_lo, box.logz_hi);
    } else if (c == TH_AFE) {
      v = clampd(v + 0.5 * sstep * counter_normal(seed, stage, pt, c), box.afe_lo, box.afe_hi);
    }
    dst[c] = v;
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  for (int c = lane; c < P; c += 64)
    if (c >= TH_NSCALAR && c < TH_NSCALAR + n_sfh) dst[c] /= part;
}

// ---------------------------------------------------------------- update
// stage 0: record logL(theta0).  stage >= 1: threshold = the logL at rank floor(B/4)
// (ascending, ties by index, NaN as -inf) of the current live points; proposals above
// it replace their point.  One workgroup per request finds the rank-q value by a bitonic
// sort (batches above kUpdMax points count ranks directly); the replacement then runs
// with one wave per point over the whole tick.  Only the value at rank q is needed, and
// equal values are interchangeable, so up to 1024 points are sorted by value alone,
// four per thread in registers: element i = 256 u + tid; partners 256 or more apart are
// in the same thread, partners less than 64 apart in the same wave (shuffles), and only
// the stages at distance 64 and 128 exchange through LDS.
constexpr int kUpdMax = 2048;

__device__ __forceinline__ double bitonic_keep(double v, double other, bool keep_min) {
  return keep_min ? fmin(v, other) : fmax(v, other);
}

// q-th smallest of the (NaN-free) values of a request with B <= 1024 points
__device__ double rank_value_1024(const double *__restrict__ x, int B, int q, double *s) {
  const int tid = threadIdx.x;
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = 256 * u + tid;
    double a = HUGE_VAL;   // padding sorts after every point
    if (i < B) {
      a = x[i];
      if (isnan(a)) a = -HUGE_VAL;
    }
    v[u] = a;
  }
  for (int k = 2; k <= 1024; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 256) {   // partner in this thread: register u ^ (j / 256)
        const int du = j >> 8;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int up = u ^ du;
          if (up > u) {
            const int i = 256 * u + tid;
            const bool asc = (i & k) == 0;
            const double a = v[u], b = v[up];
            v[u] = asc ? fmin(a, b) : fmax(a, b);
            v[up] = asc ? fmax(a, b) : fmin(a, b);
          }
        }
      } else if (j < 64) {   // partner in this wave
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = 256 * u + tid;
          const double other = __shfl_xor(v[u], j, 64);
          v[u] = bitonic_keep(v[u], other, ((i & k) == 0) == ((i & j) == 0));
        }
      } else {   // partner in another wave of the workgroup
#pragma unroll
        for (int u = 0; u < 4; ++u) s[256 * u + tid] = v[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = 256 * u + tid;
          v[u] = bitonic_keep(v[u], s[i ^ j], ((i & k) == 0) == ((i & j) == 0));
        }
        __syncthreads();
      }
    }
  // the element at rank q is held by thread q % 256 in register q / 256
  double r = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (256 * u + tid == q) r = v[u];
  if (tid == (q & 255)) s[0] = r;
  __syncthreads();
  return s[0];
}

__global__ void __launch_bounds__(256) k_update_thr(const DevReq *__restrict__ reqs, double *__restrict__ thr) {
  __shared__ double sv[kUpdMax];
  __shared__ int si[kUpdMax];
  __shared__ double s_thr;
  const DevReq rq = reqs[blockIdx.x];
  const int B = rq.B, tid = threadIdx.x;
  if (rq.stage == 0) return;
  const int q = B / 4;
  if (B <= 1024) {
    const double r = rank_value_1024(rq.logl_cur, B, q, sv);
    if (tid == 0) thr[blockIdx.x] = r;
  } else if (B <= kUpdMax) {
    int n2 = 1;
    while (n2 < B) n2 <<= 1;
    for (int i = tid; i < n2; i += 256) {
      double v = HUGE_VAL;   // padding sorts after every point (larger index on ties)
      if (i < B) {
        v = rq.logl_cur[i];
        if (isnan(v)) v = -HUGE_VAL;
      }
      sv[i] = v;
      si[i] = i;
    }
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < n2; i += 256) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const double a = sv[i], b = sv[ixj];
            const int ia = si[i], ib = si[ixj];
            const bool greater = (a > b) || (a == b && ia > ib);
            if (greater == ((i & k) == 0)) {
              sv[i] = b;
              sv[ixj] = a;
              si[i] = ib;
              si[ixj] = ia;
            }
          }
        }
        __syncthreads();
      }
    if (tid == 0) thr[blockIdx.x] = sv[q];
  } else {
    if (tid == 0) s_thr = -HUGE_VAL;
    __syncthreads();
    for (int i = tid; i < B; i += 256) {
      const double v0 = rq.logl_cur[i];
      const double v = isnan(v0) ? -HUGE_VAL : v0;
      int rank = 0;
      for (int j = 0; j < B; ++j) {
        const double u0 = rq.logl_cur[j];
        const double u = isnan(u0) ? -HUGE_VAL : u0;
        rank += (u < v) || (u == v && j < i);
      }
      if (rank == q) s_thr = v;
    }
    __syncthreads();
    if (tid == 0) thr[blockIdx.x] = s_thr;
  }
}

// one wave per point of the tick: record (stage 0) or replace an accepted point
__global__ void __launch_bounds__(256) k_accept(const DevReq *__restrict__ reqs, int n_req, int P,
                                                const double *__restrict__ theta_all,
                                                const double *__restrict__ logl_all, const double *__restrict__ thr,
                                                int n_total) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= n_total) return;   // uniform over the wave
  int lo = 0, hi = n_req - 1;   // last request with off <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].off <= p) lo = mid; else hi = mid - 1;
  }
  const DevReq rq = reqs[lo];
  const int i = p - rq.off;
  const double ln = logl_all[p];
  if (rq.stage == 0) {
    if (lane == 0) rq.logl_cur[i] = ln;
    return;
  }
  if (!(ln > thr[lo])) return;
  if (lane == 0) rq.logl_cur[i] = ln;
  const double *s = theta_all + (size_t)p * P;
  double *d = rq.theta_cur + (size_t)i * P;
  for (int c = lane; c < P; c += 64) d[c] = s[c];
}

hipError_t launch_propose(const DevReq *reqs, int n_req, int P, int n_sfh, const ProposalBox &box,
                          double *theta_all, int *point_obs, int n_total, hipStream_t s) {
  hipLaunchKernelGGL(k_propose, dim3((n_total + 3) / 4), dim3(256), 0, s, reqs, n_req, P, n_sfh, box, theta_all,
                     point_obs, n_total);
  return hipGetLastError();
}

hipError_t launch_update(const DevReq *reqs, int n_req, int P, const double *theta_all, const double *logl_all,
                         double *thr, int n_total, hipStream_t s) {
  hipLaunchKernelGGL(k_update_thr, dim3(n_req), dim3(256), 0, s, reqs, thr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_accept, dim3((n_total + 3) / 4), dim3(256), 0, s, reqs, n_req, P, theta_all, logl_all, thr,
                     n_total);
  return hipGetLastError();
}

}  // namespace sps
