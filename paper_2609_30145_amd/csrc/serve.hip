// Device side of the request server: stand-in sampler proposals and updates for every
// active request, laid out in one batch (request r owns points [off_r, off_r + B_r)).
#include "serve.h"

namespace sps {

// ---------------------------------------------------------------- proposals
__global__ void __launch_bounds__(256) k_propose(const DevReq *__restrict__ reqs, int n_req, int P, int n_sfh,
                                                 ProposalBox box, double *__restrict__ theta_all,
                                                 int *__restrict__ point_obs, int n_total) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n_total) return;
  int lo = 0, hi = n_req - 1;   // last request with off <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].off <= p) lo = mid; else hi = mid - 1;
  }
  const DevReq rq = reqs[lo];
  const int i = p - rq.off;
  const double *src = rq.theta_cur + (size_t)i * P;
  double *dst = theta_all + (size_t)p * P;
  point_obs[p] = rq.slot;
  if (rq.stage == 0) {
    for (int c = 0; c < P; ++c) dst[c] = src[c];
    return;
  }
  propose_point(src, dst, P, n_sfh, box, rq.seed, (uint64_t)rq.stage, (uint64_t)i);
}

// ---------------------------------------------------------------- update
// stage 0: record logL(theta0).  stage >= 1: threshold = the logL at rank floor(B/4)
// (ascending, ties by index) of the current live points; proposals above it replace
// their point.
__global__ void __launch_bounds__(256) k_update(const DevReq *__restrict__ reqs, int P,
                                                const double *__restrict__ theta_all,
                                                const double *__restrict__ logl_all) {
  __shared__ double thr;
  const DevReq rq = reqs[blockIdx.x];
  const int B = rq.B, tid = threadIdx.x;
  if (rq.stage == 0) {
    for (int i = tid; i < B; i += 256) rq.logl_cur[i] = logl_all[rq.off + i];
    return;
  }
  if (tid == 0) thr = -HUGE_VAL;
  __syncthreads();
  const int q = B / 4;
  for (int i = tid; i < B; i += 256) {
    const double v0 = rq.logl_cur[i];
    const double v = isnan(v0) ? -HUGE_VAL : v0;
    int rank = 0;
    for (int j = 0; j < B; ++j) {
      const double u0 = rq.logl_cur[j];
      const double u = isnan(u0) ? -HUGE_VAL : u0;
      rank += (u < v) || (u == v && j < i);
    }
    if (rank == q) thr = v;
  }
  __syncthreads();
  const double t = thr;
  __syncthreads();
  for (int i = tid; i < B; i += 256) {
    const double ln = logl_all[rq.off + i];
    if (ln > t) {
      rq.logl_cur[i] = ln;
      const double *s = theta_all + (size_t)(rq.off + i) * P;
      double *d = rq.theta_cur + (size_t)i * P;
      for (int c = 0; c < P; ++c) d[c] = s[c];
    }
  }
}

hipError_t launch_propose(const DevReq *reqs, int n_req, int P, int n_sfh, const ProposalBox &box,
                          double *theta_all, int *point_obs, int n_total, hipStream_t s) {
  hipLaunchKernelGGL(k_propose, dim3((n_total + 255) / 256), dim3(256), 0, s, reqs, n_req, P, n_sfh, box, theta_all,
                     point_obs, n_total);
  return hipGetLastError();
}

hipError_t launch_update(const DevReq *reqs, int n_req, int P, const double *theta_all, const double *logl_all,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(n_req), dim3(256), 0, s, reqs, P, theta_all, logl_all);
  return hipGetLastError();
}

}  // namespace sps
