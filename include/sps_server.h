/*
 * sps_server.h - continuous-batching request server over the batched SPS forward model.
 *
 * A fit request brings its own observation (photometry or a prism spectrum) and a
 * set of B_r live points.  The server keeps the library and every admitted
 * request's sampler state resident in HBM, admits requests while an HBM budget and
 * a per-launch point capacity allow, and on every tick evaluates the current
 * proposals of ALL active requests in one batched launch of the forward model and
 * likelihood (Sec. 4.3: nested sampling replaces a batch of live points per
 * iteration; Sec. 7: several fits sharing one device, which the paper leaves
 * unmeasured).  Requests that arrive while others run join at the next tick.
 *
 * Stand-in sampler (the nested slice sampler itself is outside this library):
 * iteration 0 evaluates theta0; each later iteration draws one proposal per live
 * point from a counter-based generator keyed by (request seed, iteration, point,
 * parameter) and accepts proposals whose logL exceeds the current worst-quartile
 * logL of the request.  Results are therefore independent of which other requests
 * share a launch.
 *
 * All calls are thread-safe.  Host arrays passed to sps_submit are copied.
 * Result arrays returned by sps_poll/sps_wait stay valid until sps_release.
 */
#ifndef SPS_SERVER_H
#define SPS_SERVER_H

#include "sps.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t hbm_budget_bytes;  /* device bytes available to admitted requests' state */
  int32_t max_points;        /* live points evaluated per launch (workspace size) */
  int32_t max_active;        /* concurrently admitted requests (observation slots) */
  int32_t precision;         /* sps_precision of the contraction */
  int32_t device;            /* HIP device; -1 = host-only mock executor (tests) */
  double mock_eval_ns;       /* mock executor: simulated ns per evaluated point */
} sps_server_desc;

typedef struct {
  sps_obs_desc obs;          /* observation of this fit (max_batch is ignored) */
  int32_t B;                 /* live points, 1 <= B <= max_points */
  const double *theta0;      /* host [B, P] initial live points */
  int32_t n_iter;            /* stand-in sampler iterations after the first evaluation */
  uint64_t seed;             /* request seed of the proposal generator */
} sps_request;

enum { SPS_REQ_PENDING = 0, SPS_REQ_ACTIVE = 1, SPS_REQ_DONE = 2, SPS_REQ_CANCELLED = 3, SPS_REQ_FAILED = 4 };

typedef struct {
  int32_t state;             /* SPS_REQ_* */
  int32_t B, P, kind;
  const double *theta;       /* host [B, P] final live points (valid until sps_release) */
  const double *logl;        /* host [B] their logL */
  double queue_s;            /* submit -> admission */
  double latency_s;          /* submit -> result available */
  int64_t evals;             /* forward-model evaluations spent on this request */
} sps_result;

typedef struct {
  int64_t submitted, completed, rejected, cancelled, active, pending;
  int64_t ticks, evals;
  double busy_s;             /* wall time with at least one batched launch in flight */
  double evals_per_s;        /* evals / busy_s */
  double mean_points_per_tick;
  double p50_latency_s[2], p99_latency_s[2];   /* [0] photometry, [1] spectra */
  int64_t completed_by_kind[2];
  double mean_queue_s, max_queue_s;
  int64_t hbm_in_use, hbm_peak, hbm_budget;
} sps_stats;

/* Errors: SPS_E_INVAL (also for a library with a free sigma_gal: each launch mixes
 * observations, while the Fourier stage's transform belongs to one), SPS_E_NOMEM,
 * SPS_E_HIP. */
sps_status sps_server_create(const sps_library *lib, const sps_server_desc *desc, sps_server **out);
/* Copies the request and queues it; returns at once.  SPS_E_BUDGET when its
 * state can never fit the budget, SPS_E_SHAPE for B outside [1, max_points],
 * SPS_E_INVAL for a bad observation, SPS_E_STATE after shutdown. */
sps_status sps_submit(sps_server *srv, const sps_request *req, uint64_t *ticket);
/* SPS_OK with out->state DONE (or CANCELLED/FAILED), or SPS_PENDING. */
sps_status sps_poll(sps_server *srv, uint64_t ticket, sps_result *out);
/* Blocks until done or timeout_us elapses (SPS_E_TIMEOUT); timeout_us < 0 waits forever. */
sps_status sps_wait(sps_server *srv, uint64_t ticket, int64_t timeout_us, sps_result *out);
/* Cancels a pending or active request (its memory is returned at the next tick). */
sps_status sps_cancel(sps_server *srv, uint64_t ticket);
/* Frees a finished request's result buffers; the ticket becomes unknown. */
sps_status sps_release(sps_server *srv, uint64_t ticket);
sps_status sps_server_stats(sps_server *srv, sps_stats *out);
/* Stops the scheduler; requests not finished are cancelled. */
void sps_server_destroy(sps_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* SPS_SERVER_H */
