// Continuous-batching request server (include/sps_server.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/sps_server.h"
#include "kernels.h"
#include "runtime.h"
#include "serve.h"

using namespace sps;

namespace {

using Clock = std::chrono::steady_clock;
double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}
size_t r256(size_t n) { return (n + 255) / 256 * 256; }

struct Request {
  uint64_t ticket = 0;
  int kind = 0, B = 0, P = 0, n_iter = 0, state = SPS_REQ_PENDING, stage = 0, slot = -1;
  uint64_t seed = 0;
  ObsHost obs;
  std::vector<double> theta, logl;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t bytes = 0, evals = 0;
  bool cancel = false;
  // device state
  DeviceBuffers mem;
  DevObs dobs{};
  double *d_theta = nullptr, *d_logl = nullptr;
};

}  // namespace

struct sps_server {
  const sps_library *lib = nullptr;
  sps_server_desc desc{};
  bool mock = false;
  int P = 0, n_sfh = 0;
  ProposalBox box{};
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  bool broken = false;   // the scheduler stopped after a device error
  std::thread thr;
  uint64_t next_ticket = 1;
  std::deque<std::shared_ptr<Request>> pending;
  std::vector<std::shared_ptr<Request>> active;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<int> free_slots;
  int64_t in_use = 0, peak = 0, active_points = 0;
  Clock::time_point t0;
  // statistics
  int64_t n_submitted = 0, n_completed = 0, n_rejected = 0, n_cancelled = 0, n_ticks = 0, n_evals = 0;
  double busy = 0, points_sum = 0, queue_sum = 0, queue_max = 0;
  std::vector<double> lat[2];
  // device resources
  Workspace ws;
  hipStream_t s_compute = nullptr, s_copy = nullptr;
  DevObs *d_obs_table = nullptr;
  DevReq *d_reqs = nullptr;
  double *d_theta_all = nullptr, *d_logl_all = nullptr;
  int *d_point_obs = nullptr;
  double *d_thr = nullptr;   // per-request acceptance thresholds of a tick
  DeviceBuffers mem;
  DeviceArena arena;         // the requests' device state, within the HBM budget
  // pipelined ticks (GPU executor): at most kInFlight enqueued; tick t uses host buffers
  // t mod kInFlight (its request descriptors, and the pinned staging its finishing
  // requests' results are copied into)
  static constexpr int kInFlight = 2;
  DevReq *h_reqs2[kInFlight] = {nullptr, nullptr};
  double *h_stage[kInFlight] = {nullptr, nullptr};
  hipEvent_t ev_tick[kInFlight] = {nullptr, nullptr};
  hipEvent_t ev_adm = nullptr;
  struct Leaving {
    std::shared_ptr<Request> r;
    size_t off;      // results at h_stage[buf] + off (theta rows, then logl)
    bool results;    // false: cancelled, released without results
  };
  struct TickRec {
    int buf = 0;
    std::vector<Leaving> leaving;
  };
  std::deque<TickRec> inflight;
  int64_t tick_no = 0;
  Clock::time_point busy_since;
  // mock buffers
  std::vector<double> m_theta_all, m_logl_all;

  void run();
  void run_mock();
  void run_gpu();
  int admit_one(std::shared_ptr<Request> &r);   // 1 admitted, 0 no room yet, -1 failed
  void release_device(Request &r);
  bool tick();
  bool enqueue_tick();
  void finish_tick(TickRec &t, bool ok);
  void admission(std::unique_lock<std::mutex> &lk);
  double mock_logl(const double *th) const;
};

// ---------------------------------------------------------------------------------
double sps_server::mock_logl(const double *th) const {
  // a smooth deterministic stand-in for the likelihood (host-only executor)
  double s = 0.0;
  for (int c = 0; c < P; ++c) {
    const double d = th[c] - 0.01 * (c % 7);
    s -= 0.5 * d * d * (1.0 + 0.1 * (c % 3));
  }
  return s;
}

int sps_server::admit_one(std::shared_ptr<Request> &r) {
  r->slot = free_slots.back();
  free_slots.pop_back();
  if (mock) return 1;
  // device state from the arena (no HIP allocation call); uploads on the copy stream, which
  // the compute stream waits for (an event) before the next tick: the host never waits
  r->mem.arena = &arena;
  r->d_theta = (double *)r->mem.alloc(r256((size_t)r->B * P * 8));
  r->d_logl = (double *)r->mem.alloc(r256((size_t)r->B * 8));
  if (!r->d_theta || !r->d_logl) return 0;
  const sps_status st = upload_obs(r->obs, r->dobs, r->mem, s_copy);
  if (st == SPS_E_NOMEM) return 0;   // the arena is fragmented: retry when blocks come back
  if (st != SPS_OK) return -1;
  if (hipMemcpyAsync(r->d_theta, r->theta.data(), (size_t)r->B * P * 8, hipMemcpyHostToDevice, s_copy) !=
      hipSuccess)
    return -1;
  if (hipMemcpyAsync(d_obs_table + r->slot, &r->dobs, sizeof(DevObs), hipMemcpyHostToDevice, s_copy) !=
      hipSuccess)
    return -1;
  return 1;
}

void sps_server::release_device(Request &r) {
  if (r.slot >= 0) free_slots.push_back(r.slot);
  r.slot = -1;
  r.mem.release();
  r.d_theta = r.d_logl = nullptr;
}

// One batched evaluation of every active request's current stage (host-only executor).
bool sps_server::tick() {
  const int n = (int)active.size();
  int total = 0;
  std::vector<DevReq> reqs(n);
  for (int q = 0; q < n; ++q) {
    Request &r = *active[q];
    reqs[q].theta_cur = mock ? r.theta.data() : r.d_theta;
    reqs[q].logl_cur = mock ? r.logl.data() : r.d_logl;
    reqs[q].seed = r.seed;
    reqs[q].off = total;
    reqs[q].B = r.B;
    reqs[q].stage = r.stage;
    reqs[q].slot = r.slot;
    total += r.B;
  }
  if (mock) {
    m_theta_all.resize((size_t)total * P);
    m_logl_all.resize(total);
    for (int q = 0; q < n; ++q) {
      const DevReq &rq = reqs[q];
      for (int i = 0; i < rq.B; ++i) {
        const double *src = rq.theta_cur + (size_t)i * P;
        double *dst = m_theta_all.data() + (size_t)(rq.off + i) * P;
        if (rq.stage == 0) std::copy(src, src + P, dst);
        else propose_point(src, dst, P, n_sfh, box, rq.seed, (uint64_t)rq.stage, (uint64_t)i);
        m_logl_all[rq.off + i] = mock_logl(dst);
      }
    }
    if (desc.mock_eval_ns > 0)
      std::this_thread::sleep_for(std::chrono::nanoseconds((int64_t)(desc.mock_eval_ns * total)));
    for (int q = 0; q < n; ++q) {   // same update rule as the device kernel
      const DevReq &rq = reqs[q];
      if (rq.stage == 0) {
        for (int i = 0; i < rq.B; ++i) rq.logl_cur[i] = m_logl_all[rq.off + i];
        continue;
      }
      const int qn = rq.B / 4;
      double thr = -HUGE_VAL;
      for (int i = 0; i < rq.B; ++i) {
        const double v = std::isnan(rq.logl_cur[i]) ? -HUGE_VAL : rq.logl_cur[i];
        int rank = 0;
        for (int j = 0; j < rq.B; ++j) {
          const double u = std::isnan(rq.logl_cur[j]) ? -HUGE_VAL : rq.logl_cur[j];
          rank += (u < v) || (u == v && j < i);
        }
        if (rank == qn) thr = v;
      }
      for (int i = 0; i < rq.B; ++i) {
        const double ln = m_logl_all[rq.off + i];
        if (ln > thr) {
          rq.logl_cur[i] = ln;
          std::copy(m_theta_all.data() + (size_t)(rq.off + i) * P, m_theta_all.data() + (size_t)(rq.off + i + 1) * P,
                    rq.theta_cur + (size_t)i * P);
        }
      }
    }
    return true;
  }
  return false;   // the GPU executor enqueues its ticks (enqueue_tick)
}

void sps_server::run() {
  if (mock) run_mock();
  else run_gpu();
}

// Admission, FIFO while the budget, the point capacity, the slots and (GPU) the arena allow.
// Called with the lock held; drops it around the uploads.
void sps_server::admission(std::unique_lock<std::mutex> &lk) {
  bool uploaded = false;
  while (!pending.empty()) {
    auto r = pending.front();
    if (r->cancel) {
      pending.pop_front();
      r->state = SPS_REQ_CANCELLED;
      r->t_done = seconds_since(t0);
      ++n_cancelled;
      done_cv.notify_all();
      continue;
    }
    if (in_use + r->bytes > desc.hbm_budget_bytes || active_points + r->B > desc.max_points || free_slots.empty())
      break;
    pending.pop_front();
    lk.unlock();
    const int ok = admit_one(r);
    lk.lock();
    if (ok == 0) {   // no contiguous room in the arena yet: back to the head of the queue
      release_device(*r);
      pending.push_front(r);
      break;
    }
    in_use += r->bytes;
    peak = std::max(peak, in_use);
    active_points += r->B;
    r->t_admit = seconds_since(t0);
    const double qd = r->t_admit - r->t_submit;
    queue_sum += qd;
    queue_max = std::max(queue_max, qd);
    if (ok < 0) {
      release_device(*r);
      in_use -= r->bytes;
      active_points -= r->B;
      r->state = SPS_REQ_FAILED;
      r->t_done = r->t_admit;
      done_cv.notify_all();
      continue;
    }
    uploaded = true;
    r->state = SPS_REQ_ACTIVE;
    active.push_back(r);
  }
  if (uploaded && !mock) {   // the next tick's kernels wait for the uploads on the GPU
    if (hipEventRecord(ev_adm, s_copy) != hipSuccess || hipStreamWaitEvent(s_compute, ev_adm, 0) != hipSuccess)
      (void)hipStreamSynchronize(s_copy);
  }
}

void sps_server::run_mock() {
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    admission(lk);
    if (active.empty()) {
      cv.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    // ---- one batched evaluation of all active requests
    const auto tb = Clock::now();
    const int points = (int)active_points;
    lk.unlock();
    const bool ok = tick();
    lk.lock();
    busy += seconds_since(tb);
    ++n_ticks;
    points_sum += points;
    n_evals += points;
    // ---- bookkeeping: finished, failed and cancelled requests leave the batch
    std::vector<std::shared_ptr<Request>> keep;
    for (auto &r : active) {
      r->evals += r->B;
      r->stage += 1;
      const bool finished = r->stage > r->n_iter;
      if (!ok || r->cancel || finished) {
        release_device(*r);
        in_use -= r->bytes;
        active_points -= r->B;
        r->t_done = seconds_since(t0);
        if (!ok) r->state = SPS_REQ_FAILED;
        else if (r->cancel) {
          r->state = SPS_REQ_CANCELLED;
          ++n_cancelled;
        } else {
          r->state = SPS_REQ_DONE;
          ++n_completed;
          lat[r->kind].push_back(r->t_done - r->t_submit);
        }
      } else {
        keep.push_back(r);
      }
    }
    active.swap(keep);
    done_cv.notify_all();
  }
  for (auto &r : active) {
    release_device(*r);
    r->state = SPS_REQ_CANCELLED;
    ++n_cancelled;
  }
  active.clear();
  for (auto &r : pending) {
    r->state = SPS_REQ_CANCELLED;
    ++n_cancelled;
  }
  pending.clear();
  done_cv.notify_all();
}

// Enqueues one tick over every active request on the compute stream (no host wait): the
// request descriptors from pinned buffer t mod kInFlight, proposals, the batched forward +
// logL, the acceptance update; requests at their last stage leave the batch, their results
// copied after the update into that tick's pinned staging.  Called without the lock (the
// active list changes on this thread only); the bookkeeping after the launches takes it.
bool sps_server::enqueue_tick() {
  const int buf = (int)(tick_no % kInFlight);
  const int n = (int)active.size();
  DevReq *hr = h_reqs2[buf];
  int total = 0;
  for (int q = 0; q < n; ++q) {
    Request &r = *active[q];
    hr[q].theta_cur = r.d_theta;
    hr[q].logl_cur = r.d_logl;
    hr[q].seed = r.seed;
    hr[q].off = total;
    hr[q].B = r.B;
    hr[q].stage = r.stage;
    hr[q].slot = r.slot;
    total += r.B;
  }
  (void)hipGetLastError();   // drop a stale code from an unrelated earlier HIP call of this thread
  hipError_t e = hipMemcpyAsync(d_reqs, hr, sizeof(DevReq) * n, hipMemcpyHostToDevice, s_compute);
  if (e == hipSuccess) e = launch_propose(d_reqs, n, P, n_sfh, box, d_theta_all, d_point_obs, total, s_compute);
  if (e != hipSuccess) return false;
  if (launch_forward(lib, ws, d_obs_table, d_point_obs, d_theta_all, total, desc.precision, d_logl_all, nullptr, 1,
                     false, 1, nullptr, nullptr, s_compute) != SPS_OK)
    return false;
  e = launch_update(d_reqs, n, P, d_theta_all, d_logl_all, d_thr, total, s_compute);
  std::lock_guard<std::mutex> g(mu);
  TickRec t;
  t.buf = buf;
  size_t off = 0;
  std::vector<std::shared_ptr<Request>> keep;
  for (auto &r : active) {
    r->evals += r->B;
    r->stage += 1;
    if (r->stage > r->n_iter) {
      double *st = h_stage[buf] + off;
      if (e == hipSuccess)
        e = hipMemcpyAsync(st, r->d_theta, (size_t)r->B * P * 8, hipMemcpyDeviceToHost, s_compute);
      if (e == hipSuccess)
        e = hipMemcpyAsync(st + (size_t)r->B * P, r->d_logl, (size_t)r->B * 8, hipMemcpyDeviceToHost, s_compute);
      t.leaving.push_back({r, off, true});
      off += (size_t)r->B * (P + 1);
      active_points -= r->B;   // no later tick holds its points (its memory stays until this one ends)
    } else {
      keep.push_back(r);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(ev_tick[buf], s_compute);
  if (inflight.empty()) busy_since = Clock::now();
  active.swap(keep);
  inflight.push_back(std::move(t));
  ++n_ticks;
  ++tick_no;
  points_sum += total;
  n_evals += total;
  return e == hipSuccess;
}

// The oldest tick has completed (ok) or the stream failed: its leaving requests finish and
// their device memory and slots return (their points left the batch when they did).
// Called with the lock held.
void sps_server::finish_tick(TickRec &t, bool ok) {
  for (auto &lv : t.leaving) {
    Request &r = *lv.r;
    if (ok && lv.results) {
      const double *st = h_stage[t.buf] + lv.off;
      std::copy(st, st + (size_t)r.B * P, r.theta.data());
      std::copy(st + (size_t)r.B * P, st + (size_t)r.B * (P + 1), r.logl.data());
    }
    release_device(r);
    in_use -= r.bytes;
    r.t_done = seconds_since(t0);
    if (!ok) {
      r.state = SPS_REQ_FAILED;
    } else if (!lv.results) {
      r.state = SPS_REQ_CANCELLED;
      ++n_cancelled;
    } else {
      r.state = SPS_REQ_DONE;
      ++n_completed;
      lat[r.kind].push_back(r.t_done - r.t_submit);
    }
  }
}

void sps_server::run_gpu() {
  (void)hipSetDevice(lib->device);
  std::unique_lock<std::mutex> lk(mu);
  bool failed = false;
  while (!stop && !failed) {
    admission(lk);
    // cancelled requests leave the batch; a tick in flight may still read their state, so
    // they are released with the newest one
    std::vector<std::shared_ptr<Request>> keep;
    for (auto &r : active) {
      if (!r->cancel) {
        keep.push_back(r);
        continue;
      }
      active_points -= r->B;
      if (!inflight.empty()) {
        inflight.back().leaving.push_back({r, 0, false});
      } else {
        TickRec t0r;
        t0r.leaving.push_back({r, 0, false});
        finish_tick(t0r, true);
      }
    }
    active.swap(keep);
    if (!active.empty() && (int)inflight.size() < kInFlight) {
      lk.unlock();
      const bool ok = enqueue_tick();
      lk.lock();
      if (!ok) failed = true;
      continue;
    }
    if (!inflight.empty()) {
      const hipEvent_t ev = ev_tick[inflight.front().buf];
      lk.unlock();
      const bool ok = hipEventSynchronize(ev) == hipSuccess;
      lk.lock();
      TickRec t = std::move(inflight.front());
      inflight.pop_front();
      if (inflight.empty()) busy += seconds_since(busy_since);
      finish_tick(t, ok);
      if (!ok) failed = true;
      done_cv.notify_all();
      continue;
    }
    cv.wait_for(lk, std::chrono::milliseconds(2));
  }
  broken = failed;
  // shutdown (or a failed stream): drain the GPU; ticks in flight finish their requests
  // (failed if the stream failed); everything else is cancelled
  lk.unlock();
  const bool drained = hipStreamSynchronize(s_compute) == hipSuccess && !failed;
  lk.lock();
  while (!inflight.empty()) {
    finish_tick(inflight.front(), drained);
    inflight.pop_front();
    if (inflight.empty()) busy += seconds_since(busy_since);
  }
  for (auto &r : active) {
    release_device(*r);
    in_use -= r->bytes;
    active_points -= r->B;
    r->state = failed ? SPS_REQ_FAILED : SPS_REQ_CANCELLED;
    if (!failed) ++n_cancelled;
    r->t_done = seconds_since(t0);
  }
  active.clear();
  for (auto &r : pending) {
    r->state = SPS_REQ_CANCELLED;
    ++n_cancelled;
  }
  pending.clear();
  done_cv.notify_all();
}

// =====================================================================================
extern "C" sps_status sps_server_create(const sps_library *L, const sps_server_desc *d, sps_server **out) {
  if (!L || !d || !out) return fail(SPS_E_INVAL, "sps_server_create: NULL argument");
  *out = nullptr;
  if (d->max_points < 1 || d->max_active < 1 || d->max_active > 4096 || d->hbm_budget_bytes <= 0)
    return fail(SPS_E_INVAL, "server needs max_points >= 1, 1 <= max_active <= 4096, budget > 0");
  const bool mock = d->device < 0;
  if (!mock && L->device < 0) return fail(SPS_E_STATE, "host-only library: the GPU server needs a device library");
  if (!mock && !precision_built(L, d->precision)) return fail(SPS_E_INVAL, "precision %d not built", d->precision);
  if (L->dev.vdisp) return fail(SPS_E_INVAL, "the server's mixed launches do not take a free sigma_gal");
  auto *S = new sps_server();
  S->lib = L;
  S->desc = *d;
  S->mock = mock;
  S->P = L->dev.P;
  S->n_sfh = L->n_sfh;
  ProposalBox &b = S->box;
  b.logmass_lo = 6.0;
  b.logmass_hi = 12.5;
  b.z_lo = 0.05;
  b.z_hi = 20.0;
  b.tau_hi = 4.0;
  b.delta_lo = -1.0;
  b.delta_hi = 0.4;
  b.logz_lo = L->logz_lo;
  b.logz_hi = L->logz_hi;
  b.afe_lo = L->afe_lo;
  b.afe_hi = L->afe_hi;
  b.step = 0.03;
  for (int q = d->max_active - 1; q >= 0; --q) S->free_slots.push_back(q);
  S->t0 = Clock::now();
  if (!mock) {
    if (hipSetDevice(L->device) != hipSuccess) {
      delete S;
      return fail(SPS_E_HIP, "hipSetDevice failed");
    }
    sps_status st = S->ws.create(L, d->max_points, 1, 0, true);
    bool ok = st == SPS_OK;
    ok = ok && hipStreamCreateWithFlags(&S->s_compute, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&S->s_copy, hipStreamNonBlocking) == hipSuccess;
    S->d_obs_table = (DevObs *)S->mem.alloc(sizeof(DevObs) * d->max_active);
    S->d_reqs = (DevReq *)S->mem.alloc(sizeof(DevReq) * d->max_active);
    S->d_theta_all = (double *)S->mem.alloc((size_t)d->max_points * S->P * 8);
    S->d_logl_all = (double *)S->mem.alloc((size_t)d->max_points * 8);
    S->d_point_obs = (int *)S->mem.alloc((size_t)d->max_points * 4);
    S->d_thr = (double *)S->mem.alloc(sizeof(double) * d->max_active);
    ok = ok && S->d_obs_table && S->d_reqs && S->d_theta_all && S->d_logl_all && S->d_point_obs && S->d_thr;
    for (int k = 0; k < sps_server::kInFlight; ++k) {
      ok = ok && hipHostMalloc((void **)&S->h_reqs2[k], sizeof(DevReq) * d->max_active, hipHostMallocDefault) ==
                     hipSuccess;
      ok = ok && hipHostMalloc((void **)&S->h_stage[k], (size_t)d->max_points * (S->P + 1) * 8,
                               hipHostMallocDefault) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&S->ev_tick[k], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipEventCreateWithFlags(&S->ev_adm, hipEventDisableTiming) == hipSuccess;
    ok = ok && S->arena.init((size_t)d->hbm_budget_bytes + (64u << 10));   // + slack for block rounding
    if (!ok) {
      sps_server_destroy(S);
      return st != SPS_OK ? st : fail(SPS_E_NOMEM, "server allocation failed");
    }
  }
  S->thr = std::thread([S]() { S->run(); });
  *out = S;
  return SPS_OK;
}

extern "C" sps_status sps_submit(sps_server *S, const sps_request *q, uint64_t *ticket) {
  if (!S || !q || !ticket) return fail(SPS_E_INVAL, "sps_submit: NULL argument");
  auto reject = [&](sps_status st) {
    std::lock_guard<std::mutex> g(S->mu);
    ++S->n_rejected;
    return st;
  };
  if (q->B < 1 || q->B > S->desc.max_points)
    return reject(fail(SPS_E_SHAPE, "B=%d outside [1, max_points=%d]", q->B, S->desc.max_points));
  if (!q->theta0) return reject(fail(SPS_E_INVAL, "theta0 is NULL"));
  if (q->n_iter < 0) return reject(fail(SPS_E_INVAL, "n_iter must be >= 0"));
  auto r = std::make_shared<Request>();
  sps_status st = build_obs_operators(S->lib, &q->obs, r->obs, nullptr);
  if (st == SPS_OK && (q->obs.kind == SPS_OBS_LINES || r->obs.calib_mode != SPS_CALIB_NONE ||
                       r->obs.lm_mode != SPS_LINEMARG_NONE))
    st = fail(SPS_E_INVAL, "the server fits photometry and spectra without a calibration polynomial or line "
              "marginalisation");
  if (st == SPS_OK) st = set_obs_data(r->obs, q->obs.data, q->obs.sigma, q->obs.mask);
  if (st != SPS_OK) {
    std::lock_guard<std::mutex> g(S->mu);
    ++S->n_rejected;
    return st;
  }
  r->kind = q->obs.kind == SPS_OBS_SPEC ? 1 : 0;
  r->B = q->B;
  r->P = S->P;
  r->n_iter = q->n_iter;
  r->seed = q->seed;
  r->theta.assign(q->theta0, q->theta0 + (size_t)q->B * S->P);
  r->logl.assign(q->B, 0.0);
  for (double v : r->theta)
    if (!std::isfinite(v)) {
      std::lock_guard<std::mutex> g(S->mu);
      ++S->n_rejected;
      return fail(SPS_E_INVAL, "theta0 must be finite");
    }
  r->bytes = obs_device_bytes(r->obs) + (int64_t)r256((size_t)q->B * S->P * 8) + (int64_t)r256((size_t)q->B * 8);
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return fail(SPS_E_STATE, "server is shutting down");
  if (S->broken) return fail(SPS_E_HIP, "the server stopped after a device error");
  if (r->bytes > S->desc.hbm_budget_bytes) {
    ++S->n_rejected;
    return fail(SPS_E_BUDGET, "request needs %lld bytes, budget is %lld", (long long)r->bytes,
                (long long)S->desc.hbm_budget_bytes);
  }
  r->ticket = S->next_ticket++;
  r->t_submit = seconds_since(S->t0);
  S->pending.push_back(r);
  S->all[r->ticket] = r;
  ++S->n_submitted;
  *ticket = r->ticket;
  S->cv.notify_all();
  return SPS_OK;
}

static void fill_result(const Request &r, sps_result *out) {
  out->state = r.state;
  out->B = r.B;
  out->P = r.P;
  out->kind = r.kind;
  const bool done = r.state == SPS_REQ_DONE;
  out->theta = done ? r.theta.data() : nullptr;
  out->logl = done ? r.logl.data() : nullptr;
  out->queue_s = r.t_admit > 0 ? r.t_admit - r.t_submit : 0.0;
  out->latency_s = r.t_done > 0 ? r.t_done - r.t_submit : 0.0;
  out->evals = r.evals;
}

static bool finished(const Request &r) {
  return r.state == SPS_REQ_DONE || r.state == SPS_REQ_CANCELLED || r.state == SPS_REQ_FAILED;
}

extern "C" sps_status sps_poll(sps_server *S, uint64_t ticket, sps_result *out) {
  if (!S || !out) return fail(SPS_E_INVAL, "sps_poll: NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SPS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  fill_result(*it->second, out);
  return finished(*it->second) ? SPS_OK : SPS_PENDING;
}

extern "C" sps_status sps_wait(sps_server *S, uint64_t ticket, int64_t timeout_us, sps_result *out) {
  if (!S || !out) return fail(SPS_E_INVAL, "sps_wait: NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SPS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  auto r = it->second;
  auto pred = [&]() { return finished(*r); };
  if (timeout_us < 0) S->done_cv.wait(lk, pred);
  else if (!S->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) {
    fill_result(*r, out);
    return fail(SPS_E_TIMEOUT, "request %llu not finished", (unsigned long long)ticket);
  }
  fill_result(*r, out);
  return SPS_OK;
}

extern "C" sps_status sps_cancel(sps_server *S, uint64_t ticket) {
  if (!S) return fail(SPS_E_INVAL, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SPS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  auto r = it->second;
  if (r->state == SPS_REQ_PENDING) {   // not admitted yet: leaves the queue at once
    auto pit = std::find(S->pending.begin(), S->pending.end(), r);
    if (pit != S->pending.end()) {
      S->pending.erase(pit);
      r->state = SPS_REQ_CANCELLED;
      r->t_done = seconds_since(S->t0);
      ++S->n_cancelled;
      S->done_cv.notify_all();
      return SPS_OK;
    }
  }
  if (!finished(*r)) r->cancel = true;
  S->cv.notify_all();
  return SPS_OK;
}

extern "C" sps_status sps_release(sps_server *S, uint64_t ticket) {
  if (!S) return fail(SPS_E_INVAL, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(SPS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (!finished(*it->second)) return fail(SPS_E_STATE, "request %llu is still running", (unsigned long long)ticket);
  S->all.erase(it);
  return SPS_OK;
}

static double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(p * v.size());
  k = std::min(std::max(k, (size_t)1), v.size());
  return v[k - 1];
}

extern "C" sps_status sps_server_stats(sps_server *S, sps_stats *o) {
  if (!S || !o) return fail(SPS_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  memset(o, 0, sizeof *o);
  o->submitted = S->n_submitted;
  o->completed = S->n_completed;
  o->rejected = S->n_rejected;
  o->cancelled = S->n_cancelled;
  o->active = (int64_t)S->active.size();
  o->pending = (int64_t)S->pending.size();
  o->ticks = S->n_ticks;
  o->evals = S->n_evals;
  o->busy_s = S->busy;
  o->evals_per_s = S->busy > 0 ? S->n_evals / S->busy : 0.0;
  o->mean_points_per_tick = S->n_ticks ? S->points_sum / S->n_ticks : 0.0;
  for (int k = 0; k < 2; ++k) {
    o->p50_latency_s[k] = percentile(S->lat[k], 0.50);
    o->p99_latency_s[k] = percentile(S->lat[k], 0.99);
    o->completed_by_kind[k] = (int64_t)S->lat[k].size();
  }
  const int64_t admitted = S->n_completed + (int64_t)S->active.size();
  o->mean_queue_s = admitted > 0 ? S->queue_sum / (double)std::max<int64_t>(1, admitted) : 0.0;
  o->max_queue_s = S->queue_max;
  o->hbm_in_use = S->in_use;
  o->hbm_peak = S->peak;
  o->hbm_budget = S->desc.hbm_budget_bytes;
  return SPS_OK;
}

extern "C" void sps_server_destroy(sps_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->thr.joinable()) S->thr.join();
  if (!S->mock) {
    (void)hipSetDevice(S->lib->device);
    if (S->s_compute) (void)hipStreamDestroy(S->s_compute);
    if (S->s_copy) (void)hipStreamDestroy(S->s_copy);
    for (int k = 0; k < sps_server::kInFlight; ++k) {
      if (S->h_reqs2[k]) (void)hipHostFree(S->h_reqs2[k]);
      if (S->h_stage[k]) (void)hipHostFree(S->h_stage[k]);
      if (S->ev_tick[k]) (void)hipEventDestroy(S->ev_tick[k]);
    }
    if (S->ev_adm) (void)hipEventDestroy(S->ev_adm);
  }
  delete S;
}
