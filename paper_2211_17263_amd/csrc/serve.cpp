// Continuous-batching server for gradient-estimate requests from many
// concurrent optimisation jobs.
//
// Jobs register a scene description and a reference image; their BVHs are built
// once on the host and kept there, so making a job resident is an upload.  A
// server thread forms batch epochs from the FIFO of pending requests: a request
// joins an epoch if its job is resident or can be admitted within the server's
// HBM budget (idle jobs are evicted least recently used first); otherwise it
// waits for a later epoch.  Up to two epochs are in flight at once on separate
// streams, so requests that arrive while an epoch runs are admitted as soon as
// a slot and memory free up and their work overlaps the running epoch on the
// device.  Each result is the same as the request alone (the batch path is
// bit-identical to the single-request path).  A request may carry a deadline:
// once it has passed, the request completes with PRDPT_E_TIMEOUT whether it is
// still queued or already running (its result is then dropped when its epoch
// ends); the other requests of its epoch are not affected.
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "ctx_internal.h"

using namespace prdpt;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
  HostScene host;
  std::vector<float> ref_host;
  prdpt_scene* scene = nullptr;
  float* d_ref = nullptr;
  size_t footprint = 0;  // scene + reference bytes when resident
  uint64_t last_used = 0;
  int in_flight = 0;
};

struct Pending {
  int64_t ticket = 0;
  int job = 0;
  float theta[PRDPT_BATCH_MAX_PARAMS];
  float sigma[PRDPT_BATCH_MAX_PARAMS];
  int N = 0, est = 0;
  uint64_t seed = 0;
  double t_submit = 0.0;
  double deadline = 0.0;  // steady-clock seconds; 0: none
};

struct Slot {
  BatchState b;
  bool busy = false;
  hipEvent_t done = nullptr;
  double t_start = 0.0;
  std::vector<Pending> items;
  std::vector<char> expired;  // items already completed with PRDPT_E_TIMEOUT
  std::vector<prdpt_request> reqs;
  std::vector<std::vector<double>> grads;
  std::vector<double> loss;
  std::vector<int> ok;
};

}  // namespace

struct prdpt_server {
  prdpt_ctx* ctx = nullptr;
  prdpt_server_config cfg{};
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::unique_ptr<Job>> jobs;
  std::deque<Pending> pending;
  std::deque<prdpt_completion> done;
  std::vector<int64_t> cancel_requests;
  Slot slots[2];
  bool stop = false;
  int64_t next_ticket = 1;
  size_t resident = 0;
  uint64_t clock = 0;
  prdpt_server_stats stats{};
  int error = PRDPT_OK;
};

namespace {

void complete(prdpt_server* sv, const Pending& p, int status, double t_start, const double* grad,
              int d, double loss) {
  prdpt_completion c;
  std::memset(&c, 0, sizeof(c));
  c.ticket = p.ticket;
  c.job = p.job;
  c.status = status;
  c.loss = loss;
  if (grad)
    for (int j = 0; j < d; ++j) c.grad[j] = grad[j];
  c.t_submit = p.t_submit;
  c.t_start = t_start;
  c.t_done = now_s();
  sv->done.push_back(c);
  if (status == PRDPT_OK) {
    sv->stats.completed++;
    sv->stats.paths += (double)p.N * sv->jobs[p.job]->host.hdr.W * sv->jobs[p.job]->host.hdr.H *
                       sv->jobs[p.job]->host.hdr.spp;
  } else {
    sv->stats.failed++;
  }
}

void evict(prdpt_server* sv, Job& j) {
  prdpt_scene_destroy(j.scene);
  hipFree(j.d_ref);
  j.scene = nullptr;
  j.d_ref = nullptr;
  sv->resident -= j.footprint;
  sv->stats.evictions++;
}

// admit(): the job cannot be made resident before a running epoch frees memory
constexpr int kWaitForMemory = 1;

// Make job `ji` resident within the budget; jobs in `protect` are not evicted.
// Returns PRDPT_OK, kWaitForMemory, or a (terminal) error status.
int admit(prdpt_server* sv, int ji, const std::vector<char>& protect) {
  Job& j = *sv->jobs[ji];
  if (j.scene) return PRDPT_OK;
  const size_t ref_bytes = j.ref_host.size() * sizeof(float);
  const size_t need = j.host.footprint + ref_bytes;
  if (sv->cfg.hbm_budget && need > sv->cfg.hbm_budget) return PRDPT_E_ADMISSION;
  while (sv->cfg.hbm_budget && sv->resident + need > sv->cfg.hbm_budget) {
    int victim = -1;
    for (size_t k = 0; k < sv->jobs.size(); ++k) {
      Job& c = *sv->jobs[k];
      if (!c.scene || c.in_flight || protect[k]) continue;
      if (victim < 0 || c.last_used < sv->jobs[victim]->last_used) victim = (int)k;
    }
    if (victim < 0) return kWaitForMemory;  // wait for running epochs to finish
    evict(sv, *sv->jobs[victim]);
  }
  if (int rc = upload_scene(sv->ctx, j.host, &j.scene)) return rc;
  if (dev_malloc((void**)&j.d_ref, ref_bytes) != hipSuccess ||
      hipMemcpy(j.d_ref, j.ref_host.data(), ref_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    prdpt_scene_destroy(j.scene);
    j.scene = nullptr;
    if (j.d_ref) hipFree(j.d_ref);
    j.d_ref = nullptr;
    return fail(PRDPT_E_NOMEM, "reference upload failed");
  }
  j.footprint = need;
  sv->resident += need;
  sv->stats.admissions++;
  return PRDPT_OK;
}

// Retire a finished slot: results to completions (server lock held).
void retire(prdpt_server* sv, Slot& s) {
  batch_collect(s.b, s.reqs.data(), s.ok);
  for (size_t i = 0; i < s.items.size(); ++i) {
    const Pending& p = s.items[i];
    Job& j = *sv->jobs[p.job];
    j.in_flight--;
    if (s.expired[i]) continue;  // completed with PRDPT_E_TIMEOUT while it ran
    const int d = j.host.hdr.n_param;
    complete(sv, p, s.reqs[i].status, s.t_start, s.grads[i].data(), d, s.loss[i]);
  }
  s.items.clear();
  s.busy = false;
  sv->stats.epochs++;
}

// Form and enqueue one epoch into slot s (server lock held).  Returns true if
// an epoch was launched.
bool launch_epoch(prdpt_server* sv, Slot& s) {
  std::vector<char> protect(sv->jobs.size(), 0);
  std::deque<Pending> keep;
  s.items.clear();
  const int max_batch = sv->cfg.max_batch > 0 ? sv->cfg.max_batch : 64;
  while (!sv->pending.empty()) {
    Pending p = sv->pending.front();
    sv->pending.pop_front();
    bool cancelled = false;
    for (int64_t t : sv->cancel_requests)
      if (t == p.ticket) cancelled = true;
    if (cancelled) {
      complete(sv, p, PRDPT_E_CANCELLED, 0.0, nullptr, 0, 0.0);
      continue;
    }
    if ((int)s.items.size() >= max_batch) {
      keep.push_back(p);
      continue;
    }
    const char was_protected = protect[p.job];
    protect[p.job] = 1;
    const int rc = admit(sv, p.job, protect);
    if (rc == kWaitForMemory) {
      protect[p.job] = was_protected;
      keep.push_back(p);  // admitted in a later epoch, when memory frees up
      continue;
    }
    if (rc != PRDPT_OK) {
      // the job can never fit the budget, or its upload failed (the context's
      // own budget, device memory, HIP): the request fails, the others go on
      protect[p.job] = was_protected;
      complete(sv, p, rc, 0.0, nullptr, 0, 0.0);
      continue;
    }
    s.items.push_back(p);
  }
  sv->cancel_requests.clear();
  for (auto it = keep.rbegin(); it != keep.rend(); ++it) sv->pending.push_front(*it);
  if (s.items.empty()) return false;
  const size_t n = s.items.size();
  s.expired.assign(n, 0);
  s.reqs.assign(n, prdpt_request{});
  s.grads.assign(n, std::vector<double>(PRDPT_BATCH_MAX_PARAMS, 0.0));
  s.loss.assign(n, 0.0);
  for (size_t i = 0; i < n; ++i) {
    Pending& p = s.items[i];
    Job& j = *sv->jobs[p.job];
    j.in_flight++;
    j.last_used = ++sv->clock;
    prdpt_request& r = s.reqs[i];
    r.scene = j.scene;
    r.ref = j.d_ref;
    r.theta = p.theta;
    r.sigma = p.sigma;
    r.N = p.N;
    r.est = p.est;
    r.seed = p.seed;
    r.grad_out = s.grads[i].data();
    r.loss_out = &s.loss[i];
    r.losses_out = nullptr;
  }
  s.b.blocks_per_cu = sv->ctx->batch.blocks_per_cu;
  s.b.tiles_per_item = sv->ctx->batch.tiles_per_item;
  s.b.use_graph = 1;
  s.t_start = now_s();
  int rc = ensure_batch(sv->ctx, s.b, 1, 1, 1, 1);
  if (rc == PRDPT_OK && !s.done) rc = hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess
                                          ? PRDPT_OK : PRDPT_E_HIP;
  if (rc == PRDPT_OK) rc = batch_enqueue(sv->ctx, s.b, s.reqs.data(), (int)n, s.ok, nullptr, nullptr);
  if (rc == PRDPT_OK) rc = hipEventRecord(s.done, s.b.stream) == hipSuccess ? PRDPT_OK : PRDPT_E_HIP;
  if (rc != PRDPT_OK) {
    for (size_t i = 0; i < n; ++i) {
      sv->jobs[s.items[i].job]->in_flight--;
      complete(sv, s.items[i], rc, s.t_start, nullptr, 0, 0.0);
    }
    s.items.clear();
    sv->error = rc;
    return false;
  }
  s.busy = true;
  return true;
}

// Requests whose deadline has passed complete with PRDPT_E_TIMEOUT: queued
// ones leave the queue, running ones are marked so that their epoch drops the
// result (server lock held).  Returns true if any request expired.
bool expire(prdpt_server* sv) {
  const double t = now_s();
  bool any = false;
  for (auto it = sv->pending.begin(); it != sv->pending.end();) {
    if (it->deadline > 0.0 && t > it->deadline) {
      complete(sv, *it, PRDPT_E_TIMEOUT, 0.0, nullptr, 0, 0.0);
      it = sv->pending.erase(it);
      any = true;
    } else {
      ++it;
    }
  }
  for (Slot& s : sv->slots) {
    if (!s.busy) continue;
    for (size_t i = 0; i < s.items.size(); ++i) {
      if (!s.expired[i] && s.items[i].deadline > 0.0 && t > s.items[i].deadline) {
        complete(sv, s.items[i], PRDPT_E_TIMEOUT, s.t_start, nullptr, 0, 0.0);
        s.expired[i] = 1;
        any = true;
      }
    }
  }
  return any;
}

void server_loop(prdpt_server* sv) {
  hipSetDevice(sv->ctx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    if (expire(sv)) sv->cv_done.notify_all();
    bool any_busy = false;
    for (Slot& s : sv->slots) {
      if (!s.busy) continue;
      if (hipEventQuery(s.done) == hipSuccess) {
        retire(sv, s);
        sv->cv_done.notify_all();
      } else {
        any_busy = true;
      }
    }
    bool launched = false;
    for (int si = 0; si < sv->cfg.max_inflight; ++si) {
      Slot& s = sv->slots[si];
      if (!s.busy && !sv->pending.empty()) {
        launched |= launch_epoch(sv, s);
        if (!sv->done.empty()) sv->cv_done.notify_all();
      }
    }
    any_busy = any_busy || launched;
    for (Slot& s : sv->slots) any_busy = any_busy || s.busy;
    if (sv->stop && !any_busy && sv->pending.empty()) break;
    if (!any_busy && !sv->pending.empty()) {
      // nothing runs and nothing queued could start (no memory can free up):
      // on stop the queue is cancelled, otherwise wait for a change instead of
      // retrying at once
      if (sv->stop) {
        for (const Pending& p : sv->pending) complete(sv, p, PRDPT_E_CANCELLED, 0.0, nullptr, 0, 0.0);
        sv->pending.clear();
        sv->cv_done.notify_all();
        continue;
      }
      sv->cv_work.wait_for(lk, std::chrono::milliseconds(1));
    } else if (any_busy || !sv->pending.empty()) {
      // poll the running epochs and the deadlines; new submissions wake us
      sv->cv_work.wait_for(lk, std::chrono::microseconds(200));
    } else {
      sv->cv_work.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
    }
  }
}

}  // namespace

extern "C" {

int prdpt_server_start(prdpt_ctx* ctx, const prdpt_server_config* cfg, prdpt_server** out) {
  if (!ctx || !out) return fail(PRDPT_E_ARG, "null argument");
  prdpt_server* sv = new prdpt_server();
  sv->ctx = ctx;
  if (cfg) sv->cfg = *cfg;
  if (sv->cfg.max_batch <= 0) sv->cfg.max_batch = 64;
  if (sv->cfg.max_inflight <= 0 || sv->cfg.max_inflight > 2) sv->cfg.max_inflight = 2;
  sv->th = std::thread(server_loop, sv);
  *out = sv;
  return PRDPT_OK;
}

int prdpt_server_add_job(prdpt_server* sv, const prdpt_scene_desc* desc, const float* ref_host,
                         int* job_id) {
  if (!sv || !desc || !ref_host || !job_id) return fail(PRDPT_E_ARG, "null argument");
  auto j = std::make_unique<Job>();
  if (int rc = build_host_scene(desc, j->host)) return rc;
  if (j->host.hdr.n_param > PRDPT_BATCH_MAX_PARAMS)
    return fail(PRDPT_E_SCENE, "served jobs take at most PRDPT_BATCH_MAX_PARAMS parameters");
  const size_t n = (size_t)desc->width * desc->height * 3;
  j->ref_host.assign(ref_host, ref_host + n);
  std::lock_guard<std::mutex> g(sv->mu);
  sv->jobs.push_back(std::move(j));
  *job_id = (int)sv->jobs.size() - 1;
  return PRDPT_OK;
}

int prdpt_server_submit(prdpt_server* sv, int job_id, const float* theta, const float* sigma, int N,
                        uint64_t seed, int est, int64_t* ticket) {
  return prdpt_server_submit_deadline(sv, job_id, theta, sigma, N, seed, est, 0.0, ticket);
}

int prdpt_server_submit_deadline(prdpt_server* sv, int job_id, const float* theta,
                                 const float* sigma, int N, uint64_t seed, int est,
                                 double timeout_s, int64_t* ticket) {
  if (!sv || !theta || !sigma || !ticket) return fail(PRDPT_E_ARG, "null argument");
  if (!(timeout_s >= 0.0) || !std::isfinite(timeout_s))
    return fail(PRDPT_E_ARG, "timeout must be finite and >= 0");
  Pending p;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (job_id < 0 || job_id >= (int)sv->jobs.size()) return fail(PRDPT_E_ARG, "no such job");
    if (sv->stop) return fail(PRDPT_E_ARG, "server is stopping");
    const int d = sv->jobs[job_id]->host.hdr.n_param;
    if (N < 2 || (N & 1)) return fail(PRDPT_E_ARG, "N must be even and >= 2");
    if (est < PRDPT_EST_GAUSS || est > PRDPT_EST_IS_PERDIM) return fail(PRDPT_E_ARG, "bad estimator");
    for (int j = 0; j < d; ++j)
      if (!(sigma[j] > 0.0f) || !std::isfinite(sigma[j]) || !std::isfinite(theta[j]))
        return fail(PRDPT_E_ARG, "theta must be finite and sigma positive");
    std::memset(&p, 0, sizeof(p));
    std::memcpy(p.theta, theta, sizeof(float) * d);
    std::memcpy(p.sigma, sigma, sizeof(float) * d);
    p.job = job_id;
    p.N = N;
    p.est = est;
    p.seed = seed;
    p.ticket = sv->next_ticket++;
    p.t_submit = now_s();
    p.deadline = timeout_s > 0.0 ? p.t_submit + timeout_s : 0.0;
    sv->pending.push_back(p);
    sv->stats.submitted++;
    *ticket = p.ticket;
  }
  sv->cv_work.notify_one();
  return PRDPT_OK;
}

int prdpt_server_cancel(prdpt_server* sv, int64_t ticket) {
  if (!sv) return fail(PRDPT_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(sv->mu);
  sv->cancel_requests.push_back(ticket);
  return PRDPT_OK;
}

int prdpt_server_poll(prdpt_server* sv, prdpt_completion* out, int max, int timeout_ms, int* n_out) {
  if (!sv || !out || !n_out || max < 0) return fail(PRDPT_E_ARG, "null argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->done.empty() && timeout_ms > 0)
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !sv->done.empty(); });
  int n = 0;
  while (n < max && !sv->done.empty()) {
    out[n++] = sv->done.front();
    sv->done.pop_front();
  }
  *n_out = n;
  return PRDPT_OK;
}

int prdpt_server_get_stats(prdpt_server* sv, prdpt_server_stats* st) {
  if (!sv || !st) return fail(PRDPT_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(sv->mu);
  *st = sv->stats;
  st->pending = (int64_t)sv->pending.size();
  st->resident_bytes = (int64_t)sv->resident;
  return PRDPT_OK;
}

int prdpt_server_stop(prdpt_server* sv) {
  if (!sv) return fail(PRDPT_E_ARG, "null argument");
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->th.joinable()) sv->th.join();
  hipSetDevice(sv->ctx->device);
  for (Slot& s : sv->slots) {
    if (s.b.stream) hipStreamSynchronize(s.b.stream);
    batch_release(s.b);
    if (s.done) hipEventDestroy(s.done);
  }
  for (auto& j : sv->jobs)
    if (j->scene) evict(sv, *j);
  const int err = sv->error;
  delete sv;
  return err == PRDPT_OK ? PRDPT_OK : fail(err, "an epoch failed while the server ran");
}

}  // extern "C"
