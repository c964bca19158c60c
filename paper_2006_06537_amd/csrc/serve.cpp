// Serving loop: GP-regression jobs (one Gibbs chain each) submitted at any time are
// admitted in arrival order while their device footprint fits the memory budget and a
// slot is free, then advanced together one sweep at a time (gibbs_step_batch over the
// active set).  A job leaves the set after its last sweep, its memory is released, and
// the jobs waiting behind it are admitted before the next sweep: continuous batching at
// sweep granularity.  Each job's chain is the chain gibbs_step would run alone (chains
// share no buffers and every reduction is deterministic).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fg_internal.h"

namespace fg {
size_t chain_device_bytes(fg_chain c);
int64_t chain_iteration(fg_chain c);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
  uint64_t id;
  fg_job job;
  std::vector<double> x, y;  // host copies of the request
  double t_submit;
  uint64_t est;              // footprint estimate (bytes)
};

struct Active {
  uint64_t id;
  fg_job job;
  fg_chain chain;
  uint64_t bytes;
  double t_submit, t_admit;
};

}  // namespace

struct fg_server_s {
  fg_serve_cfg cfg{};
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending> pending;
  std::deque<fg_result> done;
  std::vector<Active> active;  // worker thread only
  uint64_t next_id = 1;
  uint64_t used = 0;           // bytes held by active jobs (worker thread only)
  uint64_t peak_used = 0;
  int64_t sweeps = 0;
  int64_t outstanding = 0;     // submitted and not yet finished
  bool stop = false;
  std::thread worker;
  hipStream_t stream = nullptr;
  std::string fatal;
};

static double now_s(fg_server s) {
  return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

static fg_chain_cfg chain_cfg(const fg_job& j) {
  fg_chain_cfg c{};
  c.kind = j.kind;
  c.ell0 = j.ell0;
  c.nugget = j.nugget;
  c.leaf = j.leaf;
  c.tol = j.tol;
  c.tau0 = j.tau0;
  c.sigf2_0 = j.sigf2_0;
  c.a1 = c.b1 = c.a2 = c.b2 = 1.0;
  c.grid_size = 100;
  c.grid_center = 50;
  c.seed = j.seed;
  c.stream_id = j.stream_id;
  c.precision = j.precision;
  return c;
}

// worker: admit -> one batched sweep -> retire, until stopped
static void serve_loop(fg_server s) {
  std::vector<fg_chain> chains;
  for (;;) {
    // admission (FIFO, head of line): footprint within budget and a free slot
    for (;;) {
      Pending p;
      {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop) return;
        if (s->pending.empty() || (int)s->active.size() >= s->cfg.max_active) break;
        const uint64_t est = s->pending.front().est;
        if (!s->active.empty() && s->used + est > s->cfg.mem_budget) break;
        p = std::move(s->pending.front());
        s->pending.pop_front();
      }
      const fg_chain_cfg cc = chain_cfg(p.job);
      const size_t nb = sizeof(double) * (size_t)p.job.n;
      double *xd = nullptr, *yd = nullptr;
      fg_chain c = nullptr;
      fg_status st = FG_ENOMEM;
      if (hipMalloc(reinterpret_cast<void**>(&xd), nb) == hipSuccess &&
          hipMalloc(reinterpret_cast<void**>(&yd), nb) == hipSuccess &&
          hipMemcpyAsync(xd, p.x.data(), nb, hipMemcpyHostToDevice, s->stream) == hipSuccess &&
          hipMemcpyAsync(yd, p.y.data(), nb, hipMemcpyHostToDevice, s->stream) == hipSuccess)
        st = gibbs_chain_create(&cc, xd, yd, p.job.n, s->stream, &c);
      (void)hipStreamSynchronize(s->stream);
      if (xd) (void)hipFree(xd);
      if (yd) (void)hipFree(yd);
      if (st != FG_OK) {  // the job fails alone; the server goes on
        fg_result r{};
        r.id = p.id;
        r.status = st;
        r.t_submit = p.t_submit;
        r.t_admit = r.t_done = now_s(s);
        std::lock_guard<std::mutex> lk(s->mu);
        s->done.push_back(r);
        s->outstanding -= 1;
        s->cv.notify_all();
        continue;
      }
      Active a{p.id, p.job, c, fg::chain_device_bytes(c), p.t_submit, now_s(s)};
      s->used += a.bytes;
      s->peak_used = std::max(s->peak_used, s->used);
      s->active.push_back(a);
    }
    if (s->active.empty()) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::milliseconds(20),
                     [s] { return s->stop || !s->pending.empty(); });
      if (s->stop) return;
      continue;
    }
    // one sweep of every active job
    chains.clear();
    for (auto& a : s->active) chains.push_back(a.chain);
    const fg_status st = gibbs_step_batch(chains.data(), (int)chains.size(), 1, s->cfg.nstreams,
                                          s->cfg.use_graphs, s->stream);
    s->sweeps += 1;
    if (st != FG_OK) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->fatal = fg_last_error();
      s->stop = true;
      s->cv.notify_all();
      return;
    }
    // retire finished jobs
    for (size_t i = 0; i < s->active.size();) {
      Active& a = s->active[i];
      if (fg::chain_iteration(a.chain) < a.job.iters) { ++i; continue; }
      fg_result r{};
      r.id = a.id;
      r.t_submit = a.t_submit;
      r.t_admit = a.t_admit;
      r.bytes = a.bytes;
      double* fd = nullptr;
      if (a.job.f_out)
        (void)hipMalloc(reinterpret_cast<void**>(&fd), sizeof(double) * (size_t)a.job.n);
      r.status = gibbs_chain_state(a.chain, &r.snap, fd, nullptr, nullptr, s->stream);
      if (r.status == FG_OK) r.status = r.snap.status;
      if (fd) {
        (void)hipMemcpy(a.job.f_out, fd, sizeof(double) * (size_t)a.job.n, hipMemcpyDeviceToHost);
        (void)hipFree(fd);
      }
      gibbs_chain_destroy(a.chain);
      s->used -= a.bytes;
      r.t_done = now_s(s);
      s->active.erase(s->active.begin() + i);
      std::lock_guard<std::mutex> lk(s->mu);
      s->done.push_back(r);
      s->outstanding -= 1;
      s->cv.notify_all();
    }
  }
}

extern "C" {

fg_status serve_create(const fg_serve_cfg* cfg, fg_server* out) {
  if (!out) return FG_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->max_active < 1 || cfg->nstreams < 1 || cfg->nstreams > 4 || cfg->mem_budget == 0) {
    fg::set_error("bad serving configuration");
    return FG_EINVAL;
  }
  fg_server s = new fg_server_s();
  s->cfg = *cfg;
  s->t0 = Clock::now();
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    fg::set_error("stream creation failed");
    return FG_EDEVICE;
  }
  s->worker = std::thread(serve_loop, s);
  *out = s;
  return FG_OK;
}

fg_status serve_submit(fg_server s, const fg_job* job, uint64_t* id) {
  if (!s || !job || !job->x || !job->y) {
    fg::set_error("NULL argument");
    return FG_EINVAL;
  }
  if (job->n < 1 || job->n >= (int64_t(1) << 31) || job->iters < 1 || !(job->ell0 > 0) ||
      !(job->tau0 > 0) || !(job->sigf2_0 > 0)) {
    fg::set_error("bad job");
    return FG_EINVAL;
  }
  for (int64_t i = 1; i < job->n; ++i)
    if (!(job->x[i - 1] <= job->x[i])) {
      fg::set_error("x must be sorted ascending");
      return FG_EINVAL;
    }
  Pending p;
  p.job = *job;
  p.x.assign(job->x, job->x + job->n);
  p.y.assign(job->y, job->y + job->n);
  const fg_chain_cfg cc = chain_cfg(*job);
  const fg_status est_st = fg_footprint_bytes(&cc, p.x.data(), job->n, &p.est);
  if (est_st != FG_OK) return est_st;  // the plan itself is invalid (message set)
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    fg::set_error(s->fatal.empty() ? "server stopped" : s->fatal);
    return FG_EDEVICE;
  }
  p.id = s->next_id++;
  p.t_submit = now_s(s);
  if (id) *id = p.id;
  s->pending.push_back(std::move(p));
  s->outstanding += 1;
  s->cv.notify_all();
  return FG_OK;
}

fg_status serve_poll(fg_server s, fg_result* out, int32_t max, int32_t* got) {
  if (!s || !got || max < 0 || (max > 0 && !out)) return FG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *got = k;
  if (s->stop && !s->fatal.empty()) {
    fg::set_error(s->fatal);
    return FG_EDEVICE;
  }
  return FG_OK;
}

fg_status serve_drain(fg_server s, double timeout_s) {
  if (!s) return FG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                 [s] { return s->outstanding == 0 || s->stop; });
  if (s->stop && !s->fatal.empty()) {
    fg::set_error(s->fatal);
    return FG_EDEVICE;
  }
  if (!ok) {
    fg::set_error("serve_drain timed out");
    return FG_ENOTCONV;
  }
  return FG_OK;
}

fg_status serve_stats(fg_server s, fg_serve_stats* out) {
  if (!s || !out) return FG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->pending = (int64_t)s->pending.size();
  out->outstanding = s->outstanding;
  out->sweeps = s->sweeps;
  out->peak_bytes = s->peak_used;
  return FG_OK;
}

void serve_destroy(fg_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto& a : s->active) gibbs_chain_destroy(a.chain);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
