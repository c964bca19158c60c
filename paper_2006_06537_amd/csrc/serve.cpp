// Serving loop: GP-regression jobs (one Gibbs chain each, Section 4.1's sweep) submitted
// at any time, run with continuous batching.
//
//   * Planning: planner threads make each job's host plans (every grid point's tree and
//     windows) as soon as it is submitted, and with them its exact device footprint.
//   * Admission: in arrival order, a planned job takes a free slot when a block of its
//     footprint can be carved from the server's device arena (allocated once at
//     creation, sized by the memory budget).  The job's chain is built inside that block,
//     so the worker never calls the runtime allocator: no hipMalloc / hipFree, whose
//     device-wide synchronisation would stall every running job.
//   * Progress: each slot owns a stream (and the chain's proposal stream), and each job
//     advances on its own: when a slot's event reports its last sweep done, the worker
//     applies the sweep, then enqueues the next one, or retires the job, returns its
//     block and admits the next job at once.  Short jobs finish and leave while long ones
//     are still running; the sweeps of all running jobs overlap on the device.
//   * Each job's chain is the chain gibbs_step would run alone: chains share no buffers,
//     every reduction is deterministic and the random numbers are addressed by
//     (seed, iteration, stream_id).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fg_chain.h"
#include "fg_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int PLANNERS = 4;            // host threads making plans
constexpr size_t HOST_PER_SLOT = 8192;  // pinned state words of one chain (with slack)

struct Job {
  uint64_t id = 0;
  fg_job job{};
  std::vector<double> x, y;  // host copies of the request
  double t_submit = 0.0, t_admit = 0.0;
  fg_chain_cfg cfg{};
  fg::ChainPlans plans;
  int plan_state = 0;        // 0 waiting, 1 taken by a planner, 2 planned, -1 failed
  fg_status plan_status = FG_OK;
  std::string plan_err;
  size_t block_bytes = 0;    // footprint plus the rounding of every allocation
};

struct Slot {
  hipStream_t s = nullptr;
  fg::ChainStreams cs;
  hipEvent_t done = nullptr;
  std::unique_ptr<Job> job;
  fg_chain chain = nullptr;
  void* block = nullptr;     // the job's block of the server arena
  fg::Arena arena;           // view over that block
  int phase = 0;             // 0 free, 1 setting up, 2 sweeping
};

fg_chain_cfg chain_cfg(const fg_job& j) {
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

}  // namespace

struct fg_server_s {
  fg_serve_cfg cfg{};
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;        // worker: submissions, plans; callers: results
  std::condition_variable plan_cv;   // planners: submissions
  std::deque<std::unique_ptr<Job>> queue;  // submitted, not admitted (arrival order)
  std::deque<fg_result> done;
  std::vector<Slot> slots;           // worker thread only (after creation)
  fg::Arena dev_arena, host_arena;
  uint64_t next_id = 1;
  uint64_t used = 0, peak_used = 0;  // bytes of admitted jobs' blocks (under mu)
  int64_t sweeps = 0;                // under mu
  int64_t outstanding = 0;           // submitted and not yet finished (under mu)
  bool stop = false;
  std::thread worker;
  std::vector<std::thread> planners;
  std::string fatal;
};

static double now_s(fg_server s) {
  return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

// planner: plans the earliest submitted job nobody has taken yet
static void plan_loop(fg_server s) {
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) return;
        for (auto& q : s->queue)
          if (q->plan_state == 0) {
            j = q.get();
            break;
          }
        if (j) break;
        s->plan_cv.wait(lk);
      }
      j->plan_state = 1;
    }
    std::string err;
    const fg_status st = fg::chain_plan(j->cfg, j->x.data(), int(j->job.n), j->plans, err);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      j->plan_status = st;
      j->plan_err = err;
      j->block_bytes = j->plans.bytes + 256 * fg::chain_alloc_count(j->cfg) + 4096;
      j->plan_state = st == FG_OK ? 2 : -1;
    }
    s->cv.notify_all();
  }
}

static void post_result(fg_server s, const fg_result& r) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.push_back(r);
    s->outstanding -= 1;
  }
  s->cv.notify_all();
}

static void set_fatal(fg_server s, const std::string& m) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal.empty()) s->fatal = m;
    s->stop = true;
  }
  s->cv.notify_all();
  s->plan_cv.notify_all();
}

// the job in a slot is done: its result, then its chain and block go back
static void retire(fg_server s, Slot& sl) {
  Job& j = *sl.job;
  fg_result r{};
  r.id = j.id;
  r.t_submit = j.t_submit;
  r.t_admit = j.t_admit;
  r.bytes = j.block_bytes;
  r.status = gibbs_chain_state(sl.chain, &r.snap, nullptr, nullptr, nullptr, sl.s);
  if (r.status == FG_OK) r.status = r.snap.status;
  if (j.job.f_out &&
      (hipMemcpyAsync(j.job.f_out, fg::chain_f(sl.chain), sizeof(double) * (size_t)j.job.n,
                      hipMemcpyDeviceToHost, sl.s) != hipSuccess ||
       hipStreamSynchronize(sl.s) != hipSuccess) &&
      r.status == FG_OK)
    r.status = FG_EDEVICE;
  fg::chain_destroy_idle(sl.chain);  // its memory goes back to the slot's view
  sl.chain = nullptr;
  sl.arena.release();
  s->dev_arena.free(sl.block);
  sl.block = nullptr;
  sl.phase = 0;
  r.t_done = now_s(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->used -= j.block_bytes;
  }
  sl.job.reset();
  post_result(s, r);
}

static void fail_job(fg_server s, const Job& j, fg_status st) {
  fg_result r{};
  r.id = j.id;
  r.status = st;
  r.t_submit = j.t_submit;
  r.t_admit = r.t_done = now_s(s);
  post_result(s, r);
}

// admits planned jobs from the head of the queue while slots and memory allow; returns
// whether anything was admitted or failed
static bool admit(fg_server s) {
  bool any = false;
  for (;;) {
    Slot* free_slot = nullptr;
    for (auto& sl : s->slots)
      if (sl.phase == 0) {
        free_slot = &sl;
        break;
      }
    std::unique_ptr<Job> j;
    void* block = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queue.empty() || s->queue.front()->plan_state < 2) {
        if (!s->queue.empty() && s->queue.front()->plan_state == -1) {
          j = std::move(s->queue.front());
          s->queue.pop_front();
        } else {
          return any;
        }
      } else {
        if (!free_slot) return any;
        Job& h = *s->queue.front();
        if (h.block_bytes > s->dev_arena.capacity()) {
          j = std::move(s->queue.front());  // can never fit
          s->queue.pop_front();
          j->plan_state = -1;
          j->plan_status = FG_ENOMEM;
        } else {
          block = s->dev_arena.alloc(h.block_bytes);
          if (!block) return any;  // waits for running jobs to free memory (head of line)
          j = std::move(s->queue.front());
          s->queue.pop_front();
          s->used += j->block_bytes;
          s->peak_used = std::max(s->peak_used, s->used);
        }
      }
    }
    any = true;
    if (j->plan_state == -1) {
      fail_job(s, *j, j->plan_status);
      continue;
    }
    Slot& sl = *free_slot;
    sl.block = block;
    sl.arena.init_view(block, j->block_bytes);
    j->t_admit = now_s(s);
    fg_chain c = nullptr;
    std::string err;
    fg_status st;
    {
      fg::ArenaScope scope(&sl.arena, &s->host_arena);
      st = fg::chain_create_planned(j->cfg, j->plans, j->x.data(), j->y.data(), true,
                                    int(j->job.n), sl.s, &sl.cs, false, &c, err);
    }
    if (st != FG_OK) {
      sl.arena.release();
      s->dev_arena.free(block);
      sl.block = nullptr;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->used -= j->block_bytes;
      }
      fail_job(s, *j, st);
      continue;
    }
    sl.chain = c;
    sl.job = std::move(j);
    sl.phase = 1;
    if (hipEventRecord(sl.done, sl.s) != hipSuccess) {
      set_fatal(s, "event record failed");
      return any;
    }
  }
}

// worker: poll the slots, advance each job that finished its last step, admit
static void serve_loop(fg_server s) {
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) break;
    }
    bool progressed = false;
    int busy = 0;
    for (auto& sl : s->slots) {
      if (sl.phase == 0) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) {
        ++busy;
        continue;
      }
      if (q != hipSuccess) {
        set_fatal(s, std::string("serving: ") + hipGetErrorString(q));
        break;
      }
      progressed = true;
      if (sl.phase == 1) {
        sl.phase = 2;  // the chain's set-up is done
      } else {
        bool again;
        {
          // a fallback to an FP64 factor of M~ allocates: from the job's own block
          fg::ArenaScope scope(&sl.arena, &s->host_arena);
          again = fg::chain_end_sweep(sl.chain, sl.s);
        }
        if (again) {  // PCG budget too small: run it again
          if (fg::chain_begin_sweep(sl.chain, sl.s, true) != hipSuccess) {
            set_fatal(s, "serving: a sweep could not be enqueued");
            break;
          }
          (void)hipEventRecord(sl.done, sl.s);
          ++busy;
          continue;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->sweeps += 1;
      }
      if (fg::chain_iteration(sl.chain) >= sl.job->job.iters) {
        retire(s, sl);
        continue;
      }
      if (fg::chain_begin_sweep(sl.chain, sl.s, false) != hipSuccess ||
          hipEventRecord(sl.done, sl.s) != hipSuccess) {
        set_fatal(s, "serving: a sweep could not be enqueued");
        break;
      }
      ++busy;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) set_fatal(s, std::string("serving launch: ") + hipGetErrorString(e));
    if (admit(s)) {
      progressed = true;
      busy = 1;
    }
    if (progressed) continue;
    if (busy > 0) {
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    } else {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::milliseconds(20), [s] {
        return s->stop || (!s->queue.empty() && s->queue.front()->plan_state != 0 &&
                           s->queue.front()->plan_state != 1);
      });
    }
  }
  // stopping: let queued work finish, then release every running job
  for (auto& sl : s->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.cs.aux) (void)hipStreamSynchronize(sl.cs.aux);
    if (sl.chain) fg::chain_destroy_idle(sl.chain);
    sl.chain = nullptr;
    sl.arena.release();
    if (sl.block) s->dev_arena.free(sl.block);
    sl.block = nullptr;
    sl.job.reset();
    sl.phase = 0;
  }
}

static void destroy_slots(fg_server s) {
  for (auto& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    for (auto e : sl.cs.ev)
      if (e) (void)hipEventDestroy(e);
    if (sl.cs.aux) (void)hipStreamDestroy(sl.cs.aux);
    if (sl.s) (void)hipStreamDestroy(sl.s);
  }
  s->slots.clear();
}

extern "C" {

fg_status serve_create(const fg_serve_cfg* cfg, fg_server* out) {
  if (!out) return FG_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->max_active < 1 || cfg->max_active > 256 || cfg->mem_budget == 0) {
    fg::set_error("bad serving configuration");
    return FG_EINVAL;
  }
  fg_server s = new fg_server_s();
  s->cfg = *cfg;
  s->t0 = Clock::now();
  std::string err;
  fg_status st = s->dev_arena.init(cfg->mem_budget, false, err);
  if (st == FG_OK) st = s->host_arena.init(HOST_PER_SLOT * cfg->max_active, true, err);
  if (st != FG_OK) {
    delete s;
    fg::set_error(err);
    return st;
  }
  // the slots' streams and events: the chain's own stream and its proposal stream (the
  // served sweep is the two-stream form), the fork/join events and the completion event
  {
    std::vector<Slot> slots(cfg->max_active);  // (slots hold mutexes: built in place)
    s->slots.swap(slots);
  }
  for (auto& sl : s->slots) {
    bool ok = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&sl.cs.aux, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
    for (int e = 0; e < 2 && ok; ++e)
      ok = hipEventCreateWithFlags(&sl.cs.ev[e], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      destroy_slots(s);
      delete s;
      fg::set_error("stream or event creation failed");
      return FG_EDEVICE;
    }
  }
  s->worker = std::thread(serve_loop, s);
  for (int p = 0; p < PLANNERS; ++p) s->planners.emplace_back(plan_loop, s);
  *out = s;
  return FG_OK;
}

fg_status serve_submit(fg_server s, const fg_job* job, uint64_t* id) {
  if (!s || !job || !job->x || !job->y) {
    fg::set_error("NULL argument");
    return FG_EINVAL;
  }
  if (job->n < 1 || job->n >= (int64_t(1) << 31) || job->iters < 1 || !(job->ell0 > 0) ||
      !(job->tau0 > 0) || !(job->sigf2_0 > 0) ||
      (job->precision != FG_FP64 && job->precision != FG_MIXED)) {
    fg::set_error("bad job");
    return FG_EINVAL;
  }
  for (int64_t i = 1; i < job->n; ++i)
    if (!(job->x[i - 1] <= job->x[i])) {
      fg::set_error("x must be sorted ascending");
      return FG_EINVAL;
    }
  auto j = std::make_unique<Job>();
  j->job = *job;
  j->x.assign(job->x, job->x + job->n);
  j->y.assign(job->y, job->y + job->n);
  j->job.x = nullptr;  // the copies are used from here on
  j->job.y = nullptr;
  j->cfg = chain_cfg(*job);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      fg::set_error(s->fatal.empty() ? "server stopped" : s->fatal);
      return FG_EDEVICE;
    }
    j->id = s->next_id++;
    j->t_submit = now_s(s);
    if (id) *id = j->id;
    s->queue.push_back(std::move(j));
    s->outstanding += 1;
  }
  s->plan_cv.notify_all();
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
  out->pending = (int64_t)s->queue.size();
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
  }
  s->cv.notify_all();
  s->plan_cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& t : s->planners)
    if (t.joinable()) t.join();
  destroy_slots(s);
  s->queue.clear();
  delete s;  // the arenas release their memory
}

}  // extern "C"
