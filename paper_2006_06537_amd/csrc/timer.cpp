// Live per-kernel timing: HIP events recorded around every launch of one selected
// kernel on the stream it is launched on, plus a device snapshot of the per-level
// ranks so that the algorithmic bytes of each launch can be computed after the fact
// without a host round trip.  The ranks change only when their matrix is built, so one
// snapshot serves every timed launch until the next build of that matrix.  Several
// kernels may be timed at once (a mask of kernel ids); the state is guarded by one
// mutex, so builds and launches from other host threads are safe while a timer runs.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "fg_internal.h"
#include "fg_timer.h"

namespace fg {

namespace {
struct Rec {
  int kid, level, n, L, nleaf, B, ntask, ring_off;
  double sum_leaf_tri;  // sum over leaves of m (m + 1) / 2
  double fixed_bytes;   // > 0: the launch's bytes, known at launch
  bool closed;          // its stop event has been recorded
};
struct TimerState {
  bool on = false;
  unsigned mask = 0;            // bit kid: kernel kid is timed
  std::vector<hipEvent_t> ev;   // start/stop pairs
  std::vector<Rec> recs;
  int* ring = nullptr;          // device: kmax snapshots
  int ring_cap = 0, ring_used = 0;
  std::unordered_map<const int*, int> snap;  // rank buffer -> its current snapshot
};
TimerState g_t;
std::mutex g_mu;
constexpr int RING_CAP = 1 << 16;
constexpr int MAX_REC = 8192;
constexpr int NKID = KID_PREDICT + 1;
struct Result { double ms = 0, bytes = 0; int64_t launches = 0; };
Result g_res[NKID];             // per kernel, from the last fg_timer_stop
bool wants_locked(int kid) {
  return g_t.on && ((g_t.mask >> kid) & 1u) && (int)g_t.recs.size() < MAX_REC;
}
}  // namespace

__global__ void k_snapshot(const int* __restrict__ src, int count, int* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = src[i];
}

bool timer_active() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_t.on;
}

bool timer_wants(int kid) {
  std::lock_guard<std::mutex> lk(g_mu);
  return wants_locked(kid);
}

void timer_before(int kid, hipStream_t s, int level, const HostPlan& P, const int* kmax_dev,
                  int ntask) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!wants_locked(kid)) return;
  Rec r{};
  r.kid = kid; r.level = level; r.n = P.n; r.L = P.L; r.nleaf = P.nleaf; r.B = P.B;
  r.ntask = ntask; r.ring_off = -1;
  double tri = 0;
  for (int b = 0; b < P.nleaf; ++b) {
    const double m = P.leaf_lo[b + 1] - P.leaf_lo[b];
    tri += m * (m + 1) / 2;
  }
  r.sum_leaf_tri = tri;
  if (P.L > 0 && kmax_dev) {  // ranks, if the bytes use them
    const auto it = g_t.snap.find(kmax_dev);
    if (it != g_t.snap.end()) {
      r.ring_off = it->second;
    } else if (g_t.ring_used + P.L <= g_t.ring_cap) {
      r.ring_off = g_t.ring_used;
      g_t.ring_used += P.L;
      k_snapshot<<<1, 64, 0, s>>>(kmax_dev, P.L, g_t.ring + r.ring_off);
      g_t.snap[kmax_dev] = r.ring_off;
    }
  }
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  hipEventRecord(a, s);
  g_t.ev.push_back(a);
  g_t.ev.push_back(b);
  g_t.recs.push_back(r);
}

void timer_before_bytes(int kid, hipStream_t s, double bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!wants_locked(kid)) return;
  Rec r{};
  r.kid = kid;
  r.ring_off = -1;
  r.fixed_bytes = bytes;
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  hipEventRecord(a, s);
  g_t.ev.push_back(a);
  g_t.ev.push_back(b);
  g_t.recs.push_back(r);
}

void timer_forget(const int* kmax_dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_t.snap.erase(kmax_dev);
}

// closes the record opened by the matching timer_before on the same thread: the last
// record of this kernel whose stop event is not yet recorded
void timer_after(int kid, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_t.on || !((g_t.mask >> kid) & 1u) || g_t.ev.empty()) return;
  if (g_t.ev.size() != 2 * g_t.recs.size()) return;
  for (size_t i = g_t.recs.size(); i-- > 0;) {
    Rec& r = g_t.recs[i];
    if (r.kid == kid && !r.closed) {
      hipEventRecord(g_t.ev[2 * i + 1], s);
      r.closed = true;
      return;
    }
  }
}

// algorithmic bytes of one launch (see the kernel notes in each source file)
static double launch_bytes(const Rec& r, const std::vector<int>& km) {
  if (r.fixed_bytes > 0.0) return r.fixed_bytes;
  const double n = r.n;
  double K = 0;
  for (int l = 0; l < r.L; ++l) K += km[l];
  switch (r.kid) {
    case KID_LEAF:  // x in; L (lower triangle) and its 16 x 16 diagonal-block inverses out
      return 8.0 * (n + r.sum_leaf_tri + 8.5 * n);
    case KID_WHITEN:  // L, the diagonal-block inverses and every active panel row in, rows out
      return 8.0 * (2.0 * n * K + r.sum_leaf_tri + 8.5 * n);
    case KID_REDUCE: {  // every right column of the level read once + partial sums
      double W = 0;
      for (int l = 0; l <= r.level; ++l) W += km[l];
      return 8.0 * (n * W + (double)r.ntask * km[r.level] * W);
    }
    case KID_UPDATE: {  // right-child rows: V~ read, coarser columns read and written
      double Wc = 0;
      for (int l = 0; l < r.level; ++l) Wc += km[l];
      return 8.0 * (0.5 * n * (km[r.level] + 2.0 * Wc));
    }
    default:
      return 0.0;
  }
}

}  // namespace fg

extern "C" {

static fg_status timer_start_mask(unsigned mask) {
  using namespace fg;
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto e : g_t.ev) hipEventDestroy(e);
  g_t.ev.clear();
  g_t.recs.clear();
  if (!g_t.ring && hipMalloc(reinterpret_cast<void**>(&g_t.ring), sizeof(int) * RING_CAP) != hipSuccess)
    return FG_ENOMEM;
  g_t.ring_cap = RING_CAP;
  g_t.ring_used = 0;
  g_t.snap.clear();
  g_t.mask = mask;
  g_t.on = true;
  return FG_OK;
}

fg_status fg_timer_start(int32_t kernel_id) {
  using namespace fg;
  if (kernel_id < KID_LEAF || kernel_id > KID_PREDICT) return FG_EINVAL;
  return timer_start_mask(1u << kernel_id);
}

fg_status fg_timer_start_mask(uint32_t mask) {
  using namespace fg;
  const uint32_t valid = ((1u << NKID) - 1u) & ~1u;
  if (mask == 0 || (mask & ~valid)) return FG_EINVAL;
  return timer_start_mask(mask);
}

fg_status fg_timer_result(int32_t kernel_id, double* total_ms, int64_t* launches, double* bytes) {
  using namespace fg;
  if (kernel_id < KID_LEAF || kernel_id > KID_PREDICT) return FG_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const Result& r = g_res[kernel_id];
  if (total_ms) *total_ms = r.ms;
  if (launches) *launches = r.launches;
  if (bytes) *bytes = r.bytes;
  return FG_OK;
}

fg_status fg_timer_stop(double* total_ms, int64_t* launches, double* bytes) {
  using namespace fg;
  std::lock_guard<std::mutex> lk(g_mu);
  g_t.on = false;
  for (auto& r : g_res) r = Result{};
  if (hipDeviceSynchronize() != hipSuccess) return FG_EDEVICE;
  std::vector<int> ring(g_t.ring_used > 0 ? g_t.ring_used : 1);
  if (g_t.ring_used > 0)
    hipMemcpy(ring.data(), g_t.ring, sizeof(int) * g_t.ring_used, hipMemcpyDeviceToHost);
  double ms = 0, by = 0;
  int64_t cnt = 0;
  for (size_t i = 0; i < g_t.recs.size(); ++i) {
    float e = 0;
    const Rec& r = g_t.recs[i];
    if (!r.closed || hipEventElapsedTime(&e, g_t.ev[2 * i], g_t.ev[2 * i + 1]) != hipSuccess)
      continue;
    std::vector<int> km(r.L > 0 ? r.L : 1, 0);
    if (r.ring_off >= 0)
      for (int l = 0; l < r.L; ++l) km[l] = ring[r.ring_off + l];
    const double b = launch_bytes(r, km);
    ms += e;
    by += b;
    ++cnt;
    g_res[r.kid].ms += e;
    g_res[r.kid].bytes += b;
    g_res[r.kid].launches += 1;
  }
  for (auto e : g_t.ev) hipEventDestroy(e);
  g_t.ev.clear();
  g_t.recs.clear();
  if (total_ms) *total_ms = ms;
  if (launches) *launches = cnt;
  if (bytes) *bytes = by;
  return FG_OK;
}

}  // extern "C"
