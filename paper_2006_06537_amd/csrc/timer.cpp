// Live per-kernel timing: HIP events recorded around every launch of one selected
// kernel on the stream it is launched on, plus a device snapshot of the per-level
// ranks so that the algorithmic bytes of each launch can be computed after the fact
// without a host round trip.  The ranks change only when their matrix is built, so one
// snapshot serves every timed launch until the next build of that matrix.
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
};
struct TimerState {
  bool on = false;
  int kid = 0;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  std::vector<Rec> recs;
  int* ring = nullptr;          // device: kmax snapshots
  int ring_cap = 0, ring_used = 0;
  std::unordered_map<const int*, int> snap;  // rank buffer -> its current snapshot
};
TimerState g_t;
constexpr int RING_CAP = 1 << 16;
constexpr int MAX_REC = 8192;
}  // namespace

__global__ void k_snapshot(const int* __restrict__ src, int count, int* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = src[i];
}

bool timer_active() { return g_t.on; }

bool timer_wants(int kid) { return g_t.on && g_t.kid == kid && (int)g_t.recs.size() < MAX_REC; }

void timer_before(int kid, hipStream_t s, int level, const HostPlan& P, const int* kmax_dev,
                  int ntask) {
  if (!timer_wants(kid)) return;
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
  if (!timer_wants(kid)) return;
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

void timer_forget(const int* kmax_dev) { g_t.snap.erase(kmax_dev); }

void timer_after(int kid, hipStream_t s) {
  if (!g_t.on || g_t.kid != kid || g_t.ev.empty()) return;
  if (g_t.ev.size() != 2 * g_t.recs.size()) return;
  hipEventRecord(g_t.ev.back(), s);
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

fg_status fg_timer_start(int32_t kernel_id) {
  using namespace fg;
  if (kernel_id < KID_LEAF || kernel_id > KID_PREDICT) return FG_EINVAL;
  for (auto e : g_t.ev) hipEventDestroy(e);
  g_t.ev.clear();
  g_t.recs.clear();
  if (!g_t.ring && hipMalloc(reinterpret_cast<void**>(&g_t.ring), sizeof(int) * RING_CAP) != hipSuccess)
    return FG_ENOMEM;
  g_t.ring_cap = RING_CAP;
  g_t.ring_used = 0;
  g_t.snap.clear();
  g_t.kid = kernel_id;
  g_t.on = true;
  return FG_OK;
}

fg_status fg_timer_stop(double* total_ms, int64_t* launches, double* bytes) {
  using namespace fg;
  g_t.on = false;
  if (hipDeviceSynchronize() != hipSuccess) return FG_EDEVICE;
  std::vector<int> ring(g_t.ring_used > 0 ? g_t.ring_used : 1);
  if (g_t.ring_used > 0)
    hipMemcpy(ring.data(), g_t.ring, sizeof(int) * g_t.ring_used, hipMemcpyDeviceToHost);
  double ms = 0, by = 0;
  int64_t cnt = 0;
  for (size_t i = 0; i < g_t.recs.size(); ++i) {
    float e = 0;
    if (hipEventElapsedTime(&e, g_t.ev[2 * i], g_t.ev[2 * i + 1]) != hipSuccess) continue;
    const Rec& r = g_t.recs[i];
    std::vector<int> km(r.L > 0 ? r.L : 1, 0);
    if (r.ring_off >= 0)
      for (int l = 0; l < r.L; ++l) km[l] = ring[r.ring_off + l];
    ms += e;
    by += launch_bytes(r, km);
    ++cnt;
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
