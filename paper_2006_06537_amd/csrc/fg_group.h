// Grouped launches across independent problems (internal).
//
// Many chains stepped together issue the same sequence of kernels, each on its own small
// problem: at n = 32 768 a sweep is about 230 launches of a few microseconds each, and a
// batch of 64 chains is bound by launch latency, not by the device.  While a recorder is
// open on a host thread, the library's launchers do not launch: they append a record
// (kernel, grid, block, dynamic LDS, argument struct) to the recorder.  One recorder per
// chain holds that chain's sweep in program order.  The executor then walks all
// recorders at once and issues every kernel that the chains reach at the same point as
// ONE grouped launch: a wrapper kernel whose blocks are partitioned among the members
// (prefix sums of their grids), each block running the unchanged kernel body on its
// member's arguments.  Launches that have no grouped form (small scalar kernels, copies)
// are replayed one by one at their place.  Chains are independent, so any interleaving
// that keeps each chain's own order gives the results of stepping them one by one, bit for
// bit: every block runs the same code on the same data.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>

#include "fg_internal.h"

namespace fg {

struct RecLaunch;
class GroupExec;
// launches the members of one group (all with the same kernel and key)
using GroupFn = void (*)(GroupExec& ex, const RecLaunch* const* members, int m);

struct RecLaunch {
  GroupFn fn = nullptr;            // grouped kernel launcher, or null: replay `direct`
  uintptr_t key = 0;               // kernel variant and launch shape (equal keys group)
  dim3 grid, block;
  uint32_t lds = 0;
  size_t off = 0, bytes = 0;       // argument struct in the recorder's buffer
  std::function<void(hipStream_t)> direct;
  const char* args_base = nullptr; // set by the executor
  const void* args() const { return args_base + off; }
};

class Recorder {
 public:
  std::vector<RecLaunch> seq;
  std::vector<char> buf;
  void clear() {
    seq.clear();
    buf.clear();
  }
};

// the recorder open on this thread (null: launch at once)
Recorder* recording();
// opens `r` on this thread for the scope's lifetime
class RecordScope {
 public:
  explicit RecordScope(Recorder* r);
  ~RecordScope();

 private:
  Recorder* prev_;
};

// records a grouped-capable launch (the caller has checked recording() != null)
void record_group(GroupFn fn, uintptr_t key, dim3 grid, dim3 block, uint32_t lds,
                  const void* args, size_t bytes);
// runs `f` on stream s now, or records it for replay on the batch stream
void run_or_record(uintptr_t key, hipStream_t s, std::function<void(hipStream_t)> f);

// A launch without a grouped form: the statement (which launches on the stream q_) runs on
// stream s now, or is recorded for replay at its place.  Each expansion site is its own
// key, so recorders that reach the same site are replayed together.
#define FG_RUN(s, ...)                                                              \
  do {                                                                              \
    static const char fg_site_ = 0;                                                 \
    if (::fg::recording()) {                                                        \
      ::fg::run_or_record(reinterpret_cast<uintptr_t>(&fg_site_), (s),              \
                          [=](hipStream_t q_) { __VA_ARGS__; });                    \
    } else {                                                                        \
      hipStream_t q_ = (s);                                                         \
      __VA_ARGS__;                                                                  \
    }                                                                               \
  } while (0)

// Replays recorders: groups, stages every group's argument array and block offsets in one
// upload, then launches on one stream.
class GroupExec {
 public:
  ~GroupExec();
  // appends `bytes` of host data to the upload; returns its offset in the device buffer
  // (the buffer's address is known only at launch time: dev_base())
  size_t stage(const void* host, size_t bytes);
  void launch_later(std::function<void(hipStream_t)> f) { todo_.push_back(std::move(f)); }
  // groups and runs the recorders' launches on s; the recorders are cleared
  fg_status run(std::vector<Recorder*>& recs, hipStream_t s, std::string& err);
  char* dev_base() const { return dev_; }
  size_t launches = 0, groups = 0;  // statistics of the last run

 private:
  std::vector<char> host_;
  char* dev_ = nullptr;
  size_t dev_cap_ = 0;
  char* pinned_ = nullptr;
  size_t pinned_cap_ = 0;
  std::vector<std::function<void(hipStream_t)>> todo_;
};

// the member of a grouped launch that block bx belongs to (start: prefix sums, m members)
__device__ __forceinline__ int group_member(const int* __restrict__ start, int m, int bx) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= bx) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// key of a grouped kernel: its group launcher and block shape.  Members that ask for
// different dynamic LDS sizes share one launch at the largest size: on one stream, split
// groups would run one after the other (measured: 64 chains at n = 32 768 stepped 35%
// slower with a group per LDS size than with one group at the largest).
inline uintptr_t group_key(const void* fn, dim3 b, uint32_t lds) {
  (void)lds;
  uintptr_t h = reinterpret_cast<uintptr_t>(fn);
  h = h * 1000003u ^ b.x;
  h = h * 1000003u ^ b.y;
  return h;
}

// Host side of one grouped kernel: the members' argument structs A, their block offsets
// (prefix sums of grid.x) and grid.y are staged; the group kernel runs on a grid of
// sum grid.x by max grid.y with the members' block and the largest dynamic LDS.
template <class A, class L>
void grouped_launch(GroupExec& ex, const RecLaunch* const* mem, int m, L launch) {
  std::vector<A> av(m);
  std::vector<int> st(m + 1, 0), gy(m);
  unsigned gmax = 1;
  uint32_t lds = 0;
  for (int i = 0; i < m; ++i) {
    std::memcpy(static_cast<void*>(&av[i]), mem[i]->args(), sizeof(A));
    st[i + 1] = st[i] + (int)mem[i]->grid.x;
    gy[i] = (int)mem[i]->grid.y;
    gmax = std::max(gmax, mem[i]->grid.y);
    lds = std::max(lds, mem[i]->lds);
  }
  const size_t oa = ex.stage(av.data(), sizeof(A) * m);
  const size_t os = ex.stage(st.data(), sizeof(int) * (m + 1));
  const size_t og = ex.stage(gy.data(), sizeof(int) * m);
  const dim3 grid((unsigned)st[m], gmax, 1), block = mem[0]->block;
  GroupExec* e = &ex;
  ex.launch_later([=](hipStream_t s) {
    if (grid.x == 0) return;
    launch(grid, block, lds, s, reinterpret_cast<const A*>(e->dev_base() + oa),
           reinterpret_cast<const int*>(e->dev_base() + os),
           reinterpret_cast<const int*>(e->dev_base() + og), m);
  });
}

}  // namespace fg
