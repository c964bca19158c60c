// Internal chain interface shared by the C ABI and the serving loop (not public).
#pragma once
#include <string>
#include <vector>

#include "fg_internal.h"

namespace fg {

// Host plans of every grid point of one chain (no device memory yet), the capacity they
// need and the chain's exact device footprint.  Thread-safe to compute.
struct ChainPlans {
  std::vector<PlanPack*> packs;
  Caps caps;
  size_t plan_bytes = 0;
  size_t bytes = 0;  // device bytes of the chain these plans make (FP32/FP64 as configured)
  ChainPlans() = default;
  ChainPlans(const ChainPlans&) = delete;
  ChainPlans& operator=(const ChainPlans&) = delete;
  ~ChainPlans();
};
fg_status chain_plan(const fg_chain_cfg& cfg, const double* xh, int n, ChainPlans& out,
                     std::string& err);

// Streams and events a caller lends to a chain (the chain neither creates nor destroys
// them): the proposal's stream, two side streams and five events.
struct ChainStreams {
  hipStream_t aux = nullptr, zs = nullptr, ls = nullptr;
  hipEvent_t ev[5] = {};
};

// A chain from its plans (moved out of `plans`).  x, y: n values on the host
// (host_inputs) or the device.  Memory comes from dev_alloc / host_alloc.  The set-up
// (uploads, build and factor at the starting length-scale) is enqueued on s; with sync it
// is also waited for, else the caller waits for s before the first sweep reads anything.
fg_status chain_create_planned(const fg_chain_cfg& cfg, ChainPlans& plans, const double* x,
                               const double* y, bool host_inputs, int n, hipStream_t s,
                               const ChainStreams* borrowed, bool sync, fg_chain* out,
                               std::string& err);
// Frees a chain without waiting for the device: nothing queued may still use it.
void chain_destroy_idle(fg_chain c);
// One sweep in two halves, for callers that watch the stream themselves: begin enqueues
// the sweep on s (again = the same proposal once more); end, called once s has finished,
// returns true if the sweep must be run again (its state has been restored on s: call
// begin with again = true), else applies the sweep's outcome.  begin returns the first
// runtime error met while enqueuing (hipSuccess if none).
hipError_t chain_begin_sweep(fg_chain c, hipStream_t s, bool again);
bool chain_end_sweep(fg_chain c, hipStream_t s);
size_t chain_device_bytes(fg_chain c);
const double* chain_f(fg_chain c);  // device, n: f of the last sweep
// dev_alloc calls one chain makes at most (for the 256-byte rounding of each)
size_t chain_alloc_count(const fg_chain_cfg& cfg);
int64_t chain_iteration(fg_chain c);

}  // namespace fg
