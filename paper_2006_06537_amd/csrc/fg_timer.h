// Live kernel timing hooks (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "fg_internal.h"

namespace fg {
bool timer_wants(int kid);
bool timer_active();  // a kernel is being timed (launches must stay eager)
void timer_before(int kid, hipStream_t s, int level, const HostPlan& P, const int* kmax_dev,
                  int ntask);
void timer_after(int kid, hipStream_t s);
// for a kernel whose algorithmic bytes are known at launch
void timer_before_bytes(int kid, hipStream_t s, double bytes);
// the ranks behind kmax_dev are about to change (a build) or the buffer is being freed:
// the next timed launch that reads them takes a new snapshot
void timer_forget(const int* kmax_dev);
}  // namespace fg
