// Recording and grouped replay of launches (see fg_group.h).
#include <algorithm>
#include <string>
#include <unordered_map>

#include "fg_group.h"

namespace fg {

namespace {
thread_local Recorder* t_rec = nullptr;
}

Recorder* recording() { return t_rec; }

RecordScope::RecordScope(Recorder* r) : prev_(t_rec) { t_rec = r; }
RecordScope::~RecordScope() { t_rec = prev_; }

void record_group(GroupFn fn, uintptr_t key, dim3 grid, dim3 block, uint32_t lds,
                  const void* args, size_t bytes) {
  Recorder* r = t_rec;
  RecLaunch L;
  L.fn = fn;
  L.key = key;
  L.grid = grid;
  L.block = block;
  L.lds = lds;
  L.off = (r->buf.size() + 15) / 16 * 16;
  L.bytes = bytes;
  r->buf.resize(L.off + bytes);
  std::memcpy(r->buf.data() + L.off, args, bytes);
  r->seq.push_back(std::move(L));
}

void run_or_record(uintptr_t key, hipStream_t s, std::function<void(hipStream_t)> f) {
  if (Recorder* r = t_rec) {
    RecLaunch L;
    L.key = key;
    L.direct = std::move(f);
    r->seq.push_back(std::move(L));
    return;
  }
  f(s);
}

GroupExec::~GroupExec() {
  if (dev_) (void)hipFree(dev_);
  if (pinned_) (void)hipHostFree(pinned_);
}

size_t GroupExec::stage(const void* host, size_t bytes) {
  const size_t off = (host_.size() + 255) / 256 * 256;
  host_.resize(off + bytes);
  std::memcpy(host_.data() + off, host, bytes);
  return off;
}

fg_status GroupExec::run(std::vector<Recorder*>& recs, hipStream_t s, std::string& err) {
  const int R = (int)recs.size();
  for (Recorder* r : recs)
    for (auto& L : r->seq) L.args_base = r->buf.data();
  std::vector<size_t> cur(R, 0);
  size_t left = 0;
  for (Recorder* r : recs) left += r->seq.size();
  launches = left;
  groups = 0;
  host_.clear();
  todo_.clear();
  std::unordered_map<uintptr_t, int> count;
  std::vector<const RecLaunch*> mem;
  // Each step takes the key most recorders are at and issues it for all of them (one
  // grouped launch, or each member's own launch); every recorder keeps its order.
  while (left > 0) {
    count.clear();
    uintptr_t best = 0;
    int bestc = 0;
    for (int i = 0; i < R; ++i) {
      if (cur[i] >= recs[i]->seq.size()) continue;
      const int c = ++count[recs[i]->seq[cur[i]].key];
      if (c > bestc) {
        bestc = c;
        best = recs[i]->seq[cur[i]].key;
      }
    }
    mem.clear();
    for (int i = 0; i < R; ++i)
      if (cur[i] < recs[i]->seq.size() && recs[i]->seq[cur[i]].key == best) {
        mem.push_back(&recs[i]->seq[cur[i]]);
        ++cur[i];
      }
    left -= mem.size();
    ++groups;
    if (mem[0]->fn) {
      mem[0]->fn(*this, mem.data(), (int)mem.size());
    } else {
      for (const RecLaunch* L : mem) todo_.push_back(L->direct);
    }
  }
  // one upload of every staged argument array, then the launches in order
  const size_t bytes = std::max<size_t>(host_.size(), 256);
  if (bytes > dev_cap_) {
    if (dev_) (void)hipFree(dev_);
    dev_ = nullptr;
    dev_cap_ = 0;
    if (hipMalloc(reinterpret_cast<void**>(&dev_), 2 * bytes) != hipSuccess) {
      (void)hipGetLastError();
      err = "grouped launch: argument buffer allocation failed";
      return FG_ENOMEM;
    }
    dev_cap_ = 2 * bytes;
  }
  if (bytes > pinned_cap_) {
    if (pinned_) (void)hipHostFree(pinned_);
    pinned_ = nullptr;
    pinned_cap_ = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&pinned_), 2 * bytes) != hipSuccess) {
      (void)hipGetLastError();
      err = "grouped launch: staging buffer allocation failed";
      return FG_ENOMEM;
    }
    pinned_cap_ = 2 * bytes;
  }
  if (!host_.empty()) {
    std::memcpy(pinned_, host_.data(), host_.size());
    if (hipMemcpyAsync(dev_, pinned_, host_.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
      err = "grouped launch: argument upload failed";
      return FG_EDEVICE;
    }
  }
  for (auto& f : todo_) f(s);
  todo_.clear();
  for (Recorder* r : recs) r->clear();
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("grouped launch: ") + hipGetErrorString(e);
    return FG_EDEVICE;
  }
  return FG_OK;
}

}  // namespace fg
