// Device and pinned-host memory of the library.  By default every buffer is a runtime
// allocation (hipMalloc / hipHostMalloc).  A host thread that opens an ArenaScope carves
// its buffers from that arena instead: one allocation made up front and sub-allocated
// best-fit, so that code which must not call the runtime allocator (the serving loop,
// where hipFree would synchronise the device and stall every running job) can still
// create and destroy chains.  dev_free / host_free find the arena that holds a pointer
// from the pointer itself, so memory may be released from any thread.
#include <map>
#include <mutex>

#include "fg_internal.h"

namespace fg {

namespace {
constexpr size_t ALIGN = 256;

std::mutex g_reg_mu;
std::map<uintptr_t, Arena*> g_registry;  // base address -> arena
thread_local Arena* t_dev_arena = nullptr;
thread_local Arena* t_host_arena = nullptr;

// the innermost arena holding p: arenas may nest (a view over a block of another arena),
// so the search walks down from the closest base address until one contains p
Arena* owner_of(const void* p) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto it = g_registry.upper_bound(a);
  while (it != g_registry.begin()) {
    --it;
    if (a < it->first + it->second->capacity()) return it->second;
  }
  return nullptr;
}
}  // namespace

Arena::~Arena() { release(); }

fg_status Arena::init(size_t bytes, bool pinned_host, std::string& err) {
  release();
  bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
  void* p = nullptr;
  const hipError_t e = pinned_host ? hipHostMalloc(&p, bytes) : hipMalloc(&p, bytes);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    err = "arena allocation of " + std::to_string(bytes) + " bytes failed";
    return FG_ENOMEM;
  }
  base_ = static_cast<char*>(p);
  cap_ = bytes;
  pinned_ = pinned_host;
  view_ = false;
  free_.clear();
  used_.clear();
  free_[0] = bytes;
  in_use_ = 0;
  std::lock_guard<std::mutex> lk(g_reg_mu);
  g_registry[reinterpret_cast<uintptr_t>(base_)] = this;
  return FG_OK;
}

fg_status Arena::init_view(void* base, size_t bytes) {
  release();
  base_ = static_cast<char*>(base);
  cap_ = bytes / ALIGN * ALIGN;
  view_ = true;
  free_.clear();
  used_.clear();
  free_[0] = cap_;
  in_use_ = 0;
  std::lock_guard<std::mutex> lk(g_reg_mu);
  g_registry[reinterpret_cast<uintptr_t>(base_)] = this;
  return FG_OK;
}

void Arena::release() {
  if (!base_) return;
  {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_registry.find(reinterpret_cast<uintptr_t>(base_));
    if (it != g_registry.end() && it->second == this) g_registry.erase(it);
  }
  if (view_)
    ;  // the memory belongs to the enclosing arena
  else if (pinned_)
    (void)hipHostFree(base_);
  else
    (void)hipFree(base_);
  view_ = false;
  base_ = nullptr;
  cap_ = 0;
  free_.clear();
  used_.clear();
  in_use_ = 0;
}

void* Arena::alloc(size_t bytes) {
  if (bytes == 0) bytes = 1;
  bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
  std::lock_guard<std::mutex> lk(mu_);
  // best fit: the smallest free block that holds the request
  auto best = free_.end();
  for (auto it = free_.begin(); it != free_.end(); ++it)
    if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
  if (best == free_.end()) return nullptr;
  const size_t off = best->first, sz = best->second;
  free_.erase(best);
  if (sz > bytes) free_[off + bytes] = sz - bytes;
  used_[off] = bytes;
  in_use_ += bytes;
  return base_ + off;
}

void Arena::free(void* p) {
  const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
  std::lock_guard<std::mutex> lk(mu_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t start = off, sz = u->second;
  used_.erase(u);
  in_use_ -= sz;
  // coalesce with the free neighbours
  auto next = free_.lower_bound(start);
  if (next != free_.end() && next->first == start + sz) {
    sz += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == start) {
      start = prev->first;
      sz += prev->second;
      free_.erase(prev);
    }
  }
  free_[start] = sz;
}

size_t Arena::largest_free() const {
  std::lock_guard<std::mutex> lk(mu_);
  size_t m = 0;
  for (const auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

size_t Arena::in_use() const {
  std::lock_guard<std::mutex> lk(mu_);
  return in_use_;
}

ArenaScope::ArenaScope(Arena* dev, Arena* host)
    : prev_dev_(t_dev_arena), prev_host_(t_host_arena) {
  t_dev_arena = dev;
  t_host_arena = host;
}

ArenaScope::~ArenaScope() {
  t_dev_arena = prev_dev_;
  t_host_arena = prev_host_;
}

hipError_t dev_alloc(void** p, size_t bytes) {
  if (Arena* a = t_dev_arena) {
    *p = a->alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void dev_free(void* p) {
  if (!p) return;
  if (Arena* a = owner_of(p)) {
    a->free(p);
    return;
  }
  (void)hipFree(p);
}

hipError_t host_alloc(void** p, size_t bytes) {
  if (Arena* a = t_host_arena) {
    *p = a->alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipHostMalloc(p, bytes);
}

void host_free(void* p) {
  if (!p) return;
  if (Arena* a = owner_of(p)) {
    a->free(p);
    return;
  }
  (void)hipHostFree(p);
}

}  // namespace fg
