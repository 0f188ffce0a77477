// Caching device allocator of the library. Registration, tree build and batch
// calls need a few dozen device buffers each; hipMalloc and hipFree cost tens
// of microseconds apiece and hipFree waits for the device, so a released block
// is kept in a free list of its size class and handed out again once the work
// queued on it before its release has finished (an event recorded at release
// on the stream that last used it). Blocks stay cached until fga_trim_cache
// or process exit. Calls from several threads are serialised by a mutex.
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace fga {
namespace {

struct Cached {
  void* p;
  hipEvent_t done;  // recorded at release; null: no pending work
};

struct PoolState {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<Cached>> free;  // (device, class) -> blocks
  std::map<void*, std::pair<int, size_t>> live;               // block -> (device, class)
  std::vector<hipEvent_t> spare_events;
};

PoolState& pool() {
  static PoolState* ps = new PoolState;  // never destroyed: blocks live until exit
  return *ps;
}

// Size class: powers of two from 512 B to 1 MiB, then multiples of 2 MiB.
size_t size_class(size_t bytes) {
  if (bytes <= 512) return 512;
  if (bytes <= (size_t)1 << 20) {
    size_t c = 512;
    while (c < bytes) c <<= 1;
    return c;
  }
  const size_t g = (size_t)2 << 20;
  return (bytes + g - 1) / g * g;
}

// hipFree of every idle cached block (pending ones stay); called with mu held.
void trim_locked(PoolState& ps) {
  for (auto& kv : ps.free) {
    std::vector<Cached> keep;
    for (Cached& c : kv.second) {
      if (c.done && hipEventQuery(c.done) != hipSuccess) {
        keep.push_back(c);
        continue;
      }
      if (c.done) ps.spare_events.push_back(c.done);
      (void)hipFree(c.p);
    }
    kv.second.swap(keep);
  }
}

}  // namespace

void* pool_alloc(size_t bytes, hipStream_t s) {
  (void)s;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return nullptr;
  }
  const size_t cls = size_class(bytes);
  PoolState& ps = pool();
  std::lock_guard<std::mutex> lk(ps.mu);
  auto& fl = ps.free[{dev, cls}];
  for (size_t i = 0; i < fl.size(); ++i) {
    Cached c = fl[i];
    if (c.done && hipEventQuery(c.done) != hipSuccess) continue;  // still in use
    fl.erase(fl.begin() + (long)i);
    if (c.done) ps.spare_events.push_back(c.done);
    ps.live[c.p] = {dev, cls};
    return c.p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e != hipSuccess) {  // return idle cached memory to the device and retry once
    (void)hipGetLastError();
    trim_locked(ps);
    e = hipMalloc(&p, cls);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed: %s", cls, hipGetErrorString(e));
    return nullptr;
  }
  ps.live[p] = {dev, cls};
  return p;
}

void pool_free(void* p, hipStream_t s) {
  if (!p) return;
  PoolState& ps = pool();
  std::lock_guard<std::mutex> lk(ps.mu);
  auto it = ps.live.find(p);
  if (it == ps.live.end()) return;  // not a pool block
  const auto key = it->second;
  ps.live.erase(it);
  hipEvent_t ev = nullptr;
  if (!ps.spare_events.empty()) {
    ev = ps.spare_events.back();
    ps.spare_events.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    ev = nullptr;
  }
  if (ev && hipEventRecord(ev, s) != hipSuccess) {  // cannot track: wait instead
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    ps.spare_events.push_back(ev);
    ev = nullptr;
  } else if (!ev) {
    (void)hipStreamSynchronize(s);
  }
  ps.free[key].push_back(Cached{p, ev});
}

fga_status pool_trim() {
  PoolState& ps = pool();
  std::lock_guard<std::mutex> lk(ps.mu);
  trim_locked(ps);
  return FGA_OK;
}

}  // namespace fga

extern "C" fga_status fga_trim_cache(void) { return fga::pool_trim(); }
