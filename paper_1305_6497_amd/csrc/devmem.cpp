// Device memory for the library's handles.
//
// hipFree waits for the whole device, so with several requests in flight on
// their own streams (the serving loop) freeing one target's buffers would
// stall behind every other request's kernels.  Freed blocks are kept instead,
// per device, and handed out again to later allocations of about the same size
// (best fit within 25%).  Callers return a block only after the work that used
// it has finished.  The cache holds at most a quarter of the device memory;
// blocks beyond that, and the whole cache when hipMalloc runs out of memory,
// are released with hipFree.  Small pinned host blocks (the status reads of
// the solve loop) come from a pool of their own.
#include <map>
#include <mutex>
#include <vector>

#include "dda_internal.hpp"

namespace dda {

namespace {

struct DeviceCache {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void *>> free_blocks;   // device -> (size -> block)
  std::map<int, size_t> cached;                                // bytes held per device
  std::map<int, size_t> cap;                                   // cache limit per device

  size_t limit(int dev) {
    auto it = cap.find(dev);
    if (it != cap.end()) return it->second;
    size_t fr = 0, tot = 0;
    size_t c = (size_t)2 << 30;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && tot / 4 > c) c = tot / 4;
    cap[dev] = c;
    return c;
  }

  void trim(int dev) {       // caller holds mu
    auto &m = free_blocks[dev];
    for (auto &kv : m) (void)hipFree(kv.second);
    m.clear();
    cached[dev] = 0;
  }
};

DeviceCache &cache() {
  static DeviceCache *c = new DeviceCache;     // never destroyed: no hipFree during static teardown
  return *c;
}

size_t round_size(size_t bytes) {
  const size_t mib = (size_t)1 << 20;
  if (bytes < mib) {
    size_t r = 512;
    while (r < bytes) r <<= 1;
    return r;
  }
  const size_t g = 2 * mib;
  return (bytes + g - 1) / g * g;
}

}  // namespace

void *dev_alloc(int device, size_t bytes, size_t *granted) {
  const size_t want = round_size(bytes < 16 ? 16 : bytes);
  DeviceCache &c = cache();
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto &m = c.free_blocks[device];
    auto it = m.lower_bound(want);
    if (it != m.end() && it->first <= want + want / 4) {
      void *p = it->second;
      *granted = it->first;
      c.cached[device] -= it->first;
      m.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(c.mu);
    c.trim(device);
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{e == hipErrorOutOfMemory ? DDA_ENOMEM : DDA_EDEVICE,
                std::string("hipMalloc: ") + hipGetErrorString(e)};
  }
  *granted = want;
  return p;
}

void dev_release(int device, void *p, size_t granted) {
  if (!p) return;
  DeviceCache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (c.cached[device] + granted > c.limit(device)) {
    (void)hipFree(p);
    return;
  }
  c.free_blocks[device].emplace(granted, p);
  c.cached[device] += granted;
}

// Pinned host blocks for the small status reads of the solve loop.  They are
// kept for reuse, never freed: hipHostFree can wait for the device, which
// would stall a closing handle behind other requests' kernels.
namespace {
struct PinnedPool {
  std::mutex mu;
  std::multimap<size_t, void *> free_blocks;
};
PinnedPool &pinned_pool() {
  static PinnedPool *p = new PinnedPool;
  return *p;
}
}  // namespace

void *pinned_alloc(size_t bytes, size_t *granted) {
  const size_t want = round_size(bytes < 16 ? 16 : bytes);
  PinnedPool &pool = pinned_pool();
  {
    std::lock_guard<std::mutex> lk(pool.mu);
    auto it = pool.free_blocks.lower_bound(want);
    if (it != pool.free_blocks.end() && it->first <= 2 * want) {
      void *p = it->second;
      *granted = it->first;
      pool.free_blocks.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  const hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{e == hipErrorOutOfMemory ? DDA_ENOMEM : DDA_EDEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e)};
  }
  *granted = want;
  return p;
}

void pinned_release(void *p, size_t granted) {
  if (!p) return;
  PinnedPool &pool = pinned_pool();
  std::lock_guard<std::mutex> lk(pool.mu);
  pool.free_blocks.emplace(granted, p);
}

}  // namespace dda
