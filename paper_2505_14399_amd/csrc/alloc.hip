// Device memory of the library: a per-device cache of freed blocks in front of hipMalloc.
//
// A setup and a solve allocate the same buffer sizes every time they run (Krylov bases, the
// hierarchy's fields, the K-cycle's vectors); with the cache a repeated setup or solve finds its
// blocks again instead of returning them to the runtime and mapping them anew (at 32^3 x 64 with
// 12 right-hand sides the flexible outer solver alone holds two 40 GB bases).
//
// Rules:
//  * A request is rounded up (to 4 KiB below 4 MiB, to 2 MiB above) and served by the smallest
//    cached block of that device whose size lies within 1/8 above the rounded size.
//  * A block enters the cache only after the device has finished all of its work
//    (hipDeviceSynchronize, the same wait hipFree performs), so no kernel still in flight can
//    read or write it once it is handed out again, whatever stream the next user runs on.
//  * The cache of a device holds at most half of the device's memory (QMG_CACHE_GB overrides,
//    0 turns caching off); above that the blocks cached longest ago are released first.
//  * When hipMalloc fails every cached block of the device is released and the call retried.
//  * qmg_memory_trim releases the cache of the current device.
#include <cstdlib>
#include <map>
#include <mutex>

#include "qmg_internal.hpp"

namespace qmg {

namespace {

struct Cached {
  void* p;
  unsigned long long stamp;  // order of entry into the cache
};

struct DeviceCache {
  std::multimap<size_t, Cached> blocks;  // size -> block
  size_t cached = 0, cap = 0;
  unsigned long long next = 0;
  bool init = false;
};

std::mutex g_mu;
std::map<int, DeviceCache> g_dev;
std::map<void*, size_t> g_size;  // live and cached blocks -> allocated size

size_t round_up(size_t n) {
  const size_t g = n < (size_t(4) << 20) ? (size_t(4) << 10) : (size_t(2) << 20);
  return (n + g - 1) / g * g;
}

DeviceCache& cache_of(int dev) {
  DeviceCache& c = g_dev[dev];
  if (!c.init) {
    c.init = true;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = 0;
    c.cap = tot / 2;
    if (const char* e = std::getenv("QMG_CACHE_GB")) c.cap = size_t(std::strtod(e, nullptr) * double(1ull << 30));
  }
  return c;
}

void release_all(DeviceCache& c) {
  for (auto& kv : c.blocks) {
    (void)hipFree(kv.second.p);
    g_size.erase(kv.second.p);
  }
  c.blocks.clear();
  c.cached = 0;
}

int current_device() {
  int dev = 0;
  QMG_HIP(hipGetDevice(&dev));
  return dev;
}

}  // namespace

void* dev_alloc(size_t n) {
  const size_t want = round_up(n);
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCache& c = cache_of(dev);
  auto it = c.blocks.lower_bound(want);
  if (it != c.blocks.end() && it->first <= want + want / 8) {
    void* p = it->second.p;
    c.cached -= it->first;
    c.blocks.erase(it);
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess && !c.blocks.empty()) {
    (void)hipGetLastError();
    release_all(c);
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc(%zu bytes) failed: %s", want, hipGetErrorString(e));
    throw Error{QMG_ENOMEM};
  }
  g_size[p] = want;
  return p;
}

void dev_free(void* p) {  // called from destructors: never throws
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceSynchronize();  // nothing in flight may still use the block
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCache& c = cache_of(dev);
  auto sz = g_size.find(p);
  const size_t n = sz == g_size.end() ? 0 : sz->second;
  if (n == 0 || n > c.cap) {
    if (sz != g_size.end()) g_size.erase(sz);
    (void)hipFree(p);
    return;
  }
  c.blocks.emplace(n, Cached{p, c.next++});
  c.cached += n;
  while (c.cached > c.cap && !c.blocks.empty()) {  // release the blocks cached longest ago
    auto old = c.blocks.begin();
    for (auto it = c.blocks.begin(); it != c.blocks.end(); ++it)
      if (it->second.stamp < old->second.stamp) old = it;
    c.cached -= old->first;
    (void)hipFree(old->second.p);
    g_size.erase(old->second.p);
    c.blocks.erase(old);
  }
}

void dev_trim() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_mu);
  release_all(cache_of(dev));
}

size_t dev_cached() {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_mu);
  return cache_of(dev).cached;
}

}  // namespace qmg
