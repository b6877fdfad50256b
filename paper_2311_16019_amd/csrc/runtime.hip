// Process-wide device memory and stream reuse.
//
// A solve allocates a few gigabytes (the stored bases) and several streams; allocating
// them with hipMalloc / hipStreamCreate on every call, and releasing them with hipFree /
// hipStreamDestroy, costs milliseconds per solve.  Released blocks are kept in a per-device
// cache and handed out again to later requests of nearly the same size; released streams
// are kept for reuse.
//
// Safety of reuse: a released block may still be read or written by kernels in flight on
// any stream.  Every block that is released marks its device "dirty"; the first reuse of a
// cached block on a dirty device synchronises the device (which is what hipFree would have
// done at release time) and clears the mark.  Code that has already waited for all work on
// the blocks it releases says so with a quiet scope (PoolQuiet): blocks released inside it
// do not mark the device, so that concurrent solves on other host threads are not stalled
// by a device synchronisation.  A reused stream only orders new work after the work already
// queued on it.
#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.hpp"

namespace skr {
namespace {

// Cached bytes kept per device at most: 60% of the device's memory, so that the two stored
// bases of a full-length solve (60 GB each at n = 1e6, r = 4, FP64, 1876 blocks) stay cached
// from one solve to the next instead of being freed and allocated again (a free and an
// allocation of that size cost about 0.6 s per solve).
constexpr size_t kCacheCapMin = size_t(64) << 30;

thread_local int tl_quiet = 0;  // depth of quiet scopes on this host thread
constexpr int kMaxDev = 64;

struct Live {
  size_t bytes;
  int dev;
};

struct Pool {
  std::mutex mu;
  size_t cap[kMaxDev] = {};  // per device, set on its first release
  std::unordered_map<void*, Live> live;
  std::multimap<std::pair<int, size_t>, void*> cached;  // (device, bytes) -> block
  size_t cached_bytes[kMaxDev] = {};
  bool dirty[kMaxDev] = {};
  std::multimap<int, hipStream_t> streams;  // device -> idle stream
};

// Never destroyed: the HIP runtime may already be torn down when static destructors run.
Pool& pool() {
  static Pool* p = new Pool;
  return *p;
}

size_t round_bytes(size_t b) {
  const size_t g = b >= (size_t(1) << 20) ? (size_t(2) << 20) : 512;
  return (b + g - 1) / g * g;
}

int current_device() {
  int d = 0;
  SKR_HIP(hipGetDevice(&d));
  SKR_REQUIRE(d >= 0 && d < kMaxDev, "device index out of range");
  return d;
}

// Release every cached block of device `dev` (current device); caller holds the lock.
void trim_locked(Pool& P, int dev) {
  auto lo = P.cached.lower_bound({dev, 0}), hi = P.cached.lower_bound({dev + 1, 0});
  if (lo == hi) return;
  (void)hipDeviceSynchronize();
  for (auto it = lo; it != hi; ++it) (void)hipFree(it->second);
  P.cached.erase(lo, hi);
  P.cached_bytes[dev] = 0;
  P.dirty[dev] = false;
}

}  // namespace

void* pool_alloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  Pool& P = pool();
  const int dev = current_device();
  const size_t want = round_bytes(bytes);
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.cached.lower_bound({dev, want});
  if (it != P.cached.end() && it->first.first == dev && it->first.second <= want + want / 4) {
    if (P.dirty[dev]) {
      SKR_HIP(hipDeviceSynchronize());
      P.dirty[dev] = false;
    }
    void* p = it->second;
    const size_t have = it->first.second;
    P.cached.erase(it);
    P.cached_bytes[dev] -= have;
    P.live[p] = Live{have, dev};
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_locked(P, dev);
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(SKR_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
  }
  P.live[p] = Live{want, dev};
  return p;
}

void pool_free(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) {
    (void)hipFree(p);
    return;
  }
  const Live L = it->second;
  P.live.erase(it);
  if (P.cap[L.dev] == 0) {
    size_t free_b = 0, total_b = 0;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(L.dev);
    const bool ok = hipMemGetInfo(&free_b, &total_b) == hipSuccess;
    (void)hipSetDevice(cur);
    if (!ok) (void)hipGetLastError();
    P.cap[L.dev] = std::max(kCacheCapMin, ok ? total_b / 10 * 6 : size_t(0));
  }
  const size_t cap = P.cap[L.dev];
  if (L.bytes > cap) {
    (void)hipFree(p);
    return;
  }
  // keep the cache bounded: drop the largest cached blocks of this device first
  while (P.cached_bytes[L.dev] + L.bytes > cap) {
    auto hi = P.cached.lower_bound({L.dev + 1, 0});
    if (hi == P.cached.begin()) break;
    auto last = std::prev(hi);
    if (last->first.first != L.dev) break;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(L.dev);
    (void)hipDeviceSynchronize();
    (void)hipFree(last->second);
    (void)hipSetDevice(cur);
    P.cached_bytes[L.dev] -= last->first.second;
    P.cached.erase(last);
  }
  P.cached.insert({{L.dev, L.bytes}, p});
  P.cached_bytes[L.dev] += L.bytes;
  if (tl_quiet == 0) P.dirty[L.dev] = true;
}

void pool_quiet_enter() { ++tl_quiet; }
void pool_quiet_leave() { --tl_quiet; }

void pool_trim() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (int d = 0; d < kMaxDev; ++d) {
    if (P.cached_bytes[d] == 0) continue;
    (void)hipSetDevice(d);
    trim_locked(P, d);
  }
  (void)hipSetDevice(cur);
}

hipStream_t stream_acquire() {
  Pool& P = pool();
  const int dev = current_device();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.streams.find(dev);
    if (it != P.streams.end()) {
      hipStream_t s = it->second;
      P.streams.erase(it);
      return s;
    }
  }
  hipStream_t s = nullptr;
  SKR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return s;
}

void stream_release(hipStream_t s) {
  if (!s) return;
  Pool& P = pool();
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(P.mu);
  P.streams.insert({dev, s});
}

}  // namespace skr
