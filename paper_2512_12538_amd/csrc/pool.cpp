// Caching device allocator; see pool.h.
#include "pool.h"

#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

namespace devpool {
namespace {

struct Block {
  void* p;
  size_t bytes;
  hipStream_t stream;
  hipEvent_t done;  // recorded on `stream` at release (null: nothing pending)
};

struct Device {
  std::multimap<size_t, Block> free;  // by size class
  size_t cached = 0;
  size_t cap = 0;
};

std::mutex mu;
std::map<int, Device> devices;

Device& device(int& id) {
  if (hipGetDevice(&id) != hipSuccess) id = 0;
  Device& d = devices[id];
  if (d.cap == 0) {
    size_t fr = 0, total = 0;
    if (hipMemGetInfo(&fr, &total) != hipSuccess) total = 0;
    (void)hipGetLastError();
    d.cap = total / 4;
    if (const char* env = std::getenv("HH_POOL_CAP_GB")) {
      const double gb = std::atof(env);
      if (gb >= 0.0) d.cap = (size_t)(gb * 1073741824.0);
    }
    if (d.cap == 0 && total == 0) d.cap = (size_t)16 << 30;
  }
  return d;
}

void destroy(Block& b) {
  if (b.done) {
    (void)hipEventSynchronize(b.done);
    (void)hipEventDestroy(b.done);
  }
  (void)hipFree(b.p);
}

size_t trim_locked(Device& d) {
  size_t n = 0;
  for (auto& kv : d.free) {
    n += kv.second.bytes;
    destroy(kv.second);
  }
  d.free.clear();
  d.cached = 0;
  return n;
}

}  // namespace

size_t size_class(size_t bytes) {
  if (bytes == 0) return 0;
  const size_t mib = (size_t)1 << 20;
  if (bytes <= mib) return (bytes + 255) & ~(size_t)255;
  const size_t two = 2 * mib;
  return (bytes + two - 1) / two * two;
}

void* acquire(size_t bytes, hipStream_t stream) {
  const size_t sc = size_class(bytes);
  if (sc == 0) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  int id = 0;
  Device& d = device(id);
  auto it = d.free.find(sc);
  if (it != d.free.end()) {
    // prefer a block last used on this stream
    for (auto jt = it; jt != d.free.end() && jt->first == sc; ++jt)
      if (jt->second.stream == stream) {
        it = jt;
        break;
      }
    Block b = it->second;
    d.free.erase(it);
    d.cached -= b.bytes;
    if (b.done) {
      if (b.stream != stream) (void)hipEventSynchronize(b.done);
      (void)hipEventDestroy(b.done);
    }
    (void)hipGetLastError();
    return b.p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, sc) != hipSuccess) {
    (void)hipGetLastError();
    trim_locked(d);
    p = nullptr;
    if (hipMalloc(&p, sc) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  return p;
}

void release(void* p, size_t bytes, hipStream_t stream, bool idle) {
  if (!p) return;
  const size_t sc = size_class(bytes);
  std::lock_guard<std::mutex> lk(mu);
  int id = 0;
  Device& d = device(id);
  Block b{p, sc, idle ? nullptr : stream, nullptr};
  if (!idle && (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(b.done, stream) != hipSuccess)) {
    (void)hipGetLastError();
    if (b.done) (void)hipEventDestroy(b.done);
    b.done = nullptr;
    b.stream = nullptr;
    (void)hipStreamSynchronize(stream);
  }
  d.free.emplace(sc, b);
  d.cached += sc;
  // over the cap: free the largest cached blocks first
  while (d.cached > d.cap && !d.free.empty()) {
    auto last = std::prev(d.free.end());
    d.cached -= last->second.bytes;
    destroy(last->second);
    d.free.erase(last);
  }
  (void)hipGetLastError();
}

void forget_stream(hipStream_t stream) {
  std::lock_guard<std::mutex> lk(mu);
  for (auto& dv : devices)
    for (auto& kv : dv.second.free) {
      Block& b = kv.second;
      if (b.stream != stream) continue;
      if (b.done) {
        (void)hipEventSynchronize(b.done);
        (void)hipEventDestroy(b.done);
        b.done = nullptr;
      }
      b.stream = nullptr;
    }
  (void)hipGetLastError();
}

size_t trim() {
  std::lock_guard<std::mutex> lk(mu);
  int id = 0;
  return trim_locked(device(id));
}

size_t cached_bytes() {
  std::lock_guard<std::mutex> lk(mu);
  int id = 0;
  return device(id).cached;
}

}  // namespace devpool
