// Host-side device-memory plumbing shared by the library's entry points:
// a buffer record, the allocator in use (the caller's leiden_allocator or
// HIP's stream-ordered allocator) and a process-wide pool of pinned staging
// blocks.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "leiden.h"

namespace lk {

struct DBuf {
  void *p = nullptr;
  size_t cap = 0;
};

constexpr size_t kPinBytes = 65536;

// Device memory of a handle or of a stateless call: obtained from the
// caller's allocator when one is given (leiden_allocator), else from HIP's
// stream-ordered allocator; every release is ordered on a stream after the
// work that last used the memory, so no release waits for the device.
struct Alloc {
  leiden_allocator a{};
  bool custom = false;
  void *get(size_t bytes, hipStream_t s) {
    if (custom) return a.alloc(a.ctx, bytes, (void *)s);
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void *p, size_t bytes, hipStream_t s) {
    if (!p) return;
    if (custom) a.release(a.ctx, p, bytes, (void *)s);
    else (void)hipFreeAsync(p, s);
  }
};

// Pinned host staging blocks (device -> host reads of scalars and small
// arrays) are shared by all handles through a process-wide free list, so that
// releasing a handle never frees pinned memory (which would wait for the
// whole device).
struct PinPool {
  std::mutex mu;
  std::vector<void *> free;
  void *take() {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (!free.empty()) {
        void *p = free.back();
        free.pop_back();
        return p;
      }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, kPinBytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void give(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    free.push_back(p);
  }
};
inline PinPool &pin_pool() {
  static PinPool *pool = new PinPool();  // never destroyed: blocks live until the process ends
  return *pool;
}

}  // namespace lk
