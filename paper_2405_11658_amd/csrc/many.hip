// Batched updates of many independent graphs (see leiden_update_many in
// include/leiden.h): the updates run concurrently, each on a stream of its
// own driven by a host worker thread, so that the kernels of small graphs
// overlap on the device instead of running one graph after another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <unordered_set>
#include <vector>

#include "leiden.h"

namespace {
constexpr int kDefaultWorkers = 8;
constexpr int kMaxWorkers = 64;
}  // namespace

extern "C" leiden_status leiden_update_many(leiden_handle *const *handles, const leiden_batch *batches,
                                            const int32_t *modes, int32_t count,
                                            int32_t *const *membership_out, double *q_out,
                                            leiden_stats *stats, leiden_status *status_out,
                                            int32_t max_parallel, void *stream) {
  if (count < 0 || max_parallel < 0 || max_parallel > kMaxWorkers) return LEIDEN_EINVAL;
  if (count == 0) return LEIDEN_OK;
  if (!handles || !batches || !modes) return LEIDEN_EINVAL;
  {
    std::unordered_set<const void *> seen;
    for (int32_t k = 0; k < count; ++k)
      if (!handles[k] || !seen.insert(handles[k]).second) return LEIDEN_EINVAL;  // one call per handle
  }
  hipEvent_t start;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess) return LEIDEN_EHIP;
  if (hipEventRecord(start, (hipStream_t)stream) != hipSuccess) {
    (void)hipEventDestroy(start);
    return LEIDEN_EHIP;
  }
  const int workers = std::min<int>(count, max_parallel > 0 ? max_parallel : kDefaultWorkers);
  std::vector<leiden_status> st(count, LEIDEN_OK);
  std::atomic<int32_t> next{0};
  std::atomic<int> hip_fail{0};
  int device = 0;
  (void)hipGetDevice(&device);
  auto work = [&]() {
    (void)hipSetDevice(device);
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      hip_fail = 1;
      return;
    }
    hipEvent_t done;
    bool ok = hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess &&
              hipStreamWaitEvent(s, start, 0) == hipSuccess;
    for (;;) {
      const int32_t k = next.fetch_add(1);
      if (k >= count) break;
      if (!ok) {
        st[k] = LEIDEN_EHIP;
        continue;
      }
      st[k] = leiden_update(handles[k], &batches[k], modes[k], membership_out ? membership_out[k] : nullptr,
                            q_out ? &q_out[k] : nullptr, stats ? &stats[k] : nullptr, nullptr, s);
    }
    if (ok) {
      // make the caller's stream wait for this worker's work
      if (hipEventRecord(done, s) != hipSuccess || hipStreamWaitEvent((hipStream_t)stream, done, 0) != hipSuccess)
        hip_fail = 1;
      (void)hipStreamSynchronize(s);
      (void)hipEventDestroy(done);
    } else {
      hip_fail = 1;
    }
    (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  pool.reserve(workers);
  for (int t = 0; t < workers; ++t) pool.emplace_back(work);
  for (auto &t : pool) t.join();
  (void)hipEventDestroy(start);
  leiden_status first = LEIDEN_OK;
  for (int32_t k = 0; k < count; ++k) {
    if (status_out) status_out[k] = st[k];
    if (first == LEIDEN_OK && st[k] != LEIDEN_OK) first = st[k];
  }
  if (first == LEIDEN_OK && hip_fail) first = LEIDEN_EHIP;
  return first;
}
