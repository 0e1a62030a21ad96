// Serving loop for many resident dynamic graphs (see leiden_server_* in
// include/leiden.h).  Requests (an update batch for one handle) are queued on
// submission; a dispatcher admits them into free worker slots as long as the
// device-memory estimate of the admitted work stays within the budget and the
// request's handle is not already being updated (a handle is used by one
// thread at a time).  A request that does not fit does not block later ones
// that do (continuous batching).  Each worker drives its own stream, so the
// admitted updates overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <iterator>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "leiden.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id;
  leiden_handle *h;      // a handle's update, or
  leiden_fleet *fleet;   // a job on one graph of a fleet (run with the fleet's other queued jobs)
  int32_t graph;
  leiden_batch b;
  int32_t mode;
  int32_t *out;
  int64_t bytes;
  Clock::time_point submitted;
  // results
  leiden_status st = LEIDEN_OK;
  double q = 0.0;
  leiden_stats stats;
  double latency_ms = 0.0;
  double service_ms = 0.0;
  bool done = false;
};

constexpr int kMaxFleetJobs = 4096;  // jobs gathered into one fleet launch

// Device bytes an admitted update may use beyond what is already held: the
// handle's workspace growth for this batch (leiden_update_bytes: the grown
// graph, its level and aggregation buffers, the directed batch) - taken when
// the request is considered for admission, since an earlier update of the
// same handle may have grown it since submission.
int64_t request_bytes(const Request &r) {
  if (r.fleet) return 64 * (r.b.n_del + r.b.n_ins);  // the launch's batch scratch
  int64_t bytes = 0;
  if (leiden_update_bytes(r.h, r.b.n_del, r.b.n_ins, &bytes) != LEIDEN_OK) return 0;
  return bytes;
}

}  // namespace

struct leiden_server {
  int slots = 0;
  int64_t budget = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<int64_t, Request *> reqs;
  std::unordered_set<const void *> busy;  // handles and fleets being updated
  int64_t in_use = 0;
  int64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  // counters
  int64_t completed = 0;

  // First queued request that fits, into `out`; for a fleet request, also
  // every later queued request of the same fleet on another graph (in queue
  // order, each graph's first only, within the budget), so that they share one
  // launch.  Empty if none fits (called with mu held).
  void admit(std::vector<Request *> &out) {
    out.clear();
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Request *r = *it;
      const void *owner = r->fleet ? (const void *)r->fleet : (const void *)r->h;
      if (busy.count(owner)) continue;
      r->bytes = request_bytes(*r);
      if (in_use > 0 && in_use + r->bytes > budget) continue;
      busy.insert(owner);
      in_use += r->bytes;
      out.push_back(r);
      if (r->fleet) {
        std::unordered_set<int32_t> graphs{r->graph};
        for (auto jt = std::next(it); jt != queue.end() && (int)out.size() < kMaxFleetJobs; ++jt) {
          Request *q = *jt;
          if (q->fleet != r->fleet || graphs.count(q->graph)) {
            if (q->fleet == r->fleet) graphs.insert(q->graph);  // later requests of that graph wait
            continue;
          }
          q->bytes = request_bytes(*q);
          if (in_use + q->bytes > budget) continue;
          graphs.insert(q->graph);
          in_use += q->bytes;
          out.push_back(q);
        }
      }
      for (Request *a : out) queue.erase(std::find(queue.begin(), queue.end(), a));
      return;
    }
  }

  void worker() {
    (void)hipSetDevice(device);
    hipStream_t s;
    const bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    std::vector<Request *> rs;
    std::vector<int32_t> graphs, modes;
    std::vector<leiden_batch> batches;
    std::vector<int32_t *> outs;
    std::vector<double> qs;
    std::vector<leiden_status> sts;
    std::vector<leiden_stats> stats;
    for (;;) {
      rs.clear();  // the previous batch's requests may already be freed by their waiters
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          if (stop) return true;
          admit(rs);
          return !rs.empty();
        });
        if (rs.empty()) break;
      }
      const Clock::time_point t0 = Clock::now();
      Request *r = rs[0];
      if (!ok) {
        for (Request *a : rs) a->st = LEIDEN_EHIP;
      } else if (!r->fleet) {
        r->st = leiden_update(r->h, &r->b, r->mode, r->out, &r->q, &r->stats, nullptr, s);
      } else {
        const size_t k = rs.size();
        graphs.resize(k);
        modes.resize(k);
        batches.resize(k);
        outs.resize(k);
        qs.assign(k, 0.0);
        sts.assign(k, LEIDEN_OK);
        stats.resize(k);
        for (size_t j = 0; j < k; ++j) {
          graphs[j] = rs[j]->graph;
          modes[j] = rs[j]->mode;
          batches[j] = rs[j]->b;
          outs[j] = rs[j]->out;
        }
        const leiden_status st = leiden_fleet_run(r->fleet, (int32_t)k, graphs.data(), modes.data(), batches.data(),
                                                  outs.data(), qs.data(), sts.data(), stats.data(), nullptr, s);
        for (size_t j = 0; j < k; ++j) {
          rs[j]->st = (st == LEIDEN_OK || sts[j] != LEIDEN_OK) ? sts[j] : st;
          rs[j]->q = qs[j];
          rs[j]->stats = stats[j];
        }
      }
      const Clock::time_point t1 = Clock::now();
      {
        std::lock_guard<std::mutex> lk(mu);
        for (Request *a : rs) {
          a->service_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
          a->latency_ms = std::chrono::duration<double, std::milli>(t1 - a->submitted).count();
          a->done = true;
          in_use -= a->bytes;
          ++completed;
        }
        busy.erase(r->fleet ? (const void *)r->fleet : (const void *)r->h);
      }
      cv_work.notify_all();
      cv_done.notify_all();
    }
    if (ok) (void)hipStreamDestroy(s);
  }
};

extern "C" leiden_status leiden_server_create(int32_t slots, int64_t memory_budget, leiden_server **out) {
  if (!out || slots < 1 || slots > 64 || memory_budget < 0) return LEIDEN_EINVAL;
  *out = nullptr;
  leiden_server *sv = new (std::nothrow) leiden_server();
  if (!sv) return LEIDEN_ENOMEM;
  sv->slots = slots;
  sv->budget = memory_budget > 0 ? memory_budget : ((int64_t)1 << 62);
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return LEIDEN_EHIP;
  }
  try {
    for (int k = 0; k < slots; ++k) sv->workers.emplace_back([sv] { sv->worker(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto &t : sv->workers) t.join();
    delete sv;
    return LEIDEN_ENOMEM;
  }
  *out = sv;
  return LEIDEN_OK;
}

extern "C" leiden_status leiden_server_submit(leiden_server *sv, leiden_handle *h, const leiden_batch *batch,
                                              int32_t mode, int32_t *membership_out, int64_t *request_id) {
  if (!sv || !h || !batch || !request_id) return LEIDEN_EINVAL;
  if (mode != LEIDEN_ND && mode != LEIDEN_DS && mode != LEIDEN_DF) return LEIDEN_EINVAL;
  Request *r = new (std::nothrow) Request();
  if (!r) return LEIDEN_ENOMEM;
  r->h = h;
  r->fleet = nullptr;
  r->graph = -1;
  r->b = *batch;
  r->mode = mode;
  r->out = membership_out;
  r->bytes = 0;
  r->submitted = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      delete r;
      return LEIDEN_EINVAL;
    }
    r->id = sv->next_id++;
    sv->reqs[r->id] = r;
    sv->queue.push_back(r);
    *request_id = r->id;
  }
  sv->cv_work.notify_all();
  return LEIDEN_OK;
}

extern "C" leiden_status leiden_server_submit_fleet(leiden_server *sv, leiden_fleet *fleet, int32_t graph,
                                                    const leiden_batch *batch, int32_t mode,
                                                    int32_t *membership_out, int64_t *request_id) {
  if (!sv || !fleet || !request_id || graph < 0 || graph >= leiden_fleet_count(fleet)) return LEIDEN_EINVAL;
  if (mode != 0 && mode != LEIDEN_ND && mode != LEIDEN_DS && mode != LEIDEN_DF) return LEIDEN_EINVAL;
  if (mode != 0 && !batch) return LEIDEN_EINVAL;
  Request *r = new (std::nothrow) Request();
  if (!r) return LEIDEN_ENOMEM;
  r->h = nullptr;
  r->fleet = fleet;
  r->graph = graph;
  if (batch) r->b = *batch;
  else memset(&r->b, 0, sizeof(r->b));
  r->mode = mode;
  r->out = membership_out;
  r->bytes = 0;
  r->submitted = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      delete r;
      return LEIDEN_EINVAL;
    }
    r->id = sv->next_id++;
    sv->reqs[r->id] = r;
    sv->queue.push_back(r);
    *request_id = r->id;
  }
  sv->cv_work.notify_all();
  return LEIDEN_OK;
}

extern "C" leiden_status leiden_server_wait(leiden_server *sv, int64_t request_id, leiden_status *status,
                                            double *q_out, leiden_stats *stats, double *latency_ms,
                                            double *service_ms) {
  if (!sv) return LEIDEN_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(request_id);
  if (it == sv->reqs.end()) return LEIDEN_EINVAL;
  Request *r = it->second;
  sv->cv_done.wait(lk, [&] { return r->done; });
  if (status) *status = r->st;
  if (q_out) *q_out = r->q;
  if (stats) *stats = r->stats;
  if (latency_ms) *latency_ms = r->latency_ms;
  if (service_ms) *service_ms = r->service_ms;
  sv->reqs.erase(it);
  delete r;
  return LEIDEN_OK;
}

extern "C" leiden_status leiden_server_destroy(leiden_server *sv) {
  if (!sv) return LEIDEN_EINVAL;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    // finish everything already submitted
    sv->cv_done.wait(lk, [&] {
      for (auto &kv : sv->reqs)
        if (!kv.second->done) return false;
      return true;
    });
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto &t : sv->workers) t.join();
  for (auto &kv : sv->reqs) delete kv.second;
  delete sv;
  return LEIDEN_OK;
}
