// Host side of the fused many-graph engine (leiden_fleet_* in
// include/leiden.h; kernels in k_fleet.hip).  The graphs of a fleet live in
// per-graph device arenas; one run writes a job table (graph, mode, batch,
// scratch) to device memory and replays a captured HIP graph holding the
// single persistent launch, then reads the per-job results back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <unordered_set>
#include <vector>

#include "fleet_kernels.hpp"
#include "host_alloc.hpp"
#include "kernels.hpp"
#include "leiden.h"

using namespace lk;

namespace {

constexpr int kFleetBlocks = 1024;      // workgroups of the persistent launch
constexpr int kFleetMaxPasses = 16;     // per-pass statistics kept by the kernel

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Sub-buffers of one graph's arena.
struct Carve {
  char *base;
  size_t at = 0;
  template <class T>
  T *take(int64_t count) {
    T *p = (T *)(base + at);
    at += align256((size_t)std::max<int64_t>(count, 1) * sizeof(T));
    return p;
  }
};

size_t arena_bytes(int64_t n, int64_t cap) {
  Carve c{nullptr};
  const int64_t n1 = n + 1;
  for (int b = 0; b < 2; ++b) {
    c.take<int64_t>(n1);
    c.take<int32_t>(cap);
    c.take<float>(cap);
  }
  c.take<int32_t>(n);
  c.take<double>(n);
  c.take<double>(n);
  for (int k = 0; k < 3; ++k) c.take<int32_t>(n);
  c.take<int32_t>(n1);
  for (int k = 0; k < 4; ++k) c.take<double>(n);
  c.take<int32_t>(n);
  c.take<int32_t>(n);
  for (int k = 0; k < 6; ++k) c.take<uint8_t>(n);
  for (int b = 0; b < 2; ++b) {
    c.take<int64_t>(n1);
    c.take<int32_t>(cap);
    c.take<float>(cap);
  }
  c.take<int32_t>(n);
  c.take<int64_t>(n1);
  for (int b = 0; b < 2; ++b) {
    c.take<unsigned long long>(cap);
    c.take<int32_t>(cap);
  }
  c.take<double>(cap);
  return c.at;
}

void carve_graph(FleetGraph &g, char *base, int64_t n, int64_t cap) {
  Carve c{base};
  const int64_t n1 = n + 1;
  for (int b = 0; b < 2; ++b) {
    g.off[b] = c.take<int64_t>(n1);
    g.idx[b] = c.take<int32_t>(cap);
    g.w[b] = c.take<float>(cap);
  }
  g.C = c.take<int32_t>(n);
  g.K = c.take<double>(n);
  g.Sig = c.take<double>(n);
  g.Cl = c.take<int32_t>(n);
  g.CB = c.take<int32_t>(n);
  g.Ctop = c.take<int32_t>(n);
  g.tmpi = c.take<int32_t>(n1);
  g.Kl = c.take<double>(n);
  g.Sl = c.take<double>(n);
  g.S2 = c.take<double>(n);
  g.dense = c.take<double>(n);
  g.tflag = c.take<int32_t>(n);
  g.tlist = c.take<int32_t>(n);
  g.dC = c.take<uint8_t>(n);
  g.dC2 = c.take<uint8_t>(n);
  g.U = c.take<uint8_t>(n);
  g.rng = c.take<uint8_t>(n);
  g.dE = c.take<uint8_t>(n);
  g.dCm = c.take<uint8_t>(n);
  for (int b = 0; b < 2; ++b) {
    g.loff[b] = c.take<int64_t>(n1);
    g.lidx[b] = c.take<int32_t>(cap);
    g.lw[b] = c.take<float>(cap);
  }
  g.rowd = c.take<int32_t>(n);
  g.mcnt = c.take<int64_t>(n1);
  for (int b = 0; b < 2; ++b) {
    g.akey[b] = c.take<unsigned long long>(cap);
    g.apay[b] = c.take<int32_t>(cap);
  }
  g.asum = c.take<double>(cap);
}

struct Fail {
  leiden_status st;
};

}  // namespace

struct leiden_fleet {
  int32_t count = 0;
  leiden_params prm;
  int variant = 0;
  Alloc al;
  std::string err;
  std::vector<FleetGraph> host;     // mirror of the device graph table
  std::vector<DBuf> arena;          // per graph
  DBuf table;                       // FleetGraph[count]
  DBuf jobs;                        // header (njobs, next) + FleetJob[cap]
  int64_t jobs_cap = 0;
  DBuf results;                     // FleetResult[jobs_cap]
  DBuf scratch;                     // batch scratch of a run
  void *pin = nullptr;              // pinned staging (jobs up, results down)
  size_t pin_cap = 0;
  hipStream_t cap_stream = nullptr; // stream used to capture the launch
  hipGraphExec_t exec = nullptr;
  int exec_variant = -1;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipStream_t last = nullptr;
  bool used = false;           // a call has enqueued work (recorded in `order`)
  hipEvent_t order = nullptr;  // end of the latest call's work

  void check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
      err = std::string(what) + ": " + hipGetErrorString(e);
      throw Fail{e == hipErrorOutOfMemory ? LEIDEN_ENOMEM : LEIDEN_EHIP};
    }
  }
  void ensure(DBuf &b, size_t bytes, hipStream_t s) {
    if (b.cap >= bytes) return;
    const size_t want = align256(std::max(bytes, b.cap + b.cap / 4));
    al.put(b.p, b.cap, s);
    b = DBuf{};
    void *p = al.get(want, s);
    if (!p) {
      err = "device allocation of " + std::to_string(want) + " bytes failed";
      throw Fail{LEIDEN_ENOMEM};
    }
    b.p = p;
    b.cap = want;
  }
  void ensure_pin(size_t bytes) {
    if (pin_cap >= bytes) return;
    if (pin) check(hipHostFree(pin), "hipHostFree");
    pin = nullptr;
    pin_cap = 0;
    const size_t want = std::max(bytes, (size_t)1 << 16);
    check(hipHostMalloc(&pin, want, hipHostMallocDefault), "hipHostMalloc");
    pin_cap = want;
  }
  FleetParams params() const {
    FleetParams p;
    memset(&p, 0, sizeof(p));
    p.tau0 = prm.tau0;
    p.tol_drop = prm.tol_drop;
    p.agg_tol = prm.agg_tol;
    p.max_iter = prm.max_iter;
    p.max_passes = std::min(prm.max_passes, kFleetMaxPasses);
    p.refine_variant = prm.refine_variant;
    return p;
  }
  // (Re)builds the captured launch for the current variant and job capacity.
  void capture() {
    if (exec && exec_variant == variant) return;
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    if (!cap_stream) check(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    FleetLaunch L;
    L.graphs = (FleetGraph *)table.p;
    L.njobs = (const int32_t *)jobs.p;
    L.next = (unsigned long long *)((char *)jobs.p + 8);
    L.jobs = (const FleetJob *)((char *)jobs.p + 256);
    L.results = (FleetResult *)results.p;
    L.prm = params();
    hipGraph_t graph;
    check(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const hipError_t le = fleet_launch(L, variant, kFleetBlocks, cap_stream);
    const hipError_t ce = hipStreamEndCapture(cap_stream, &graph);
    check(le, "fleet launch capture");
    check(ce, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check(ie, "hipGraphInstantiate");
    exec_variant = variant;
  }
  void release(hipStream_t s) {
    for (auto &b : arena) {
      al.put(b.p, b.cap, s);
      b = DBuf{};
    }
    for (DBuf *b : {&table, &jobs, &results, &scratch}) {
      al.put(b->p, b->cap, s);
      *b = DBuf{};
    }
  }
};

namespace {

leiden_status guarded(leiden_fleet *f, const std::function<void()> &fn) {
  try {
    fn();
    return LEIDEN_OK;
  } catch (const Fail &e) {
    return e.st;
  } catch (...) {
    f->err = "unexpected error";
    return LEIDEN_EHIP;
  }
}

// A graph's arena for capacity cap (entries); the current CSR (if any) is
// copied into buffer 0 of the new arena and the workspace cleared.
void place_graph(leiden_fleet *f, int32_t k, int64_t cap, hipStream_t s) {
  FleetGraph &g = f->host[k];
  const int64_t n = g.n;
  DBuf nb;
  const size_t bytes = arena_bytes(n, cap);
  void *p = f->al.get(bytes, s);
  if (!p) {
    f->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    throw Fail{LEIDEN_ENOMEM};
  }
  nb.p = p;
  nb.cap = bytes;
  f->check(hipMemsetAsync(p, 0, bytes, s), "hipMemsetAsync");
  FleetGraph ng = g;
  carve_graph(ng, (char *)p, n, cap);
  ng.cap = cap;
  if (f->arena[k].p) {
    // keep the graph and its state
    const int c = g.cur;
    f->check(hipMemcpyAsync(ng.off[0], g.off[c], (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s), "copy");
    if (g.nnz > 0) {
      f->check(hipMemcpyAsync(ng.idx[0], g.idx[c], g.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
      f->check(hipMemcpyAsync(ng.w[0], g.w[c], g.nnz * sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
    }
    if (n > 0) {
      f->check(hipMemcpyAsync(ng.C, g.C, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
      f->check(hipMemcpyAsync(ng.K, g.K, n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
      f->check(hipMemcpyAsync(ng.Sig, g.Sig, n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
    }
    ng.cur = 0;
    f->al.put(f->arena[k].p, f->arena[k].cap, s);
  }
  f->arena[k] = nb;
  g = ng;
}

void upload_table(leiden_fleet *f, hipStream_t s) {
  const size_t bytes = sizeof(FleetGraph) * (size_t)f->count;
  f->ensure_pin(bytes);
  memcpy(f->pin, f->host.data(), bytes);
  f->check(hipMemcpyAsync(f->table.p, f->pin, bytes, hipMemcpyHostToDevice, s), "H2D");
  f->check(hipStreamSynchronize(s), "sync");  // the staging area is reused
}

bool valid_params(const leiden_params *p) {
  return p && p->tau0 >= 0 && p->tol_drop > 0 && p->agg_tol > 0 && p->max_iter >= 1 && p->max_passes >= 1 &&
         p->max_passes <= kFleetMaxPasses && p->refine_variant >= 0 && p->refine_variant <= 2;
}

// A call on a stream other than the previous call's first waits for the
// fleet's latest work, recorded at the end of every call (the previous
// stream itself may no longer exist).
void enter(leiden_fleet *f, hipStream_t s) {
  if (!f->order) f->check(hipEventCreateWithFlags(&f->order, hipEventDisableTiming), "hipEventCreate");
  if (f->used && f->last != s) f->check(hipStreamWaitEvent(s, f->order, 0), "hipStreamWaitEvent");
  f->last = s;
}
void leave(leiden_fleet *f, hipStream_t s) {
  if (f->order && hipEventRecord(f->order, s) == hipSuccess) f->used = true;
  else (void)hipGetLastError();
}
// A fleet call: ordered after the fleet's previous work, guarded.
leiden_status run_fleet(leiden_fleet *f, hipStream_t s, const std::function<void()> &fn) {
  const leiden_status st = guarded(f, [&] {
    enter(f, s);
    fn();
  });
  leave(f, s);
  return st;
}

}  // namespace

extern "C" {

leiden_status leiden_fleet_create(int32_t count, const int64_t *n, const int64_t *nnz,
                                  const int64_t *const *offsets, const int32_t *const *indices,
                                  const float *const *weights, const leiden_params *params,
                                  const leiden_allocator *alloc, void *stream, leiden_fleet **out) {
  if (!out || count < 1 || !n || !nnz || !offsets || !indices || !weights) return LEIDEN_EINVAL;
  if (params && !valid_params(params)) return LEIDEN_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->release)) return LEIDEN_EINVAL;
  for (int32_t k = 0; k < count; ++k)
    if (n[k] < 0 || n[k] > INT32_MAX - 1 || nnz[k] < 0 || !offsets[k] || (nnz[k] > 0 && (!indices[k] || !weights[k])) ||
        (n[k] > 0 && n[k] > (int64_t)1 << 31) || (double)n[k] * (double)n[k] > 1.8e19)
      return LEIDEN_EINVAL;
  *out = nullptr;
  leiden_fleet *f = new (std::nothrow) leiden_fleet();
  if (!f) return LEIDEN_ENOMEM;
  f->count = count;
  if (params) f->prm = *params;
  else leiden_default_params(&f->prm);
  if (alloc) {
    f->al.a = *alloc;
    f->al.custom = true;
  }
  hipStream_t s = (hipStream_t)stream;
  const leiden_status st = run_fleet(f, s, [&] {
    f->host.assign(count, FleetGraph{});
    f->arena.assign(count, DBuf{});
    f->ensure(f->table, sizeof(FleetGraph) * count, s);
    // validation scratch: row sort and checks
    DBuf err, crow, tidx, tw, tmp;
    auto drop = [&] {
      for (DBuf *b : {&err, &crow, &tidx, &tw, &tmp}) {
        f->al.put(b->p, b->cap, s);
        *b = DBuf{};
      }
    };
    try {
      f->ensure(err, 256, s);
      for (int32_t k = 0; k < count; ++k) {
        FleetGraph &g = f->host[k];
        memset(&g, 0, sizeof(g));
        g.n = n[k];
        g.nnz = nnz[k];
        const int64_t cap = nnz[k] + std::max<int64_t>(nnz[k] / 4, 1024);
        place_graph(f, k, cap, s);
        f->check(hipMemcpyAsync(g.off[0], offsets[k], (n[k] + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s),
                 "copy");
        if (nnz[k] > 0) {
          f->check(hipMemcpyAsync(g.idx[0], indices[k], nnz[k] * sizeof(int32_t), hipMemcpyDeviceToDevice, s),
                   "copy");
          f->check(hipMemcpyAsync(g.w[0], weights[k], nnz[k] * sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
        }
        int32_t *e = (int32_t *)err.p;
        f->check(hipMemsetAsync(e, 0, sizeof(int32_t), s), "memset");
        check_offsets(g.off[0], n[k], nnz[k], e, s);
        int32_t he = 0;
        f->check(hipMemcpyAsync(&he, e, sizeof(int32_t), hipMemcpyDeviceToHost, s), "D2H");
        f->check(hipStreamSynchronize(s), "sync");
        if (he) {
          f->err = "graph " + std::to_string(k) + ": offsets are not a valid CSR of nnz entries";
          throw Fail{LEIDEN_EINVAL};
        }
        if (nnz[k] > 0) {
          f->ensure(tidx, nnz[k] * sizeof(int32_t), s);
          f->ensure(tw, nnz[k] * sizeof(float), s);
          size_t tb = seg_sort_i32_f32(nullptr, 0, g.idx[0], (int32_t *)tidx.p, g.w[0], (float *)tw.p, nnz[k], n[k],
                                       g.off[0], s);
          f->ensure(tmp, tb + 16, s);
          seg_sort_i32_f32(tmp.p, tb, g.idx[0], (int32_t *)tidx.p, g.w[0], (float *)tw.p, nnz[k], n[k], g.off[0], s);
          f->check(hipMemcpyAsync(g.idx[0], tidx.p, nnz[k] * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
          f->check(hipMemcpyAsync(g.w[0], tw.p, nnz[k] * sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
        }
        const int64_t nch = ceil_div(std::max<int64_t>(nnz[k], 1), kChunk);
        f->ensure(crow, (nch + 2) * sizeof(int32_t), s);
        chunk_start_rows(g.off[0], n[k], nnz[k], (int32_t *)crow.p, s);
        check_rows_chunked(g.off[0], g.idx[0], g.w[0], n[k], nnz[k], (const int32_t *)crow.p, e, s);
        f->check(hipGetLastError(), "validation kernels");
        f->check(hipMemcpyAsync(&he, e, sizeof(int32_t), hipMemcpyDeviceToHost, s), "D2H");
        f->check(hipStreamSynchronize(s), "sync");
        if (he) {
          f->err = "graph " + std::to_string(k) +
                   ": an id out of range, a non-positive or non-finite weight, or a repeated entry";
          throw Fail{LEIDEN_EINVAL};
        }
      }
    } catch (...) {
      drop();
      throw;
    }
    drop();
    upload_table(f, s);
  });
  if (st != LEIDEN_OK) {
    f->release(s);
    delete f;
    return st;
  }
  *out = f;
  return LEIDEN_OK;
}

leiden_status leiden_fleet_destroy(leiden_fleet *f) {
  if (!f) return LEIDEN_EINVAL;
  // no wait for the device: the releases are ordered after the fleet's last
  // work (on the null stream, which first waits for that work)
  hipStream_t s = nullptr;
  if (f->used && f->order) (void)hipStreamWaitEvent(s, f->order, 0);
  f->release(s);
  if (f->exec) (void)hipGraphExecDestroy(f->exec);
  if (f->cap_stream) (void)hipStreamDestroy(f->cap_stream);
  if (f->t0) (void)hipEventDestroy(f->t0);
  if (f->t1) (void)hipEventDestroy(f->t1);
  if (f->order) (void)hipEventDestroy(f->order);
  if (f->pin) {
    (void)hipStreamSynchronize(s);
    (void)hipHostFree(f->pin);
  }
  (void)hipGetLastError();
  delete f;
  return LEIDEN_OK;
}

leiden_status leiden_fleet_set_variant(leiden_fleet *f, int32_t variant) {
  if (!f || variant < 0 || variant >= kFleetVariants) return LEIDEN_EINVAL;
  f->variant = variant;
  return LEIDEN_OK;
}

leiden_status leiden_fleet_variant_info(int32_t variant, int32_t *waves, int32_t *slots) {
  if (variant < 0 || variant >= kFleetVariants) return LEIDEN_EINVAL;
  if (waves) *waves = kFleetVariant[variant].waves;
  if (slots) *slots = kFleetVariant[variant].slots;
  return LEIDEN_OK;
}

leiden_status leiden_fleet_run(leiden_fleet *f, int32_t count, const int32_t *graphs, const int32_t *modes,
                               const leiden_batch *batches, int32_t *const *membership_out, double *q_out,
                               leiden_status *status_out, leiden_stats *stats, double *ms_out, void *stream) {
  if (!f || count < 0 || (count > 0 && (!graphs || !modes))) return LEIDEN_EINVAL;
  if (count == 0) return LEIDEN_OK;
  {
    std::unordered_set<int32_t> seen;
    for (int32_t k = 0; k < count; ++k) {
      if (graphs[k] < 0 || graphs[k] >= f->count || !seen.insert(graphs[k]).second) return LEIDEN_EINVAL;
      if (modes[k] < 0 || modes[k] > LEIDEN_DF) return LEIDEN_EINVAL;
      if (modes[k] != 0) {
        if (!batches) return LEIDEN_EINVAL;
        const leiden_batch &b = batches[k];
        if (b.n_del < 0 || b.n_ins < 0 || (b.n_del > 0 && (!b.del_u || !b.del_v)) ||
            (b.n_ins > 0 && (!b.ins_u || !b.ins_v || !b.ins_w)))
          return LEIDEN_EINVAL;
      }
    }
  }
  hipStream_t s = (hipStream_t)stream;
  return run_fleet(f, s, [&] {
    // capacity of each graph for its insertions
    bool grown = false;
    for (int32_t k = 0; k < count; ++k) {
      if (modes[k] == 0) continue;
      FleetGraph &g = f->host[graphs[k]];
      const int64_t need = g.nnz + 2 * batches[k].n_ins;
      if (need > g.cap) {
        place_graph(f, graphs[k], need + std::max<int64_t>(need / 4, 1024), s);
        grown = true;
      }
    }
    if (grown) upload_table(f, s);
    // batch scratch, carved per job
    size_t sbytes = 0;
    for (int32_t k = 0; k < count; ++k) {
      const int64_t E = modes[k] == 0 ? 1 : std::max<int64_t>(1, 2 * (batches[k].n_del + batches[k].n_ins));
      sbytes += 2 * align256(E * 8) + 2 * align256(E * 4) + align256(E * 4) + align256((E + 1) * 4);
    }
    f->ensure(f->scratch, sbytes, s);
    if (count > f->jobs_cap) {
      const int64_t cap = std::max<int64_t>(count, f->jobs_cap * 2);
      f->ensure(f->jobs, 256 + sizeof(FleetJob) * cap, s);
      f->ensure(f->results, sizeof(FleetResult) * cap, s);
      f->jobs_cap = cap;
      if (f->exec) {
        (void)hipGraphExecDestroy(f->exec);
        f->exec = nullptr;
      }
    }
    const size_t jbytes = 256 + sizeof(FleetJob) * count;
    const size_t rbytes = sizeof(FleetResult) * count + sizeof(FleetGraph) * f->count;
    f->ensure_pin(std::max(jbytes, rbytes));
    char *hp = (char *)f->pin;
    memset(hp, 0, 256);
    *(int32_t *)hp = count;  // njobs; the next-job counter (hp + 8) starts at 0
    FleetJob *J = (FleetJob *)(hp + 256);
    Carve c{(char *)f->scratch.p};
    for (int32_t k = 0; k < count; ++k) {
      FleetJob &j = J[k];
      memset(&j, 0, sizeof(j));
      j.graph = graphs[k];
      j.mode = modes[k];
      if (modes[k] != 0) {
        const leiden_batch &b = batches[k];
        j.nd = b.n_del;
        j.ni = b.n_ins;
        j.du = b.del_u;
        j.dv = b.del_v;
        j.iu = b.ins_u;
        j.iv = b.ins_v;
        j.iw = b.ins_w;
      }
      const int64_t E = std::max<int64_t>(1, 2 * (j.nd + j.ni));
      j.bkey[0] = c.take<unsigned long long>(E);
      j.bkey[1] = c.take<unsigned long long>(E);
      j.bpay[0] = c.take<int32_t>(E);
      j.bpay[1] = c.take<int32_t>(E);
      j.bw = c.take<float>(E);
      j.bpre = c.take<int32_t>(E + 1);
      j.out = membership_out ? membership_out[k] : nullptr;
    }
    f->check(hipMemcpyAsync(f->jobs.p, hp, jbytes, hipMemcpyHostToDevice, s), "H2D jobs");
    f->capture();
    if (!f->t0) {
      f->check(hipEventCreate(&f->t0), "hipEventCreate");
      f->check(hipEventCreate(&f->t1), "hipEventCreate");
    }
    f->check(hipEventRecord(f->t0, s), "hipEventRecord");
    f->check(hipGraphLaunch(f->exec, s), "hipGraphLaunch");
    f->check(hipEventRecord(f->t1, s), "hipEventRecord");
    f->check(hipMemcpyAsync(hp, f->results.p, sizeof(FleetResult) * count, hipMemcpyDeviceToHost, s), "D2H");
    char *tp = hp + sizeof(FleetResult) * count;
    f->check(hipMemcpyAsync(tp, f->table.p, sizeof(FleetGraph) * f->count, hipMemcpyDeviceToHost, s), "D2H");
    f->check(hipStreamSynchronize(s), "sync");
    float ms = 0.f;
    f->check(hipEventElapsedTime(&ms, f->t0, f->t1), "hipEventElapsedTime");
    if (ms_out) *ms_out = ms;
    memcpy(f->host.data(), tp, sizeof(FleetGraph) * f->count);
    const FleetResult *R = (const FleetResult *)hp;
    leiden_status first = LEIDEN_OK;
    for (int32_t k = 0; k < count; ++k) {
      const FleetResult &r = R[k];
      leiden_status st = r.status == 0 ? LEIDEN_OK : r.status == 3 ? LEIDEN_ESTATE : LEIDEN_EINVAL;
      if (status_out) status_out[k] = st;
      if (q_out) q_out[k] = r.q;
      if (stats) {
        leiden_stats &o = stats[k];
        memset(&o, 0, sizeof(o));
        o.passes = r.passes;
        for (int p = 0; p < std::min(r.passes, kFleetMaxPasses); ++p) {
          o.move_iters[p] = r.move_iters[p];
          o.refine_rounds[p] = 1;
          o.level_vertices[p] = r.level_vertices[p];
          o.communities[p] = r.communities[p];
        }
        o.affected = r.affected;
        o.changed = r.changed;
        o.moves_pass0 = r.moves_pass0;
        o.ms_total = ms;
      }
      if (first == LEIDEN_OK && st != LEIDEN_OK) {
        first = st;
        f->err = "job " + std::to_string(k) + " (graph " + std::to_string(graphs[k]) + "): " +
                 (st == LEIDEN_ESTATE ? std::string("no community state (run a static job first)")
                                      : "invalid batch (error bits " + std::to_string(r.err) + ")");
      }
    }
    if (first != LEIDEN_OK) throw Fail{first};
  });
}

leiden_status leiden_fleet_get_graph(leiden_fleet *f, int32_t graph, int64_t *offsets, int32_t *indices,
                                     float *weights, int64_t *nnz, void *stream) {
  if (!f || graph < 0 || graph >= f->count) return LEIDEN_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  return run_fleet(f, s, [&] {
    const FleetGraph &g = f->host[graph];
    if (nnz) *nnz = g.nnz;
    const int c = g.cur;
    if (offsets) f->check(hipMemcpyAsync(offsets, g.off[c], (g.n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s), "copy");
    if (indices && g.nnz > 0)
      f->check(hipMemcpyAsync(indices, g.idx[c], g.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
    if (weights && g.nnz > 0)
      f->check(hipMemcpyAsync(weights, g.w[c], g.nnz * sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
    f->check(hipStreamSynchronize(s), "sync");
  });
}

leiden_status leiden_fleet_get_state(leiden_fleet *f, int32_t graph, int32_t *membership, double *K, double *Sigma,
                                     double *m2, void *stream) {
  if (!f || graph < 0 || graph >= f->count) return LEIDEN_EINVAL;
  if (!f->host[graph].has_state) return LEIDEN_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  return run_fleet(f, s, [&] {
    const FleetGraph &g = f->host[graph];
    if (membership && g.n > 0)
      f->check(hipMemcpyAsync(membership, g.C, g.n * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
    if (K && g.n > 0) f->check(hipMemcpyAsync(K, g.K, g.n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
    if (Sigma && g.n > 0)
      f->check(hipMemcpyAsync(Sigma, g.Sig, g.n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
    if (m2) *m2 = g.M2;
    f->check(hipStreamSynchronize(s), "sync");
  });
}

int32_t leiden_fleet_count(const leiden_fleet *f) { return f ? f->count : -1; }

const char *leiden_fleet_last_error(const leiden_fleet *f) { return f ? f->err.c_str() : ""; }

}  // extern "C"
