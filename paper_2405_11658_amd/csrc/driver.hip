// Host driver and C ABI of the dynamic Leiden library (see include/leiden.h).
//
// The pass loop follows Alg. "leiden": local-moving (k_move.hip), subset
// renumbering, breaking of changed communities and refinement (k_refine.hip),
// then - unless a later pass converged in one iteration - dense renumbering,
// dendrogram lookup and aggregation (k_aggregate.hip) into the next level.
// Front-ends (Alg. "naiveDynamic", "deltaScreening", "dynamicFrontier") and
// "updateWeights" run on the device (k_batch.hip).  Data-dependent loop
// control reads one scalar per iteration back to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "host_alloc.hpp"
#include "kernels.hpp"
#include "leiden.h"

using namespace lk;

namespace {



enum Slot {
  // level arrays (size n of level 0)
  L_C, L_K, L_S, L_S2, L_dC, L_dC2, L_U, L_rng, L_CB, L_Ctop, L_prop, L_from, L_gp, L_gi, L_Sz,
  L_rep, L_lists, L_region, L_tiles, L_flags, L_map, L_scnt, L_vbs, L_soff, L_sfill, L_CP,
  // level graphs (ping-pong), and the first aggregated level kept for the
  // modularity of the result (with its FP64 weights and the level-0 map)
  G0_off, G0_idx, G0_w, G0_crow, G1_off, G1_idx, G1_w, G1_crow, L1_off, L1_idx, L1_w, L1_crow, L1_w64,
  L1_map, L1_lab, A_v64, L_fa, L_map2,
  // aggregation
  A_vk, A_vk2, A_vv, A_vv2, A_eoff, A_pos, A_seg, A_hpos, A_gkey, A_gval, A_ukey, A_uval, A_lflag,
  A_lidx, A_lc, A_lsb, A_lse, A_ltn, A_tseg, A_hc, A_tin, A_rowlen,
  // hubs
  H_v, H_cnt, H_ch, H_tab, H_sg, H_chub, H_shub, H_tk, H_tv, H_own, H_pg, H_pc, H_soff,
  H_fill, H_bnd, H_flag, L_act, W_keys, W_vals, W_list,
  // primitives
  T_tmp,
  // batch
  B_keys, B_vals, B_skeys, B_svals, B_ew, B_bstart, B_bcnt, B_dcnt, B_icnt, B_isdel, B_delpre,
  B_newdeg,
  // marking
  M_dE, M_dCm, M_k2, M_k2s, M_v2, M_v2s, M_list,
  // modularity
  Q_S, Q_crow,
  NSLOT
};

struct DevScal {
  double gain;
  unsigned long long moves;
  int32_t accepted;
  int32_t err;
  unsigned long long refined;
  double acc[4];
  double m2delta;
  double tiles_total;
  int32_t list_count;
  int32_t pad;
  unsigned long long nz;
  unsigned long long hub_scanned;
  unsigned long long sweep_work[4];  // [vertices, edges] of the move sweeps, then of the refine sweeps
  unsigned long long anext;
};

struct Workspace {
  DBuf ws[NSLOT];
  DBuf scal;
  Alloc al;
  void *hpin = nullptr;
  std::string err;
  std::vector<hipEvent_t> events;
  std::vector<hipEvent_t> kevents;
  // releases every buffer, ordered after the work enqueued on `s`
  void release(hipStream_t s) {
    for (auto &b : ws) {
      al.put(b.p, b.cap, s);
      b = DBuf{};
    }
    al.put(scal.p, scal.cap, s);
    scal = DBuf{};
  }
  // device bytes held
  size_t held() const {
    size_t t = scal.cap;
    for (const auto &b : ws) t += b.cap;
    return t;
  }
  ~Workspace() {
    pin_pool().give(hpin);
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto e : kevents) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct leiden_handle {
  int64_t n = 0;
  int64_t nnz = 0;
  leiden_params prm;
  DBuf g_off, g_idx, g_w, g_crow;
  DBuf t_off, t_idx, t_w;
  DBuf C, K, Sig;
  double M2 = 0.0;
  bool has_state = false;
  Workspace w;
  hipStream_t last = nullptr;  // stream of the latest call
  bool used = false;           // a call has enqueued work on `last`
  hipEvent_t order = nullptr;  // orders a call on another stream after `last`
  void release(hipStream_t s) {
    for (DBuf *b : {&g_off, &g_idx, &g_w, &g_crow, &t_off, &t_idx, &t_w, &C, &K, &Sig}) {
      w.al.put(b->p, b->cap, s);
      *b = DBuf{};
    }
    w.release(s);
  }
  ~leiden_handle() {
    if (order) (void)hipEventDestroy(order);
  }
};

namespace {

struct Fail {
  leiden_status st;
};

constexpr int kMaxSlices = 256;
// hub slices of the asynchronous mode: with 1/64 of the hubs moving at a time a
// DF update on RMAT-22 stays within about 7e-4 of the serial sweep's
// modularity when both start from the same state (1.0e-3 with 32 slices,
// 1.6e-3 with 16), for ~12 % more time than 32 slices
constexpr int kDefaultHubSlices = 64;
// a stalled level keeping more than this fraction of its vertices as
// communities ends the pass loop (the paper's default aggregation tolerance)
constexpr double kStallKeep = 0.8;
// Default hub threshold of the asynchronous mode: a vertex whose neighbour
// table does not fit a wavefront's 512-slot LDS table (degree > 256) moves in
// the multi-workgroup hub slices.
constexpr int kDefaultHubDeg = 256;
// Levels of at least this many vertices (C alone 64 MB, 16x an XCD's L2)
// read neighbour communities and community totals through the caches in the
// asynchronous sweeps.
constexpr int64_t kCachedLevel = 16 << 20;
constexpr int kDefaultAsyncWaves = 4096;  // wavefronts of the asynchronous sweeps, at most
constexpr int kMaxAsyncWaves = 65536;
constexpr int64_t kVertsPerWave = 1024;  // level-0 vertices with edges per sweeping wavefront, at least
constexpr int64_t kVertsPerWaveUpper = 256;  // the same for the aggregated levels
constexpr int kStallIters = 3;  // see the iteration loop of run_core

// Wavefronts of an asynchronous sweep over a level with n vertices that have
// edges: at most `cap`, and few enough that the vertices in flight stay a
// small fraction of the level (with much of a level in flight the sweep
// degenerates into a synchronous update that oscillates and loses modularity).
// The first level decides most of the final modularity; the aggregated ones
// tolerate four times as many vertices in flight.
// Larger per-wavefront LDS tables when the level's average degree is high.
bool wide_tables(int64_t nnz, int64_t with_edges) { return with_edges > 0 && nnz / with_edges > 128; }

int level_waves(const leiden_params &p, int cap, int64_t n, int pass) {
  const int64_t vpw0 = p.verts_per_wave > 0 ? p.verts_per_wave : kVertsPerWave;
  const int64_t vpw1 = p.verts_per_wave_upper > 0 ? p.verts_per_wave_upper : kVertsPerWaveUpper;
  int64_t w = n / (pass == 0 ? vpw0 : vpw1);
  w = std::max<int64_t>(1, std::min<int64_t>(w, cap));
  return (int)(w < 4 ? w : w / 4 * 4);  // whole 4-wavefront workgroups, never above cap
}

struct KProf;

// Call context: workspace + stream; helpers throw Fail, caught at the ABI.
struct Ctx {
  Workspace *w;
  hipStream_t s;
  KProf *kp = nullptr;  // kernel timing, when requested

  void check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
      w->err = std::string(what) + ": " + hipGetErrorString(e);
      throw Fail{e == hipErrorOutOfMemory ? LEIDEN_ENOMEM : LEIDEN_EHIP};
    }
  }
  void launched(const char *what) { check(hipGetLastError(), what); }
  void invalid(const std::string &msg) {
    w->err = msg;
    throw Fail{LEIDEN_EINVAL};
  }

  void ensure(DBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return;
    // grow by at least a quarter, so that sizes creeping up from call to call
    // (a graph growing by batches) do not reallocate every time
    size_t want = std::max(bytes, (size_t)(b.cap + b.cap / 4));
    want = (want + 255) & ~(size_t)255;
    // the old contents are not kept; its release is ordered after the work
    // already enqueued on the stream
    w->al.put(b.p, b.cap, s);
    b.p = nullptr;
    b.cap = 0;
    void *p = w->al.get(want, s);
    if (!p) {
      w->err = "device allocation of " + std::to_string(want) + " bytes failed";
      throw Fail{LEIDEN_ENOMEM};
    }
    b.p = p;
    b.cap = want;
  }
  template <class T>
  T *get(Slot k, int64_t count) {
    ensure(w->ws[k], (size_t)std::max<int64_t>(count, 1) * sizeof(T));
    return (T *)w->ws[k].p;
  }
  DevScal *scal() {
    if (!w->scal.p) {
      ensure(w->scal, sizeof(DevScal));
      check(hipMemsetAsync(w->scal.p, 0, sizeof(DevScal), s), "memset");
    }
    return (DevScal *)w->scal.p;
  }
  void *pin() {
    if (!w->hpin) {
      w->hpin = pin_pool().take();
      if (!w->hpin) {
        w->err = "pinned host allocation failed";
        throw Fail{LEIDEN_ENOMEM};
      }
    }
    return w->hpin;
  }
  template <class T>
  void zero(T *p, int64_t count) {
    if (count > 0) check(hipMemsetAsync(p, 0, (size_t)count * sizeof(T), s), "hipMemsetAsync");
  }
  template <class T>
  T read(const T *dev) {
    T *hp = (T *)pin();
    check(hipMemcpyAsync(hp, dev, sizeof(T), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    return *hp;
  }
  template <class T>
  void copy(T *dst, const T *src, int64_t count) {
    if (count > 0)
      check(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync D2D");
  }
  void *tmp(size_t bytes) { return get<unsigned char>(T_tmp, (int64_t)bytes); }
};

// Phase timing with events on the call's stream.
enum Cat { CAT_APPLY, CAT_MARK, CAT_MOVE, CAT_REFINE, CAT_AGG, CAT_OTHER, NCAT };
struct Timer {
  Ctx &x;
  bool on;
  struct Mark {
    hipEvent_t e;
    int cat;
    int pass;
  };
  std::vector<Mark> marks;
  size_t used = 0;
  int pass = -1;  // pass the following intervals belong to (-1: none)
  Timer(Ctx &c, bool enabled) : x(c), on(enabled) {}
  void mark(int cat) {  // the interval ending here is attributed to `cat`
    if (!on) return;
    if (used == x.w->events.size()) {
      hipEvent_t e;
      x.check(hipEventCreate(&e), "hipEventCreate");
      x.w->events.push_back(e);
    }
    hipEvent_t e = x.w->events[used++];
    x.check(hipEventRecord(e, x.s), "hipEventRecord");
    marks.push_back({e, cat, pass});
  }
  void finish(leiden_stats *st) {
    if (!on || !st || marks.size() < 2) return;
    x.check(hipEventSynchronize(marks.back().e), "hipEventSynchronize");
    double t[NCAT] = {0};
    for (size_t k = 1; k < marks.size(); ++k) {
      float ms = 0.f;
      x.check(hipEventElapsedTime(&ms, marks[k - 1].e, marks[k].e), "hipEventElapsedTime");
      t[marks[k].cat] += ms;
      const int ps = marks[k].pass;
      if (ps >= 0 && ps < LEIDEN_MAX_PASSES) {
        if (marks[k].cat == CAT_MOVE) st->pass_move_ms[ps] += ms;
        if (marks[k].cat == CAT_REFINE) st->pass_refine_ms[ps] += ms;
        if (marks[k].cat == CAT_AGG) st->pass_agg_ms[ps] += ms;
      }
    }
    float tot = 0.f;
    x.check(hipEventElapsedTime(&tot, marks.front().e, marks.back().e), "hipEventElapsedTime");
    st->ms_total = tot;
    st->ms_apply = t[CAT_APPLY];
    st->ms_mark = t[CAT_MARK];
    st->ms_move = t[CAT_MOVE];
    st->ms_refine = t[CAT_REFINE];
    st->ms_aggregate = t[CAT_AGG];
    st->ms_other = t[CAT_OTHER];
  }
};

// Kernel-level timing (leiden_params.profile): HIP events on the call's
// stream immediately before and after each launch of the timed kernels.
struct KProf {
  struct Rec {
    hipEvent_t a, b;
    int id;
    int64_t entries, vertices;
  };
  Ctx &x;
  bool on;
  std::vector<Rec> recs;
  size_t used = 0;
  KProf(Ctx &c, bool enabled) : x(c), on(enabled) {}
  hipEvent_t ev() {
    if (used == x.w->kevents.size()) {
      hipEvent_t e;
      x.check(hipEventCreate(&e), "hipEventCreate");
      x.w->kevents.push_back(e);
    }
    hipEvent_t e = x.w->kevents[used++];
    x.check(hipEventRecord(e, x.s), "hipEventRecord");
    return e;
  }
  hipEvent_t begin() { return on ? ev() : nullptr; }
  void end(hipEvent_t a, int id, int64_t entries, int64_t vertices) {
    if (!on) return;
    recs.push_back({a, ev(), id, entries, vertices});
  }
  void finish(leiden_stats *st, const unsigned long long *hub_scanned, const unsigned long long *sweep_work) {
    if (!on || !st || recs.empty()) return;
    x.check(hipEventSynchronize(recs.back().b), "hipEventSynchronize");
    for (const Rec &r : recs) {
      float ms = 0.f;
      x.check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
      st->prof_launches[r.id] += 1;
      st->prof_ms[r.id] += ms;
      st->prof_entries[r.id] += r.entries;
      st->prof_vertices[r.id] += r.vertices;
    }
    if (hub_scanned) st->prof_entries[LEIDEN_PROF_HUB_GATHER] = (int64_t)x.read(hub_scanned);
    if (sweep_work) {
      st->prof_vertices[LEIDEN_PROF_MOVE_SWEEP] = (int64_t)x.read(&sweep_work[0]);
      st->prof_entries[LEIDEN_PROF_MOVE_SWEEP] = (int64_t)x.read(&sweep_work[1]);
      st->prof_vertices[LEIDEN_PROF_REFINE_SWEEP] = (int64_t)x.read(&sweep_work[2]);
      st->prof_entries[LEIDEN_PROF_REFINE_SWEEP] = (int64_t)x.read(&sweep_work[3]);
    }
  }
};

struct Level {
  int64_t n, nnz;
  const int64_t *off;
  const int32_t *idx;
  const float *w;
  const int32_t *crow;
};

int64_t pow2_at_least(int64_t x) {
  int64_t c = 2;
  while (c < x) c <<= 1;
  return c;
}

// Eq. 1 for a level graph and membership (labels < n).
double modularity_dev(Ctx &x, const Level &g, const int32_t *C) {
  DevScal *sc = x.scal();
  double *S = x.get<double>(Q_S, g.n);
  x.zero(S, g.n);
  x.zero(sc->acc, 4);
  hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
  modularity_edges(g.off, g.idx, g.w, g.crow, g.n, g.nnz, C, sc->acc, S, x.s);
  if (x.kp) x.kp->end(t0, LEIDEN_PROF_MOD_SCAN, g.nnz, g.n);
  modularity_comm(S, g.n, sc->acc, x.s);
  x.launched("modularity");
  double acc[4];
  x.check(hipMemcpyAsync(x.pin(), sc->acc, sizeof(acc), hipMemcpyDeviceToHost, x.s), "D2H");
  x.check(hipStreamSynchronize(x.s), "sync");
  memcpy(acc, x.pin(), sizeof(acc));
  const double M2 = acc[1];
  if (!(M2 > 0.0)) return 0.0;
  modularity_comm_sq(S, g.n, M2, sc->acc, x.s);
  x.launched("modularity_sq");
  const double sq = x.read(&sc->acc[2]);
  return acc[0] / M2 - sq;
}

// Eq. 1 when Sigma (by label, n entries) and 2m are known: one edge pass for
// the internal weight, one pass over Sigma.
double modularity_known(Ctx &x, const Level &g, const int32_t *C, const double *Sig, double M2) {
  if (!(M2 > 0.0)) return 0.0;
  DevScal *sc = x.scal();
  x.zero(sc->acc, 4);
  hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
  modularity_intra(g.off, g.idx, g.w, g.crow, g.nnz, C, sc->acc, x.s);
  if (x.kp) x.kp->end(t0, LEIDEN_PROF_MOD_SCAN, g.nnz, g.n);
  modularity_comm_sq(Sig, g.n, M2, sc->acc, x.s);
  x.launched("modularity");
  double acc[4];
  x.check(hipMemcpyAsync(x.pin(), sc->acc, sizeof(acc), hipMemcpyDeviceToHost, x.s), "D2H");
  x.check(hipStreamSynchronize(x.s), "sync");
  memcpy(acc, x.pin(), sizeof(acc));
  return acc[0] / M2 - acc[2];
}

// Per-level slice and degree-bucket layout: host copy of the region starts
// (index s*kNB+b), the device copy, and the vertex-by-slice grouping.
struct Layout {
  int S;
  std::vector<int64_t> region;  // S*kNB+1
  std::vector<int64_t> soff;    // S+1
  int64_t nhub;
};

Layout level_layout(Ctx &x, const Level &g, int S, int64_t hubdeg, int32_t *region_dev, int32_t *counts_tmp,
                    int32_t *scnt,
                    int32_t *soff_dev, int32_t *sfill, int32_t *vbyslice) {
  Layout L;
  L.S = S;
  const int nb = S * kNB;
  x.zero(counts_tmp, nb);
  x.zero(scnt, S);
  slice_hist(g.off, g.n, S, hubdeg, counts_tmp, scnt, x.s);
  x.launched("slice_hist");
  int32_t *hp = (int32_t *)x.pin();
  x.check(hipMemcpyAsync(hp, counts_tmp, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, x.s), "D2H");
  x.check(hipMemcpyAsync(hp + nb, scnt, sizeof(int32_t) * S, hipMemcpyDeviceToHost, x.s), "D2H");
  x.check(hipStreamSynchronize(x.s), "sync");
  L.region.assign(nb + 1, 0);
  L.soff.assign(S + 1, 0);
  for (int k = 0; k < nb; ++k) L.region[k + 1] = L.region[k] + hp[k];
  for (int k = 0; k < S; ++k) L.soff[k + 1] = L.soff[k] + hp[nb + k];
  L.nhub = 0;
  for (int s = 0; s < S; ++s) L.nhub += hp[s * kNB + kNB - 1];
  int32_t *up = hp + nb + S;
  for (int k = 0; k <= nb; ++k) up[k] = (int32_t)L.region[k];
  for (int k = 0; k <= S; ++k) up[nb + 1 + k] = (int32_t)L.soff[k];
  x.check(hipMemcpyAsync(region_dev, up, sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, x.s), "H2D");
  x.check(hipMemcpyAsync(soff_dev, up + nb + 1, sizeof(int32_t) * (S + 1), hipMemcpyHostToDevice, x.s), "H2D");
  x.zero(sfill, S);
  slice_scatter(g.n, S, soff_dev, sfill, vbyslice, x.s);
  x.launched("slice_scatter");
  x.check(hipStreamSynchronize(x.s), "sync");  // the pinned staging area is reused
  return L;
}


// exclusive scans through the shared temp buffer
void scan_i32(Ctx &x, const int32_t *in, int32_t *out, int64_t n) {
  size_t tb = scan_excl_i32(nullptr, 0, in, out, n, x.s);
  scan_excl_i32(x.tmp(tb), tb, in, out, n, x.s);
  x.launched("scan_i32");
}
void scan_i64(Ctx &x, const int64_t *in, int64_t *out, int64_t n) {
  size_t tb = scan_excl_i64(nullptr, 0, in, out, n, x.s);
  scan_excl_i64(x.tmp(tb), tb, in, out, n, x.s);
  x.launched("scan_i64");
}
void scan_i32_i64(Ctx &x, const int32_t *in, int64_t *out, int64_t n) {
  size_t tb = scan_excl_i32_to_i64(nullptr, 0, in, out, n, x.s);
  scan_excl_i32_to_i64(x.tmp(tb), tb, in, out, n, x.s);
  x.launched("scan_i32_i64");
}

// Multi-workgroup hub plan of a level (local-moving of the largest degree
// bucket): hub list per slice, chunk / table / segment layout, tables
// cleared, and per-slice bounds on the host.
struct HubHost {
  HubPlan p;
  int64_t nhub = 0;
  std::vector<int64_t> hs, qs, gs;  // per-slice starts (S+1): hubs, chunks, segments
};

HubHost hub_plan(Ctx &x, const Level &g, int S, int64_t hubdeg, const Layout &B) {
  HubHost H;
  memset(&H.p, 0, sizeof(H.p));
  H.hs.assign(S + 1, 0);
  H.qs.assign(S + 1, 0);
  H.gs.assign(S + 1, 0);
  for (int s = 0; s < S; ++s)
    H.hs[s + 1] = H.hs[s] + (B.region[s * kNB + kNB] - B.region[s * kNB + kNB - 1]);
  H.nhub = H.hs[S];
  if (H.nhub == 0) return H;
  const int64_t nh = H.nhub;
  int32_t *hsoff = x.get<int32_t>(H_soff, S + 1);
  int32_t *hfill = x.get<int32_t>(H_fill, S);
  int32_t *up = (int32_t *)x.pin();
  for (int s = 0; s <= S; ++s) up[s] = (int32_t)H.hs[s];
  x.check(hipMemcpyAsync(hsoff, up, sizeof(int32_t) * (S + 1), hipMemcpyHostToDevice, x.s), "H2D");
  x.zero(hfill, S);
  H.p.hubv = x.get<int32_t>(H_v, nh);
  hub_find(g.off, g.n, S, hubdeg, hsoff, hfill, H.p.hubv, x.s);
  int64_t *cnt = x.get<int64_t>(H_cnt, 3 * (nh + 1));
  hub_sizes(g.off, H.p.hubv, nh, cnt, cnt + (nh + 1), cnt + 2 * (nh + 1), x.s);
  x.launched("hub plan");
  H.p.hch = x.get<int64_t>(H_ch, nh + 1);
  H.p.htab = x.get<int64_t>(H_tab, nh + 1);
  H.p.hsg = x.get<int64_t>(H_sg, nh + 1);
  H.p.hcap = cnt + (nh + 1);
  scan_i64(x, cnt, H.p.hch, nh + 1);
  scan_i64(x, cnt + (nh + 1), H.p.htab, nh + 1);
  scan_i64(x, cnt + 2 * (nh + 1), H.p.hsg, nh + 1);
  int64_t *bnd = x.get<int64_t>(H_bnd, 3 * (S + 1));
  gather_bounds(H.p.hch, hsoff, S + 1, bnd, x.s);
  gather_bounds(H.p.hsg, hsoff, S + 1, bnd + (S + 1), x.s);
  gather_bounds(H.p.htab, hsoff, S + 1, bnd + 2 * (S + 1), x.s);
  hub_rel(H.p.htab, nh, hsoff, S, bnd + 2 * (S + 1), x.s);
  x.launched("hub bounds");
  int64_t *hb = (int64_t *)((char *)x.pin() + 8192);
  x.check(hipMemcpyAsync(hb, bnd, sizeof(int64_t) * 3 * (S + 1), hipMemcpyDeviceToHost, x.s), "D2H");
  x.check(hipStreamSynchronize(x.s), "sync");
  int64_t ntab = 0;  // the largest slice's tables
  for (int s = 0; s <= S; ++s) {
    H.qs[s] = hb[s];
    H.gs[s] = hb[S + 1 + s];
    if (s < S) ntab = std::max(ntab, hb[2 * (S + 1) + s + 1] - hb[2 * (S + 1) + s]);
  }
  H.p.chub = x.get<int32_t>(H_chub, H.qs[S]);
  H.p.shub = x.get<int32_t>(H_shub, H.gs[S]);
  hub_expand(H.p, nh, x.s);
  H.p.keys = x.get<int>(H_tk, ntab);
  H.p.vals = x.get<double>(H_tv, ntab);
  fill_i32(H.p.keys, -1, ntab, x.s);  // empty slots
  x.zero(H.p.vals, ntab);
  H.p.own = x.get<double>(H_own, nh);
  x.zero(H.p.own, nh);
  H.p.flag = x.get<int32_t>(H_flag, nh);
  x.zero(H.p.flag, nh);
  H.p.pg = x.get<double>(H_pg, H.gs[S]);
  H.p.pc = x.get<int32_t>(H_pc, H.gs[S]);
  x.launched("hub tables");
  return H;
}

// Dense relabel of C[0..n) (labels < bound) in ascending order; returns count.
int64_t renumber_dense(Ctx &x, int32_t *C, int64_t n, int64_t bound) {
  int32_t *flags = x.get<int32_t>(L_flags, bound + 1);
  int32_t *map = x.get<int32_t>(L_map, bound + 1);
  x.zero(flags, bound + 1);
  mark_used(C, n, flags, x.s);
  scan_i32(x, flags, map, bound + 1);
  gather_map(C, map, n, x.s);
  x.launched("renumber");
  return (int64_t)x.read(&map[bound]);
}

// renumber_dense with the labels that have a member with edges first (in
// ascending order, *na of them), then the others: the aggregated level's
// vertices without edges (the level-0 vertices without edges, each alone)
// are then the last ones and can be left out of it.
int64_t renumber_active_first(Ctx &x, int32_t *C, int64_t n, const int64_t *off, int64_t *na) {
  int32_t *used = x.get<int32_t>(L_flags, n + 1);
  int32_t *act = x.get<int32_t>(L_fa, n + 1);
  int32_t *pa = x.get<int32_t>(L_map, n + 1);
  int32_t *pi = x.get<int32_t>(L_map2, n + 1);
  x.zero(used, n + 1);
  x.zero(act, n + 1);
  mark_used_active(C, off, n, used, act, x.s);
  flags_inactive(used, act, n, x.s);
  scan_i32(x, act, pa, n + 1);
  scan_i32(x, used, pi, n + 1);
  const int64_t nact = (int64_t)x.read(&pa[n]);
  const int64_t nin = (int64_t)x.read(&pi[n]);
  active_first_map(act, pa, pi, nact, n, used, x.s);
  gather_map(C, used, n, x.s);
  x.launched("renumber");
  *na = nact;
  return nact + nin;
}

// Alg. "leidenAggregate": level g with dense labels C (< ncomm) -> out level.
// Entries grouped by the community of their source (vertices in community
// order), each community's group sorted by neighbour community and summed:
// rows come out sorted by id, with FP64 sums rounded to float32.  outbuf 0
// and 1 are the ping-pong level graphs, 2 the kept first level; with w64 the
// rows' FP64 sums are kept too (*w64, one per stored entry).  Neighbour
// labels are below nkey (ncomm when 0; fewer when the labels of communities
// without edges come last, since no entry points to those).
Level aggregate_level(Ctx &x, const Level &g, const int32_t *C, int64_t ncomm, int outbuf, double *Kout,
                      double **w64 = nullptr, int64_t nkey = 0) {
  AggArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g.n;
  a.nnz = g.nnz;
  a.ncomm = ncomm;
  a.off = g.off;
  a.idx = g.idx;
  a.w = g.w;
  a.C = C;
  const Slot so = outbuf == 2 ? L1_off : outbuf ? G1_off : G0_off;
  const Slot si = outbuf == 2 ? L1_idx : outbuf ? G1_idx : G0_idx;
  const Slot sw = outbuf == 2 ? L1_w : outbuf ? G1_w : G0_w;
  const Slot sc = outbuf == 2 ? L1_crow : outbuf ? G1_crow : G0_crow;
  double *v64 = (w64 && g.nnz > 0) ? x.get<double>(A_v64, g.nnz) : nullptr;
  int64_t *out_off = x.get<int64_t>(so, ncomm + 1);
  int32_t *rowlen = x.get<int32_t>(A_rowlen, ncomm + 1);
  x.zero(rowlen, ncomm + 1);
  if (Kout) x.zero(Kout, ncomm);
  const int cb = key_bits((unsigned long long)std::max<int64_t>(ncomm - 1, 0));
  int64_t nl = 0;
  int64_t *seg = nullptr;
  int32_t *lc = nullptr;
  int64_t *lsb = nullptr;
  int32_t *tseg = nullptr;  // large segments' input tiles: owning segment, first tile per segment
  int64_t *ltn = nullptr;
  int64_t ntl = 0;
  uint32_t *ukey = nullptr, *lkey = nullptr;
  float *uval = nullptr, *lval = nullptr;
  if (g.nnz > 0) {
    const int64_t n = g.n, nnz = g.nnz;
    hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
    // 1. vertices in community order
    uint32_t *vk = x.get<uint32_t>(A_vk, n), *vk2 = x.get<uint32_t>(A_vk2, n);
    int32_t *vv = x.get<int32_t>(A_vv, n), *vv2 = x.get<int32_t>(A_vv2, n);
    agg_vkeys(n, C, vk, vv, x.s);
    const RsSeg vseg = rs_plain(n);
    if (rsort<uint32_t, int32_t>(vk, vv, vk2, vv2, vseg, cb, x.tmp(rs_tmp_bytes(vseg.ntiles)), x.s)) {
      std::swap(vk, vk2);
      std::swap(vv, vv2);
    }
    // 2. places of the vertices' entries and the communities' segments
    int64_t *eoff = x.get<int64_t>(A_eoff, n + 1);
    int32_t *pos = x.get<int32_t>(A_pos, n);
    agg_vdeg(n, g.off, vv, eoff, pos, x.s);
    scan_i64(x, eoff, eoff, n + 1);
    seg = x.get<int64_t>(A_seg, ncomm + 1);
    int64_t *hpos = x.get<int64_t>(A_hpos, ncomm);
    x.zero(seg, ncomm + 1);
    agg_cdeg(n, vk, eoff, hpos, seg, x.s);
    scan_i64(x, seg, seg, ncomm + 1);
    // 3. grouped entries
    uint32_t *gkey = x.get<uint32_t>(A_gkey, nnz);
    float *gval = x.get<float>(A_gval, nnz);
    ukey = x.get<uint32_t>(A_ukey, nnz);
    uval = x.get<float>(A_uval, nnz);
    agg_group(a, g.crow, pos, eoff, gkey, gval, x.s);
    // 4. small segments
    agg_small(seg, ncomm, gkey, gval, ukey, uval, v64, rowlen, Kout, x.s);
    // 5. large segments
    int32_t *lflag = x.get<int32_t>(A_lflag, ncomm + 1);
    int32_t *lidx = x.get<int32_t>(A_lidx, ncomm + 1);
    agg_large_flags(seg, ncomm, lflag, x.s);
    scan_i32(x, lflag, lidx, ncomm + 1);
    nl = x.read(&lidx[ncomm]);
    if (nl > 0) {
      lc = x.get<int32_t>(A_lc, nl);
      lsb = x.get<int64_t>(A_lsb, nl);
      int64_t *lse = x.get<int64_t>(A_lse, nl);
      ltn = x.get<int64_t>(A_ltn, nl + 1);
      agg_large_list(seg, ncomm, lflag, lidx, lc, lsb, lse, ltn, x.s);
      scan_i64(x, ltn, ltn, nl + 1);
      ntl = x.read(&ltn[nl]);
      tseg = x.get<int32_t>(A_tseg, ntl);
      agg_tile_seg(ltn, nl, ntl, tseg, x.s);
      RsSeg rs;
      rs.ntiles = ntl;
      rs.n = 0;
      rs.tseg = tseg;
      rs.tfirst = ltn;
      rs.sbeg = lsb;
      rs.send = lse;
      // sorted segments in (skey, sval); their rows go to the other pair
      const int cbe = nkey > 0 ? key_bits((unsigned long long)std::max<int64_t>(nkey - 1, 0)) : cb;
      const int r = rsort<uint32_t, float>(gkey, gval, ukey, uval, rs, cbe, x.tmp(rs_tmp_bytes(ntl)), x.s);
      uint32_t *skey = r ? ukey : gkey;
      float *sval = r ? uval : gval;
      lkey = r ? gkey : ukey;
      lval = r ? gval : uval;
      int64_t *hc = x.get<int64_t>(A_hc, ntl + 1);
      double *tin = x.get<double>(A_tin, 2 * ntl);
      double *tks = tin + ntl;
      x.zero(hc, ntl + 1);
      agg_large_runs(0, skey, sval, rs, hc, tin, lkey, lval, nullptr, nullptr, x.s);
      scan_i64(x, hc, hc, ntl + 1);
      agg_large_runs(1, skey, sval, rs, hc, tin, lkey, lval, v64, Kout ? tks : nullptr, x.s);
      agg_large_rows(nl, lc, ltn, hc, tks, rowlen, Kout, x.s);
    }
    if (x.kp) x.kp->end(t0, LEIDEN_PROF_AGG_MERGE, g.nnz, g.n);
    x.launched("aggregate");
  }
  scan_i32_i64(x, rowlen, out_off, ncomm + 1);
  const int64_t nu = g.nnz > 0 ? x.read(&out_off[ncomm]) : 0;
  int32_t *out_idx = x.get<int32_t>(si, nu);
  float *out_w = x.get<float>(sw, nu);
  double *out_w64 = v64 ? x.get<double>(L1_w64, nu) : nullptr;
  if (w64) *w64 = out_w64;
  if (g.nnz > 0)
    agg_compact(seg, ncomm, lc, lsb, tseg, ltn, ntl, rowlen, out_off, ukey, uval, lkey, lval, v64, out_idx, out_w,
                out_w64, x.s);
  int32_t *out_crow = x.get<int32_t>(sc, ceil_div(std::max<int64_t>(nu, 1), kChunk) + 2);
  chunk_start_rows(out_off, ncomm, nu, out_crow, x.s);
  x.launched("agg_rows");
  Level o{ncomm, nu, out_off, out_idx, out_w, out_crow};
  return o;
}

// The first aggregated level of a run, kept for the modularity of its result:
// every level-0 vertex of one first-level vertex (a refined community of the
// first pass) ends in the same community, so the internal weight of the
// result is the weight of the first level's entries inside communities,
// summed from their FP64 run sums (exact for these sums of float weights, up
// to the order of the final additions), over ~1/7 of the entries on RMAT.
struct Level1 {
  bool ok = false;
  Level g{};
  const double *w64 = nullptr;
  const int32_t *map = nullptr;  // level-0 vertex -> first-level vertex
  int64_t nlab = 0;              // first-level labels (with those left out of the level)
};

// modularity_known from the first aggregated level: the result's labels
// (C, n level-0 entries) carried to the first-level vertices, then one pass
// over the first level's entries with their FP64 weights.
double modularity_level1(Ctx &x, const Level1 &l1, const int32_t *C, int64_t n, const double *Sig, double M2) {
  if (!(M2 > 0.0)) return 0.0;
  DevScal *sc = x.scal();
  x.zero(sc->acc, 4);
  hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
  int32_t *lab = x.get<int32_t>(L1_lab, l1.nlab);
  scatter_labels(l1.map, C, n, lab, x.s);
  modularity_intra64(l1.g.off, l1.g.idx, l1.w64, l1.g.crow, l1.g.nnz, lab, sc->acc, x.s);
  if (x.kp) x.kp->end(t0, LEIDEN_PROF_MOD_SCAN, l1.g.nnz, n);
  modularity_comm_sq(Sig, n, M2, sc->acc, x.s);
  x.launched("modularity");
  double acc[4];
  x.check(hipMemcpyAsync(x.pin(), sc->acc, sizeof(acc), hipMemcpyDeviceToHost, x.s), "D2H");
  x.check(hipStreamSynchronize(x.s), "sync");
  memcpy(acc, x.pin(), sizeof(acc));
  return acc[0] / M2 - acc[2];
}

// The pass loop of Alg. "leiden".  On entry the level arrays hold the
// previous membership (L_C), K (L_K), Sigma (L_S), changed flags (L_dC),
// affected flags (L_U) and range flags (L_rng) for the level-0 graph g0.
// On exit `out` (n) holds dense labels.
void run_core(Ctx &x, const leiden_params &p, const Level &g0, double M2, bool track, int32_t *out,
              leiden_stats *st, Timer &tm, Level1 *l1 = nullptr) {
  const int64_t n = g0.n;
  DevScal *sc = x.scal();
  int32_t *C = x.get<int32_t>(L_C, n);
  double *K = x.get<double>(L_K, n);
  double *S = x.get<double>(L_S, n);
  double *S2 = x.get<double>(L_S2, n);
  uint8_t *dC = x.get<uint8_t>(L_dC, n);
  uint8_t *dC2 = x.get<uint8_t>(L_dC2, n);
  uint8_t *U = x.get<uint8_t>(L_U, n);
  uint8_t *rng = x.get<uint8_t>(L_rng, n);
  int32_t *CB = x.get<int32_t>(L_CB, n);
  int32_t *Ctop = x.get<int32_t>(L_Ctop, n);
  int32_t *prop = x.get<int32_t>(L_prop, n);
  int32_t *from = x.get<int32_t>(L_from, n);
  double *gp = x.get<double>(L_gp, n);
  double *gi = p.sync_mode ? x.get<double>(L_gi, n) : nullptr;
  int32_t *Sz = x.get<int32_t>(L_Sz, n);
  int32_t *rep = x.get<int32_t>(L_rep, n + 1);
  const int NS = p.sync_mode ? std::max(1, std::min(p.nslices, kMaxSlices))
                             : (p.hub_slices > 0 ? std::min(p.hub_slices, kMaxSlices) : kDefaultHubSlices);
  int32_t *lists = x.get<int32_t>(L_lists, n);
  int32_t *region = x.get<int32_t>(L_region, NS * kNB + 1);
  int32_t *counts = x.get<int32_t>(L_scnt, NS * kNB + NS);
  int32_t *scnt = counts + NS * kNB;
  int32_t *vbs = x.get<int32_t>(L_vbs, n);
  int32_t *soff = x.get<int32_t>(L_soff, NS + 1);
  int32_t *sfill = x.get<int32_t>(L_sfill, NS);
  double *tiles = x.get<double>(L_tiles, n / 256 + 2);
  uint8_t *act = x.get<uint8_t>(L_act, n);
  const bool async = p.sync_mode == 0;
  // degree above which a vertex moves in the hub slices before the sweep
  // (asynchronous mode); the synchronous mode keeps the table-size boundary
  const int64_t hubdeg = (async && p.hub_degree > 0) ? p.hub_degree : kHubDeg;
  const int NW = async ? (p.async_waves > 0 ? p.async_waves : kDefaultAsyncWaves) : 0;
  int *akeys = async ? x.get<int>(W_keys, (int64_t)NW * 2 * kHubDeg) : nullptr;
  double *avals = async ? x.get<double>(W_vals, (int64_t)NW * 2 * kHubDeg) : nullptr;

  if (p.refine_variant == 1) {
    fill_u8(dC, 1, n, x.s);
    track = false;
  }
  if (st) {
    x.zero(&sc->nz, 1);
    count_nonzero_u8(U, n, &sc->nz, x.s);
    x.launched("count");
    st->affected = (int64_t)x.read(&sc->nz);
  }
  iota_i32(Ctop, n, x.s);
  fill_i32(prop, -1, n, x.s);
  x.launched("core init");
  tm.mark(CAT_OTHER);

  Level g = g0;
  int curbuf = -1;  // -1: the level-0 graph
  // Asynchronous mode with several wavefronts: the first level's vertices
  // without edges (level-0 vertices without edges, alone in every pass) are
  // left out of the aggregated levels; their labels stay above every later
  // level's and the pass loop's rules and statistics count them as before.
  // (One wavefront keeps the serial order and labels.)
  const bool compact = async && NW > 1;
  int64_t niso = 0;
  double tau = p.tau0;
  int pass = 0;
  for (pass = 0; pass < p.max_passes; ++pass) {
    tm.pass = pass;
    const int64_t nl = g.n;
    const int64_t nfull = nl + niso;
    const Layout B = level_layout(x, g, NS, hubdeg, region, counts, scnt, soff, sfill, vbs);
    const HubHost hh = hub_plan(x, g, NS, hubdeg, B);
    const int64_t alen = B.region[NS * kNB];  // vertices with edges
    int32_t *alist = nullptr;
    if (async && alen > 0) {
      int32_t *flags = x.get<int32_t>(L_flags, nl + 1);
      int32_t *pos = x.get<int32_t>(L_map, nl + 1);
      alist = x.get<int32_t>(W_list, alen);
      edge_flags(g.off, nl, flags, x.s);
      scan_i32(x, flags, pos, nl);
      edge_list(g.off, nl, pos, alist, x.s);
      x.launched("edge list");
    }
    if (pass > 0) fill_u8(rng, 1, nl, x.s);
    const double Tp = tau * M2 * M2 / 2.0;

    MoveArgs ma;
    memset(&ma, 0, sizeof(ma));
    ma.n = nl; ma.off = g.off; ma.idx = g.idx; ma.w = g.w;
    ma.C = C; ma.K = K; ma.Sig = S; ma.dC = dC; ma.U = U; ma.rng = rng; ma.M2 = M2;
    ma.track = (track && pass == 0) ? 1 : 0;
    ma.prop = prop; ma.from = from; ma.gp = gp; ma.gi = gi;
    ma.lists = lists; ma.region = region; ma.counts = counts; ma.nsl = NS; ma.vbyslice = vbs;
    ma.gain = gi ? nullptr : &sc->gain; ma.moves = &sc->moves;
    ma.hp = hh.p;
    ma.act = hh.nhub > 0 ? act : nullptr;
    ma.hub_front = async ? 1 : 0;
    ma.hub_scanned = x.kp && x.kp->on ? &sc->hub_scanned : nullptr;
    ma.sweep_work = x.kp && x.kp->on ? sc->sweep_work : nullptr;
    ma.anext = &sc->anext; ma.akeys = akeys; ma.avals = avals;
    ma.alist = alist; ma.alen = alen;
    ma.hubdeg = hubdeg;
    ma.cached = async && nfull >= kCachedLevel;
    ma.defer = async && NW > 1;
    int li = 0;
    int64_t moves_total = 0;
    unsigned long long min_moves = ~0ull;
    int stall = 0;
    bool stalled = false;
    tm.mark(CAT_OTHER);
    for (int it = 0; it < p.max_iter; ++it) {
      reset_iter(counts, NS * kNB, &sc->gain, &sc->moves, async ? &sc->anext : nullptr, x.s);
      if (gi) x.zero(gi, nl);
      // asynchronous mode: the hub slices of the iteration timed as one region
      hipEvent_t th = (x.kp && async && hh.nhub > 0) ? x.kp->begin() : nullptr;
      for (int sl = 0; sl < NS; ++sl) {
        ma.s = sl;
        ma.vbeg = B.soff[sl];
        ma.vend = B.soff[sl + 1];
        ma.hbeg = hh.hs[sl]; ma.hend = hh.hs[sl + 1];
        ma.qbeg = hh.qs[sl]; ma.qend = hh.qs[sl + 1];
        ma.gbeg = hh.gs[sl]; ma.gend = hh.gs[sl + 1];
        if (async) {
          // hubs: synchronous among the hubs of the slice; the rest below
          if (ma.hend == ma.hbeg) continue;
          move_hub_gather(ma, x.s);
          move_hub_score(ma, x.s);
          move_apply_bucket(ma, B.region.data(), kNB - 1, x.s);
          continue;
        }
        move_frontier(ma, x.s);
        for (int b = 0; b + 1 < kNB; ++b) move_propose_bucket(ma, B.region.data(), b, x.s);
        if (ma.qend > ma.qbeg) {
          hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
          move_hub_gather(ma, x.s);
          if (x.kp) x.kp->end(t0, LEIDEN_PROF_HUB_GATHER, 0, 0);
          move_hub_score(ma, x.s);
        }
        move_apply(ma, B.region.data(), x.s);
      }
      if (th) x.kp->end(th, LEIDEN_PROF_HUB_GATHER, 0, 0);
      if (async) {
        // after the hubs: the other vertices then see the hubs' new communities
        hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
        move_async(ma, level_waves(p, NW, alen, pass), wide_tables(g.nnz, alen), x.s);
        if (x.kp) x.kp->end(t0, LEIDEN_PROF_MOVE_SWEEP, 0, 0);
      }
      if (gi) tiled_sum(gi, nl, tiles, &sc->gain, x.s);
      x.launched("move iteration");
      struct {
        double gain;
        unsigned long long moves;
      } r;
      x.check(hipMemcpyAsync(x.pin(), &sc->gain, sizeof(r), hipMemcpyDeviceToHost, x.s), "D2H");
      x.check(hipStreamSynchronize(x.s), "sync");
      memcpy(&r, x.pin(), sizeof(r));
      moves_total += (int64_t)r.moves;
      li = it + 1;
      if (r.gain <= Tp) break;
      // Asynchronous mode, aggregated levels: vertices moved against a state
      // that concurrently processed neighbours are changing can trade places
      // indefinitely, each move scored as a gain; the tolerance test then
      // never passes.  Stop when the number of moves has not reached a new
      // minimum for kStallIters iterations in a row.
      if (async && pass > 0 && level_waves(p, NW, alen, pass) > 1) {
        if (r.moves < min_moves) {
          min_moves = r.moves;
          stall = 0;
        } else if (++stall >= kStallIters) {
          stalled = true;
          break;
        }
      }
    }
    tm.mark(CAT_MOVE);
    if (st && pass < LEIDEN_MAX_PASSES) {
      st->move_iters[pass] = li;
      st->level_vertices[pass] = nfull;
      st->level_entries[pass] = g.nnz;
      if (pass == 0) {
        st->moves_pass0 = moves_total;
        x.zero(&sc->nz, 1);
        count_nonzero_u8(dC, nl, &sc->nz, x.s);
        x.launched("count");
        st->changed = (int64_t)x.read(&sc->nz);
      }
    }
    // subset renumber, bounds, break, refine
    subset_renumber(nl, C, rep, S, S2, dC, dC2, x.s);
    std::swap(S, S2);
    std::swap(dC, dC2);
    x.launched("subset_renumber");
    RefineArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.n = nl; ra.off = g.off; ra.idx = g.idx; ra.w = g.w;
    ra.C = C; ra.CB = CB; ra.K = K; ra.Sig = S; ra.dC = dC; ra.S = Sz; ra.M2 = M2;
    ra.prop = prop; ra.gp = gp; ra.lists = lists; ra.region = region; ra.counts = counts; ra.nsl = NS;
    ra.refined = &sc->refined;
    ra.anext = &sc->anext; ra.akeys = akeys; ra.avals = avals;
    ra.alist = alist; ra.alen = alen;
    ra.hubdeg = hubdeg;
    ra.cached = async && nfull >= kCachedLevel;
    ra.defer = async && NW > 1;
    ra.sweep_work = x.kp && x.kp->on ? sc->sweep_work + 2 : nullptr;
    reset_iter(counts, NS * kNB, nullptr, &sc->refined, async ? &sc->anext : nullptr, x.s);
    refine_break(ra, x.s);
    x.launched("break");
    ra.hp = hh.p;
    ra.act = act;
    if (async) {
      // communities and bounds packed for the hub slices and the sweep (the
      // accept kernel and the sweep keep them with C)
      ra.CP = x.get<unsigned long long>(L_CP, nl);
      pack_cb(C, CB, nl, ra.CP, x.s);
    }
    for (int sl = 0; sl < NS; ++sl) {
      ra.s = sl;
      ra.hbeg = hh.hs[sl]; ra.hend = hh.hs[sl + 1];
      ra.qbeg = hh.qs[sl]; ra.qend = hh.qs[sl + 1];
      ra.gbeg = hh.gs[sl]; ra.gend = hh.gs[sl + 1];
      if (async) {
        // hubs of the slice (synchronous among themselves), the rest below
        if (B.region[sl * kNB + kNB] == B.region[sl * kNB + kNB - 1]) continue;
        refine_propose_bucket(ra, B.region.data(), kNB - 1, x.s);
      } else {
        refine_propose(ra, B.region.data(), x.s);
      }
      refine_accept(ra, B.region.data(), x.s);
    }
    if (async) {
      hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
      refine_async(ra, level_waves(p, NW, alen, pass), wide_tables(g.nnz, alen), x.s);
      if (x.kp) x.kp->end(t0, LEIDEN_PROF_REFINE_SWEEP, 0, 0);
    }
    x.launched("refine sweep");
    const int rounds = 1;
    tm.mark(CAT_REFINE);
    if (st && pass < LEIDEN_MAX_PASSES) {
      st->refine_rounds[pass] = rounds;
      st->refined_vertices[pass] = (int64_t)x.read(&sc->refined);
      st->passes = pass + 1;
    }
    if ((pass > 0 || p.refine_variant == 2) && li <= 1) {
      if (st && pass < LEIDEN_MAX_PASSES) {
        // communities of this level, for the statistics only
        int32_t *tmpC = x.get<int32_t>(L_CB, nl);
        x.copy(tmpC, C, nl);
        st->communities[pass] = renumber_dense(x, tmpC, nl, nl) + niso;
      }
      tm.mark(CAT_OTHER);
      break;
    }
    int64_t nact = 0;
    const int64_t ncomm = (compact && pass == 0) ? renumber_active_first(x, C, nl, g.off, &nact)
                                                 : renumber_dense(x, C, nl, nl);
    if (!(compact && pass == 0)) nact = ncomm;
    if (st && pass < LEIDEN_MAX_PASSES) st->communities[pass] = ncomm + niso;
    if (p.agg_tol < 1.0 && (double)(ncomm + niso) / (double)nfull > p.agg_tol) {
      tm.mark(CAT_OTHER);
      break;
    }
    // A stalled level that merged few of its vertices has converged up to the
    // trades: it ends the passes as a level that converged in one iteration
    // would.  A stalled level that still merged many (slowly converging
    // levels, e.g. of road-like graphs) goes on to the next pass.
    if (stalled && (double)(ncomm + niso) > kStallKeep * (double)nfull) {
      tm.mark(CAT_OTHER);
      break;
    }
    gather_map_bounded(Ctop, C, n, nl, x.s);  // dendrogram lookup (left-out labels stay)
    x.launched("lookup");
    tm.mark(CAT_OTHER);
    if (l1 && pass == 0) {
      // the first level with its FP64 weights and the level-0 map (C here)
      int32_t *map = x.get<int32_t>(L1_map, n);
      x.copy(map, C, n);
      double *w64 = nullptr;
      g = aggregate_level(x, g, C, ncomm, 2, K, &w64, nact);
      curbuf = 2;
      l1->ok = w64 != nullptr;
      l1->w64 = w64;
      l1->map = map;
      l1->nlab = ncomm;
    } else {
      const int outbuf = (curbuf == 0) ? 1 : 0;
      g = aggregate_level(x, g, C, ncomm, outbuf, K, nullptr, nact);
      curbuf = outbuf;
    }
    if (nact < ncomm) {
      // the trailing rows are the left-out vertices' (empty): drop them
      g.n = nact;
      chunk_start_rows(g.off, nact, g.nnz, const_cast<int32_t *>(g.crow), x.s);
      niso += ncomm - nact;
    }
    if (l1 && pass == 0) l1->g = g;
    tm.mark(CAT_AGG);
    x.copy(S, K, nact);
    fill_u8(U, 1, nact, x.s);
    iota_i32(C, nact, x.s);
    fill_u8(dC, 1, nact, x.s);
    x.launched("pass reset");
    tau = tau / p.tol_drop;
  }
  tm.pass = -1;
  if (st && pass >= p.max_passes) st->passes = p.max_passes;
  gather_map_bounded(Ctop, C, n, g.n, x.s);
  renumber_dense(x, Ctop, n, n);
  x.copy(out, Ctop, n);
  x.launched("final lookup");
  tm.mark(CAT_OTHER);
}

}  // namespace

namespace {
leiden_status run_guarded(Workspace &w, const std::function<void()> &f) {
  try {
    f();
    return LEIDEN_OK;
  } catch (const Fail &e) {
    return e.st;
  } catch (const std::bad_alloc &) {
    w.err = "host allocation failed";
    return LEIDEN_ENOMEM;
  } catch (...) {
    w.err = "unexpected error";
    return LEIDEN_EHIP;
  }
}

// Sort rows of a CSR in place (keys = neighbour ids, values = weights).
void sort_rows(Ctx &x, int64_t n, int64_t nnz, int64_t *off, int32_t *idx, float *w, int32_t *idx2, float *w2) {
  if (nnz == 0) return;
  size_t tb = seg_sort_i32_f32(nullptr, 0, idx, idx2, w, w2, nnz, n, off, x.s);
  seg_sort_i32_f32(x.tmp(tb), tb, idx, idx2, w, w2, nnz, n, off, x.s);
  x.launched("segmented sort");
  x.copy(idx, idx2, nnz);
  x.copy(w, w2, nnz);
}

Level handle_level(leiden_handle *h) {
  return Level{h->n, h->nnz, (const int64_t *)h->g_off.p, (const int32_t *)h->g_idx.p,
               (const float *)h->g_w.p, (const int32_t *)h->g_crow.p};
}

void refresh_crow(Ctx &x, leiden_handle *h) {
  const int64_t nch = ceil_div(std::max<int64_t>(h->nnz, 1), kChunk);
  x.ensure(h->g_crow, (size_t)(nch + 2) * sizeof(int32_t));
  chunk_start_rows((const int64_t *)h->g_off.p, h->n, h->nnz, (int32_t *)h->g_crow.p, x.s);
  x.launched("chunk_start_rows");
}

bool valid_params(const leiden_params *p) {
  return p && p->tau0 >= 0 && p->tol_drop > 0 && p->agg_tol > 0 && p->max_iter >= 1 &&
         p->max_passes >= 1 && p->max_passes <= LEIDEN_MAX_PASSES && (p->sync_mode == 0 || p->sync_mode == 1) &&
         p->refine_variant >= 0 && p->refine_variant <= 2 && p->nslices >= 1 && p->nslices <= kMaxSlices &&
         (p->profile == 0 || p->profile == 1) && p->async_waves >= 0 && p->async_waves <= kMaxAsyncWaves &&
         p->hub_slices >= 0 && p->hub_slices <= kMaxSlices && (p->trim == 0 || p->trim == 1) &&
         p->verts_per_wave >= 0 && p->verts_per_wave_upper >= 0 && p->hub_degree >= 0 &&
         p->hub_degree <= kHubDeg && (p->hub_degree == 0 || p->hub_degree >= 64);
}

}  // namespace

namespace {
bool batch_pointers_ok(const leiden_batch *batch) {
  if (batch->n_del < 0 || batch->n_ins < 0) return false;
  if (batch->n_del > 0 && (!batch->del_u || !batch->del_v)) return false;
  if (batch->n_ins > 0 && (!batch->ins_u || !batch->ins_v || !batch->ins_w)) return false;
  return true;
}

// Validates the batch against G^{t-1} (the handle's graph) and builds G^t,
// rows sorted, in the handle's spare CSR (t_off, t_idx, t_w); the handle's
// graph and state are not modified.  Returns |E^t|; b keeps the sorted
// directed batch for the marking.
int64_t stage_batch(Ctx &x, leiden_handle *h, const leiden_batch &batch, BatchArgs &b) {
  const int64_t n = h->n;
  DevScal *sc = x.scal();
  memset(&b, 0, sizeof(b));
  b.n = n;
  b.nnz = h->nnz;
  b.off = (const int64_t *)h->g_off.p;
  b.idx = (const int32_t *)h->g_idx.p;
  b.w = (const float *)h->g_w.p;
  b.nd = batch.n_del;
  b.ni = batch.n_ins;
  b.du = batch.del_u; b.dv = batch.del_v;
  b.iu = batch.ins_u; b.iv = batch.ins_v; b.iw = batch.ins_w;
  b.E = 2 * (b.nd + b.ni);
  const int64_t E = b.E;
  b.keys = x.get<unsigned long long>(B_keys, E);
  b.vals = x.get<int32_t>(B_vals, E);
  b.skeys = x.get<unsigned long long>(B_skeys, E);
  b.svals = x.get<int32_t>(B_svals, E);
  b.ew = x.get<float>(B_ew, E);
  b.err = &sc->err;
  b.bstart = x.get<int64_t>(B_bstart, n);
  b.bcnt = x.get<int32_t>(B_bcnt, n);
  b.dcnt = x.get<int32_t>(B_dcnt, n);
  b.icnt = x.get<int32_t>(B_icnt, n);
  b.isdel = x.get<int32_t>(B_isdel, E + 1);
  b.delpre = x.get<int32_t>(B_delpre, E + 1);
  b.newdeg = x.get<int64_t>(B_newdeg, n + 1);
  b.crow = (const int32_t *)h->g_crow.p;
  x.zero(&sc->err, 1);
  x.zero(b.bcnt, n);
  x.zero(b.dcnt, n);
  x.zero(b.icnt, n);
  batch_build(b, x.s);
  x.launched("batch_build");
  if (E > 0) {
    size_t tb = sort_pairs_u64_i32(nullptr, 0, b.keys, b.skeys, b.vals, b.svals, E, x.s);
    sort_pairs_u64_i32(x.tmp(tb), tb, b.keys, b.skeys, b.vals, b.svals, E, x.s);
    x.launched("batch sort");
  }
  batch_dups_rows(b, x.s);
  x.launched("batch_dups");
  const int32_t err = x.read(&sc->err);
  if (err) {
    std::string why;
    if (err & 1) why += " id out of range;";
    if (err & 2) why += " self-loop;";
    if (err & 4) why += " repeated edge;";
    if (err & 8) why += " deletion of a missing edge;";
    if (err & 16) why += " insertion of an existing edge;";
    if (err & 32) why += " non-positive or non-finite weight;";
    x.invalid("invalid batch:" + why);
  }
  x.ensure(h->t_off, (size_t)(n + 1) * sizeof(int64_t));
  b.newoff = (int64_t *)h->t_off.p;
  batch_newdeg(b, x.s);
  scan_i64(x, b.newdeg, b.newoff, n + 1);
  scan_i32(x, b.isdel, b.delpre, E + 1);
  const int64_t nnz_new = x.read(&b.newoff[n]);
  x.ensure(h->t_idx, (size_t)std::max<int64_t>(nnz_new, 1) * sizeof(int32_t));
  x.ensure(h->t_w, (size_t)std::max<int64_t>(nnz_new, 1) * sizeof(float));
  b.nidx = (int32_t *)h->t_idx.p;
  b.nw = (float *)h->t_w.p;
  hipEvent_t t0 = x.kp ? x.kp->begin() : nullptr;
  batch_apply_old(b, x.s);
  if (x.kp) x.kp->end(t0, LEIDEN_PROF_BATCH_MERGE, nnz_new, n);
  batch_apply_ins(b, x.s);
  x.launched("batch_apply");
  return nnz_new;
}

// Alg. "naiveDynamic" / "deltaScreening" / "dynamicFrontier" and
// changedCommunities: flags dV (affected), rng (in range) and dC (changed,
// keyed by C^{t-1}) from the staged batch b, G^t = g and the handle's
// C^{t-1}, K^{t-1}, Sigma^{t-1}; m is left ready for updateWeights.
void mark_batch(Ctx &x, leiden_handle *h, int32_t mode, const BatchArgs &b, const Level &g, uint8_t *dV,
                uint8_t *rng, uint8_t *dC, MarkArgs &m) {
  const int64_t n = h->n;
  const int64_t E = b.E;
  DevScal *sc = x.scal();
  x.zero(dV, n);
  x.zero(rng, n);
  x.zero(dC, n);
  memset(&m, 0, sizeof(m));
  m.n = n;
  m.off = g.off;
  m.idx = g.idx;
  m.E = E;
  m.nd2 = 2 * b.nd;
  m.skeys = b.skeys;
  m.svals = b.svals;
  m.ew = b.ew;
  m.C = (const int32_t *)h->C.p;
  m.K = (const double *)h->K.p;
  m.Sig = (const double *)h->Sig.p;
  m.M2 = h->M2;
  m.dV = dV;
  m.rng = rng;
  m.dC = dC;
  if (mode == LEIDEN_ND) {
    fill_u8(dV, 1, n, x.s);
    fill_u8(rng, 1, n, x.s);
    mark_changed(m, x.s);
  } else if (mode == LEIDEN_DF) {
    mark_df(m, x.s);
    fill_u8(rng, 1, n, x.s);
  } else {
    m.dE = x.get<uint8_t>(M_dE, n);
    m.dCm = x.get<uint8_t>(M_dCm, n);
    m.k2 = x.get<unsigned long long>(M_k2, E);
    m.k2s = x.get<unsigned long long>(M_k2s, E);
    m.v2 = x.get<double>(M_v2, E);
    m.v2s = x.get<double>(M_v2s, E);
    m.list = x.get<int32_t>(M_list, n);
    m.count = &sc->list_count;
    x.zero(m.dE, n);
    x.zero(m.dCm, n);
    x.zero(m.count, 1);
    mark_ds_del(m, x.s);
    mark_ds_keys(m, x.s);
    if (E > 0) {
      size_t tb = sort_pairs_u64_f64(nullptr, 0, m.k2, m.k2s, m.v2, m.v2s, E, x.s);
      sort_pairs_u64_f64(x.tmp(tb), tb, m.k2, m.k2s, m.v2, m.v2s, E, x.s);
    }
    mark_ds_best(m, x.s);
    mark_ds_expand(m, x.s);
  }
  x.launched("marking");
}
}  // namespace

namespace {
// A call on a stream other than the previous call's first waits for the
// handle's latest work (recorded in h->order at the end of every call), so
// calls on different streams never overlap on the handle's memory.
void enter(Ctx &x, leiden_handle *h) {
  if (!h->order) x.check(hipEventCreateWithFlags(&h->order, hipEventDisableTiming), "hipEventCreate");
  if (h->used && h->last != x.s) x.check(hipStreamWaitEvent(x.s, h->order, 0), "hipStreamWaitEvent");
  h->last = x.s;
}
void leave(leiden_handle *h, hipStream_t s) {
  if (h->order && hipEventRecord(h->order, s) == hipSuccess) h->used = true;
  else (void)hipGetLastError();
}
// A call on handle h: ordered after the handle's previous work, guarded;
// with leiden_params.trim the working buffers and the spare CSR are released
// (stream-ordered) when it ends.
leiden_status run_handle(leiden_handle *h, Ctx &x, const std::function<void()> &f) {
  leiden_status st = run_guarded(h->w, [&] {
    enter(x, h);
    f();
  });
  if (h->prm.trim) {
    h->w.release(x.s);
    for (DBuf *b : {&h->t_off, &h->t_idx, &h->t_w}) {
      h->w.al.put(b->p, b->cap, x.s);
      *b = DBuf{};
    }
  }
  leave(h, x.s);
  return st;
}
}  // namespace

// ============================ C ABI =========================================
extern "C" {

void leiden_default_params(leiden_params *p) {
  if (!p) return;
  p->tau0 = 0.01;
  p->tol_drop = 10.0;
  p->agg_tol = 1.0;
  p->max_iter = 20;
  p->max_passes = 10;
  p->sync_mode = 0;
  p->refine_variant = 0;
  p->nslices = 16;
  p->profile = 0;
  p->async_waves = 0;
  p->hub_slices = 0;
  p->verts_per_wave = 0;
  p->verts_per_wave_upper = 0;
  p->hub_degree = kDefaultHubDeg;
  p->trim = 0;
}

const char *leiden_strerror(int32_t status) {
  switch (status) {
    case LEIDEN_OK: return "ok";
    case LEIDEN_EINVAL: return "invalid argument";
    case LEIDEN_ENOMEM: return "out of device memory";
    case LEIDEN_ESTATE: return "no community state (run leiden_static or leiden_set_state first)";
    case LEIDEN_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *leiden_last_error(const leiden_handle *h) { return h ? h->w.err.c_str() : ""; }
int64_t leiden_num_vertices(const leiden_handle *h) { return h ? h->n : -1; }
int64_t leiden_num_entries(const leiden_handle *h) { return h ? h->nnz : -1; }

leiden_status leiden_create(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *indices,
                            const float *weights, const leiden_params *params, const leiden_allocator *alloc,
                            void *stream, leiden_handle **out) {
  if (!out || n < 0 || nnz < 0 || n > INT32_MAX - 1 || !offsets || (nnz > 0 && (!indices || !weights)))
    return LEIDEN_EINVAL;
  if (params && !valid_params(params)) return LEIDEN_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->release)) return LEIDEN_EINVAL;
  *out = nullptr;
  leiden_handle *h = new (std::nothrow) leiden_handle();
  if (!h) return LEIDEN_ENOMEM;
  h->n = n;
  h->nnz = nnz;
  if (params) h->prm = *params;
  else leiden_default_params(&h->prm);
  if (alloc) {
    h->w.al.a = *alloc;
    h->w.al.custom = true;
  }
  Ctx x{&h->w, (hipStream_t)stream};
  leiden_status st = run_guarded(h->w, [&] {
    enter(x, h);
    x.ensure(h->g_off, (size_t)(n + 1) * sizeof(int64_t));
    x.ensure(h->g_idx, (size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));
    x.ensure(h->g_w, (size_t)std::max<int64_t>(nnz, 1) * sizeof(float));
    x.copy((int64_t *)h->g_off.p, offsets, n + 1);
    x.copy((int32_t *)h->g_idx.p, indices, nnz);
    x.copy((float *)h->g_w.p, weights, nnz);
    DevScal *sc = x.scal();
    x.zero(&sc->err, 1);
    check_offsets((const int64_t *)h->g_off.p, n, nnz, &sc->err, x.s);
    x.launched("check_offsets");
    if (x.read(&sc->err)) x.invalid("offsets are not a valid CSR of nnz entries");
    x.ensure(h->t_idx, (size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));
    x.ensure(h->t_w, (size_t)std::max<int64_t>(nnz, 1) * sizeof(float));
    sort_rows(x, n, nnz, (int64_t *)h->g_off.p, (int32_t *)h->g_idx.p, (float *)h->g_w.p,
              (int32_t *)h->t_idx.p, (float *)h->t_w.p);
    refresh_crow(x, h);
    check_rows_chunked((const int64_t *)h->g_off.p, (const int32_t *)h->g_idx.p, (const float *)h->g_w.p, n,
                       nnz, (const int32_t *)h->g_crow.p, &sc->err, x.s);
    x.launched("check_rows");
    if (x.read(&sc->err))
      x.invalid("graph has an id out of range, a non-positive or non-finite weight, or a repeated entry");
  });
  if (st != LEIDEN_OK) {
    h->release(x.s);
    delete h;
    return st;
  }
  if (h->prm.trim) {
    h->w.release(x.s);
    for (DBuf *b : {&h->t_off, &h->t_idx, &h->t_w}) {
      h->w.al.put(b->p, b->cap, x.s);
      *b = DBuf{};
    }
  }
  leave(h, x.s);
  *out = h;
  return LEIDEN_OK;
}

leiden_status leiden_destroy(leiden_handle *h) {
  if (!h) return LEIDEN_EINVAL;
  // no wait for the device: the releases are ordered after the handle's last
  // work (on the null stream, which first waits for that work)
  hipStream_t s = nullptr;
  if (h->used && h->order) (void)hipStreamWaitEvent(s, h->order, 0);
  h->release(s);
  (void)hipGetLastError();
  delete h;
  return LEIDEN_OK;
}

leiden_status leiden_set_params(leiden_handle *h, const leiden_params *params) {
  if (!h || !valid_params(params)) return LEIDEN_EINVAL;
  h->prm = *params;
  return LEIDEN_OK;
}

leiden_status leiden_static(leiden_handle *h, int32_t *membership_out, double *q_out, leiden_stats *stats,
                            void *stream) {
  if (!h) return LEIDEN_EINVAL;
  if (stats) memset(stats, 0, sizeof(*stats));
  Ctx x{&h->w, (hipStream_t)stream};
  return run_handle(h, x, [&] {
    Timer tm(x, stats != nullptr);
    KProf kp(x, stats != nullptr && h->prm.profile != 0);
    x.kp = &kp;
    Level1 l1;
    if (kp.on) {
      x.zero(&x.scal()->hub_scanned, 1);
      x.zero(x.scal()->sweep_work, 4);
    }
    tm.mark(CAT_OTHER);
    const int64_t n = h->n;
    x.ensure(h->C, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
    x.ensure(h->K, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
    x.ensure(h->Sig, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
    int32_t *C = (int32_t *)h->C.p;
    double *K = (double *)h->K.p;
    double *Sig = (double *)h->Sig.p;
    const Level g = handle_level(h);
    DevScal *sc = x.scal();
    x.zero(K, n);
    row_sums(g.off, g.w, n, g.nnz, g.crow, K, x.s);
    x.zero(sc->acc, 4);
    modularity_comm(K, n, sc->acc, x.s);
    x.launched("static init");
    const double M2 = x.read(&sc->acc[1]);
    if (n > 0) {
      iota_i32(x.get<int32_t>(L_C, n), n, x.s);
      x.copy(x.get<double>(L_K, n), K, n);
      x.copy(x.get<double>(L_S, n), K, n);
      fill_u8(x.get<uint8_t>(L_dC, n), 1, n, x.s);
      fill_u8(x.get<uint8_t>(L_U, n), 1, n, x.s);
      fill_u8(x.get<uint8_t>(L_rng, n), 1, n, x.s);
      x.launched("static init");
      run_core(x, h->prm, g, M2, false, C, stats, tm, q_out ? &l1 : nullptr);
      x.zero(Sig, n);
      scatter_add(K, C, n, Sig, x.s);
      x.launched("sigma");
    }
    h->M2 = M2;
    h->has_state = true;
    if (membership_out) x.copy(membership_out, (const int32_t *)C, n);
    if (q_out)
      *q_out = n <= 0 ? 0.0 : l1.ok ? modularity_level1(x, l1, C, n, Sig, M2) : modularity_known(x, g, C, Sig, M2);
    tm.mark(CAT_OTHER);
    tm.finish(stats);
    kp.finish(stats, kp.on ? &x.scal()->hub_scanned : nullptr, kp.on ? x.scal()->sweep_work : nullptr);
    x.check(hipStreamSynchronize(x.s), "sync");
  });
}

leiden_status leiden_update(leiden_handle *h, const leiden_batch *batch, int32_t mode, int32_t *membership_out,
                            double *q_out, leiden_stats *stats, const leiden_trace *trace, void *stream) {
  if (!h || !batch) return LEIDEN_EINVAL;
  if (mode != LEIDEN_ND && mode != LEIDEN_DS && mode != LEIDEN_DF) return LEIDEN_EINVAL;
  if (!batch_pointers_ok(batch)) return LEIDEN_EINVAL;
  if (!h->has_state) {
    h->w.err = "update before leiden_static or leiden_set_state";
    return LEIDEN_ESTATE;
  }
  if (stats) memset(stats, 0, sizeof(*stats));
  Ctx x{&h->w, (hipStream_t)stream};
  bool mutated = false;  // the handle holds G^t (set once the new graph is installed)
  const leiden_status status = run_handle(h, x, [&] {
    Timer tm(x, stats != nullptr);
    KProf kp(x, stats != nullptr && h->prm.profile != 0);
    x.kp = &kp;
    Level1 l1;
    if (kp.on) {
      x.zero(&x.scal()->hub_scanned, 1);
      x.zero(x.scal()->sweep_work, 4);
    }
    tm.mark(CAT_OTHER);
    const int64_t n = h->n;
    DevScal *sc = x.scal();
    // ---- validate the batch and build G^t in the spare CSR ----
    BatchArgs b;
    const int64_t nnz_new = stage_batch(x, h, *batch, b);
    const int64_t E = b.E;
    std::swap(h->g_off, h->t_off);
    std::swap(h->g_idx, h->t_idx);
    std::swap(h->g_w, h->t_w);
    h->nnz = nnz_new;
    mutated = true;
    refresh_crow(x, h);
    tm.mark(CAT_APPLY);

    // ---- marking, changedCommunities, updateWeights ----
    const Level g = handle_level(h);
    uint8_t *dV = x.get<uint8_t>(L_U, n);
    uint8_t *rng = x.get<uint8_t>(L_rng, n);
    uint8_t *dC = x.get<uint8_t>(L_dC, n);
    MarkArgs m;
    mark_batch(x, h, mode, b, g, dV, rng, dC, m);
    if (trace) {
      if (trace->affected) x.copy(trace->affected, (const uint8_t *)dV, n);
      if (trace->in_range) x.copy(trace->in_range, (const uint8_t *)rng, n);
      if (trace->changed) x.copy(trace->changed, (const uint8_t *)dC, n);
    }
    (void)E;
    x.zero(&sc->m2delta, 1);
    update_weights(m, (double *)h->K.p, (double *)h->Sig.p, &sc->m2delta, x.s);
    x.launched("update_weights");
    h->M2 += x.read(&sc->m2delta);
    tm.mark(CAT_MARK);

    // ---- the pass loop from the previous membership ----
    if (n > 0) {
      x.copy(x.get<int32_t>(L_C, n), (const int32_t *)h->C.p, n);
      x.copy(x.get<double>(L_K, n), (const double *)h->K.p, n);
      x.copy(x.get<double>(L_S, n), (const double *)h->Sig.p, n);
      run_core(x, h->prm, g, h->M2, true, (int32_t *)h->C.p, stats, tm, q_out ? &l1 : nullptr);
      x.zero((double *)h->Sig.p, n);
      scatter_add((const double *)h->K.p, (const int32_t *)h->C.p, n, (double *)h->Sig.p, x.s);
      x.launched("sigma");
    }
    if (membership_out) x.copy(membership_out, (const int32_t *)h->C.p, n);
    if (q_out)
      *q_out = n <= 0 ? 0.0
               : l1.ok ? modularity_level1(x, l1, (const int32_t *)h->C.p, n, (const double *)h->Sig.p, h->M2)
                       : modularity_known(x, g, (const int32_t *)h->C.p, (const double *)h->Sig.p, h->M2);
    tm.mark(CAT_OTHER);
    tm.finish(stats);
    kp.finish(stats, kp.on ? &x.scal()->hub_scanned : nullptr, kp.on ? x.scal()->sweep_work : nullptr);
    x.check(hipStreamSynchronize(x.s), "sync");
  });
  if (status != LEIDEN_OK && mutated) {
    // G^t is installed but C, K, Sigma may be part-way through the update:
    // the handle keeps the new graph and refuses updates until a membership
    // is installed again
    h->has_state = false;
    h->w.err += " (the handle holds the updated graph without a community state: call leiden_static or "
                "leiden_set_state before the next update)";
  }
  return status;
}

leiden_status leiden_update_bytes(const leiden_handle *h, int64_t n_del, int64_t n_ins, int64_t *bytes) {
  if (!h || !bytes || n_del < 0 || n_ins < 0) return LEIDEN_EINVAL;
  // working set of an update (per vertex: level state, flags, lists, batch
  // rows, the aggregation's community order, the first level's map and
  // labels; per entry: the graph and its spare copy, two level graphs, the
  // aggregation's grouped entries and results (16 bytes), the first level's
  // FP64 run sums and their rows (16 bytes at most), room for the hub
  // tables; per directed batch entry: keys, values and their sorted copies;
  // plus the per-wavefront tables of the asynchronous sweeps) minus what the
  // handle already holds.  At RMAT scale 26 (67M vertices, 2.1e9 entries)
  // this is ~183 GB, above the measured peak of ~170 GB.
  const int64_t n = h->n;
  const int64_t nnz = h->nnz + 2 * n_ins;
  const int64_t E = 2 * (n_del + n_ins);
  const int64_t async_tables = (int64_t)kDefaultAsyncWaves * 2 * kHubDeg * 12;
  const int64_t need = 211 * n + 80 * nnz + 68 * E + async_tables;
  int64_t held = (int64_t)h->w.held();
  for (const DBuf *b : {&h->g_off, &h->g_idx, &h->g_w, &h->g_crow, &h->t_off, &h->t_idx, &h->t_w, &h->C, &h->K,
                        &h->Sig})
    held += (int64_t)b->cap;
  *bytes = std::max<int64_t>(0, need - held);
  return LEIDEN_OK;
}

leiden_status leiden_mark_affected(leiden_handle *h, const leiden_batch *batch, int32_t mode, uint8_t *affected,
                                   uint8_t *in_range, uint8_t *changed, void *stream) {
  if (!h || !batch) return LEIDEN_EINVAL;
  if (mode != LEIDEN_ND && mode != LEIDEN_DS && mode != LEIDEN_DF) return LEIDEN_EINVAL;
  if (!batch_pointers_ok(batch)) return LEIDEN_EINVAL;
  if (!h->has_state) {
    h->w.err = "marking before leiden_static or leiden_set_state";
    return LEIDEN_ESTATE;
  }
  Ctx x{&h->w, (hipStream_t)stream};
  return run_handle(h, x, [&] {
    const int64_t n = h->n;
    BatchArgs b;
    const int64_t nnz_new = stage_batch(x, h, *batch, b);
    // G^t lives in the spare CSR; the handle's graph and state are untouched
    const int64_t nch = ceil_div(std::max<int64_t>(nnz_new, 1), kChunk);
    int32_t *crow = x.get<int32_t>(Q_crow, nch + 2);
    chunk_start_rows((const int64_t *)h->t_off.p, n, nnz_new, crow, x.s);
    x.launched("chunk_start_rows");
    const Level gt{n, nnz_new, (const int64_t *)h->t_off.p, (const int32_t *)h->t_idx.p,
                   (const float *)h->t_w.p, crow};
    uint8_t *dV = x.get<uint8_t>(L_U, n);
    uint8_t *rng = x.get<uint8_t>(L_rng, n);
    uint8_t *dC = x.get<uint8_t>(L_dC, n);
    MarkArgs m;
    mark_batch(x, h, mode, b, gt, dV, rng, dC, m);
    if (affected) x.copy(affected, (const uint8_t *)dV, n);
    if (in_range) x.copy(in_range, (const uint8_t *)rng, n);
    if (changed) x.copy(changed, (const uint8_t *)dC, n);
    x.check(hipStreamSynchronize(x.s), "sync");
  });
}

leiden_status leiden_modularity(int64_t n, const int64_t *offsets, const int32_t *indices, const float *weights,
                                const int32_t *membership, double *q_out, void *stream) {
  if (n < 0 || !q_out || (n > 0 && (!offsets || !membership))) return LEIDEN_EINVAL;
  Workspace w;
  Ctx x{&w, (hipStream_t)stream};
  const leiden_status st = run_guarded(w, [&] {
    if (n == 0) { *q_out = 0.0; return; }
    const int64_t nnz = x.read(offsets + n);
    if (nnz > 0 && (!indices || !weights)) x.invalid("null edge arrays");
    DevScal *sc = x.scal();
    x.zero(&sc->err, 1);
    check_labels(membership, n, n, &sc->err, x.s);
    x.launched("check_labels");
    if (x.read(&sc->err)) x.invalid("membership label out of range");
    int32_t *crow = x.get<int32_t>(Q_crow, ceil_div(std::max<int64_t>(nnz, 1), kChunk) + 2);
    chunk_start_rows(offsets, n, nnz, crow, x.s);
    Level g{n, nnz, offsets, indices, weights, crow};
    *q_out = modularity_dev(x, g, membership);
  });
  w.release(x.s);
  return st;
}

leiden_status leiden_aggregate(int64_t n, const int64_t *offsets, const int32_t *indices, const float *weights,
                               const int32_t *membership, int64_t ncomm, int64_t *out_offsets,
                               int32_t *out_indices, float *out_weights, int64_t *nnz_out, void *stream) {
  if (n < 0 || ncomm < 0 || !nnz_out || !out_offsets || (n > 0 && (!offsets || !membership))) return LEIDEN_EINVAL;
  Workspace w;
  Ctx x{&w, (hipStream_t)stream};
  const leiden_status st = run_guarded(w, [&] {
    const int64_t nnz = (n > 0) ? x.read(offsets + n) : 0;
    DevScal *sc = x.scal();
    x.zero(&sc->err, 1);
    check_labels(membership, n, ncomm, &sc->err, x.s);
    x.launched("check_labels");
    if (x.read(&sc->err)) x.invalid("membership label outside [0, ncomm)");
    int32_t *crow = x.get<int32_t>(Q_crow, ceil_div(std::max<int64_t>(nnz, 1), kChunk) + 2);
    chunk_start_rows(offsets, n, nnz, crow, x.s);
    Level g{n, nnz, offsets, indices, weights, crow};
    const Level o = aggregate_level(x, g, membership, ncomm, 0, nullptr);
    x.copy(out_offsets, o.off, ncomm + 1);
    if (o.nnz > 0) {
      if (!out_indices || !out_weights) x.invalid("null output arrays");
      x.copy(out_indices, o.idx, o.nnz);
      x.copy(out_weights, o.w, o.nnz);
    }
    *nnz_out = o.nnz;
    x.check(hipStreamSynchronize(x.s), "sync");
  });
  w.release(x.s);
  return st;
}

leiden_status leiden_get_graph(leiden_handle *h, int64_t *offsets, int32_t *indices, float *weights,
                               int64_t *nnz, void *stream) {
  if (!h) return LEIDEN_EINVAL;
  Ctx x{&h->w, (hipStream_t)stream};
  return run_handle(h, x, [&] {
    if (nnz) *nnz = h->nnz;
    if (offsets) x.copy(offsets, (const int64_t *)h->g_off.p, h->n + 1);
    if (indices) x.copy(indices, (const int32_t *)h->g_idx.p, h->nnz);
    if (weights) x.copy(weights, (const float *)h->g_w.p, h->nnz);
    x.check(hipStreamSynchronize(x.s), "sync");
  });
}

leiden_status leiden_get_state(leiden_handle *h, int32_t *membership, double *K, double *Sigma, double *m2,
                               void *stream) {
  if (!h) return LEIDEN_EINVAL;
  if (!h->has_state) return LEIDEN_ESTATE;
  Ctx x{&h->w, (hipStream_t)stream};
  return run_handle(h, x, [&] {
    if (membership) x.copy(membership, (const int32_t *)h->C.p, h->n);
    if (K) x.copy(K, (const double *)h->K.p, h->n);
    if (Sigma) x.copy(Sigma, (const double *)h->Sig.p, h->n);
    if (m2) *m2 = h->M2;
    x.check(hipStreamSynchronize(x.s), "sync");
  });
}

leiden_status leiden_set_state(leiden_handle *h, const int32_t *membership, void *stream) {
  if (!h || (h->n > 0 && !membership)) return LEIDEN_EINVAL;
  Ctx x{&h->w, (hipStream_t)stream};
  return run_handle(h, x, [&] {
    const int64_t n = h->n;
    DevScal *sc = x.scal();
    x.zero(&sc->err, 1);
    check_labels(membership, n, n, &sc->err, x.s);
    x.launched("check_labels");
    if (x.read(&sc->err)) x.invalid("membership label out of range");
    x.ensure(h->C, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
    x.ensure(h->K, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
    x.ensure(h->Sig, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
    const Level g = handle_level(h);
    x.copy((int32_t *)h->C.p, membership, n);
    x.zero((double *)h->K.p, n);
    row_sums(g.off, g.w, n, g.nnz, g.crow, (double *)h->K.p, x.s);
    x.zero((double *)h->Sig.p, n);
    scatter_add((const double *)h->K.p, (const int32_t *)h->C.p, n, (double *)h->Sig.p, x.s);
    x.zero(sc->acc, 4);
    modularity_comm((const double *)h->K.p, n, sc->acc, x.s);
    x.launched("set_state");
    h->M2 = x.read(&sc->acc[1]);
    h->has_state = true;
  });
}

}  // extern "C"
