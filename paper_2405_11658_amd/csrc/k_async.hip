// Asynchronous local-moving and refinement sweeps (the default fast path).
//
// The paper runs Alg. "leidenMove" and Alg. "leidenRefine" with many threads
// that read the live membership and community weights and apply their moves
// at once (Sec. 4.6: asynchronous, with atomics on Sigma).  Here a fixed
// number of wavefronts sweep the vertex ids in ascending order, each taking
// the next chunk of ids from a global counter; a wavefront processes the
// vertices of its chunk one after another, so the vertices in flight at any
// time are at most one per wavefront.  Every vertex reads the current C and
// Sigma (agent-scope loads, not a stale L1 line), builds its neighbour
// community table in LDS (degree <= 256) or in a global-memory region of the
// wavefront (degree <= 2048), and applies its best move immediately: C store,
// Sigma atomics, neighbours marked unprocessed.  Changes to the Sigma of the
// few communities holding a large share of the weight are summed per
// wavefront and added every few chunks (Pend below).  Vertices of higher
// degree are handled before the sweep by the multi-workgroup hub kernels.
//
// Refinement follows the same scheme: an isolated vertex of a changed bound
// (Sigma of its community equal to its own K) looks for the best community
// inside its bound, claims its own community with a compare-and-swap of
// Sigma from K_i to 0, and joins the target if the target's representative
// still holds its label (checked only while the target may still be a
// singleton).
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

// Two shapes: 4 wavefronts per workgroup with 512 LDS table slots each
// (degree <= 256 in LDS), or 2 with 2048 slots (degree <= 1024 in LDS) for
// levels whose vertices have high average degree.
constexpr int kAsyncWaves = 4;

__device__ __forceinline__ int ld_int(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dbl(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Reads of neighbour communities and community totals.  CA = false:
// agent-scope loads, which always see the latest value of any wavefront on
// the device.  CA = true (levels whose state is many times the size of an
// XCD's L2): workgroup-scope loads, which may be served by this XCD's
// caches; a line there is evicted within microseconds by the level's random
// traffic, so a value is at most that stale - the same order as the
// staleness the vertices in flight already see - and the loads avoid the
// memory-side round trip that bounds the sweep.
template <bool CA>
__device__ __forceinline__ int ld_c(const int32_t *p) {
  if (CA) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool CA>
__device__ __forceinline__ double ld_s(const double *p) {
  if (CA) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool CA>
__device__ __forceinline__ unsigned long long ld_p(const unsigned long long *p) {
  if (CA) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint8_t ld_u8(const uint8_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u8(uint8_t *p, uint8_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_int(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Completes this wavefront's outstanding memory operations before the next
// ones (a global-memory table is written and read by different lanes).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}
// Orders the wavefront's LDS accesses only: LDS executes one wavefront's
// instructions in issue order, so a compiler barrier suffices for an LDS
// table that only this wavefront uses, and outstanding global stores (the
// previous vertex's move and marks) are not waited for.
__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t table_cap(int64_t deg) {
  uint32_t c = 2;
  while (c < 2 * (uint64_t)deg) c <<= 1;
  return c;
}

// One wavefront's table: LDS for small degrees, its global region otherwise.
// An LDS table is kept clear between vertices: the slots a vertex takes are
// listed (slot index, in insertion order) and only those are scanned and
// reset, so a vertex costs O(distinct neighbour communities), not O(capacity).
// A global table is cleared and scanned in full.
struct WaveTable {
  int *keys;
  double *vals;
  uint32_t mask;
  bool global;
  uint16_t *list;  // LDS only
  int *cnt;        // LDS only: length of list
};

// Sigma updates of popular communities held back by one wavefront.  Every
// wavefront adds into the few communities that hold a large share of the
// level's weight (on RMAT graphs most moves and joins involve them), and
// device-scope atomics on one address are performed one after another at
// the memory side; a wavefront waits for its own before its next load, so
// the sweep would run at the pace of that one address.  A wavefront
// therefore sums its changes to such a community here while the sum stays
// below kHotEps / W of the community's Sigma (W wavefronts in the sweep, so
// all held-back changes together stay below kHotEps of it), and adds it
// with one atomic when it would exceed that, every kGrabChunks chunks, and
// when the list is full.
constexpr int kPend = 16;
constexpr double kHotShare = 1.0 / 4096;  // popular: Sigma >= this share of 2m
constexpr double kHotEps = 1.0 / 64;
struct Pend {
  int c[kPend];
  double d[kPend];
  int n;
};

// LDS area of one wavefront for capacity LDSCAP.
template <int LDSCAP>
struct WaveLds {
  int keys[LDSCAP];
  double vals[LDSCAP];
  uint16_t list[LDSCAP / 2];
  int cnt;
  Pend pend;
};

template <int LDSCAP>
__device__ __forceinline__ void lds_table_init(WaveLds<LDSCAP> &l) {
  for (int s = lane(); s < LDSCAP; s += kWave) { l.keys[s] = kEmpty; l.vals[s] = 0.0; }
  if (lane() == 0) { l.cnt = 0; l.pend.n = 0; }
  lds_fence();
}

// Adds the held-back deltas to Sigma (one atomic per community, from
// different lanes) and empties the list.
__device__ __forceinline__ void pend_flush(Pend &p, double *Sig) {
  const int n = p.n;
  if (lane() < n) unsafeAtomicAdd(&Sig[p.c[lane()]], p.d[lane()]);
  lds_fence();
  if (lane() == 0) p.n = 0;
  lds_fence();
}

// Holds back Sigma[c] += x (c, x and lim uniform over the wavefront): the
// community's held-back sum is added at once when its magnitude would
// exceed lim.
__device__ __forceinline__ void pend_add(Pend &p, double *Sig, int c, double x, double lim) {
  int n = p.n;
  const unsigned long long hit = __ballot(lane() < n && p.c[lane()] == c);
  if (hit) {
    if (lane() == 0) {
      const int h = __ffsll(hit) - 1;
      const double d = p.d[h] + x;
      if (fabs(d) > lim) {
        unsafeAtomicAdd(&Sig[c], d);
        p.d[h] = 0.0;
      } else {
        p.d[h] = d;
      }
    }
  } else if (fabs(x) > lim) {
    if (lane() == 0) unsafeAtomicAdd(&Sig[c], x);
  } else {
    if (n == kPend) {
      pend_flush(p, Sig);
      n = 0;
    }
    if (lane() == 0) {
      p.c[n] = c;
      p.d[n] = x;
      p.n = n + 1;
    }
  }
  lds_fence();
}

template <int LDSCAP>
__device__ __forceinline__ WaveTable wave_table(WaveLds<LDSCAP> &l, int *gk, double *gv, int64_t deg) {
  WaveTable t;
  const uint32_t cap = table_cap(deg);
  t.global = cap > (uint32_t)LDSCAP;
  t.mask = cap - 1;
  if (t.global) {
    t.keys = gk;
    t.vals = gv;
    t.list = nullptr;
    t.cnt = nullptr;
    for (uint32_t s = lane(); s < cap; s += kWave) { gk[s] = kEmpty; gv[s] = 0.0; }
    wave_fence();
  } else {
    t.keys = l.keys;
    t.vals = l.vals;
    t.list = l.list;
    t.cnt = &l.cnt;
  }
  return t;
}

// Adds w to key's slot; a slot newly taken in an LDS table is listed.
__device__ __forceinline__ void tab_add(const WaveTable &t, int key, double w) {
  if (t.global) {
    table_add(t.keys, t.vals, t.mask, key, w);
    return;
  }
  uint32_t h = mix32((uint32_t)key) & t.mask;
  for (uint32_t probe = 0; probe <= t.mask; ++probe) {
    const int k = __atomic_load_n(&t.keys[h], __ATOMIC_RELAXED);
    if (k == key) { atomicAdd(&t.vals[h], w); return; }
    if (k == kEmpty) {
      const int old = atomicCAS(&t.keys[h], kEmpty, key);
      if (old == kEmpty) {
        atomicAdd(&t.vals[h], w);
        t.list[atomicAdd(t.cnt, 1)] = (uint16_t)h;
        return;
      }
      if (old == key) { atomicAdd(&t.vals[h], w); return; }
    }
    h = (h + 1) & t.mask;
  }
}

// Makes the table's inserts visible to all lanes.
__device__ __forceinline__ void tab_sync(const WaveTable &t) {
  if (t.global) wave_fence();
  else lds_fence();
}

// Returns an LDS table to the all-clear state.
__device__ __forceinline__ void tab_release(const WaveTable &t) {
  if (t.global) return;
  const int n = *t.cnt;
  for (int q = lane(); q < n; q += kWave) {
    const int s = t.list[q];
    t.keys[s] = kEmpty;
    t.vals[s] = 0.0;
  }
  lds_fence();
  if (lane() == 0) *t.cnt = 0;
  lds_fence();
}

// Edges per lane whose loads are issued together: the neighbour ids of
// kUnroll wavefront-widths of edges, then their communities, then the table
// inserts, so that a vertex costs two memory round trips per 256 edges
// instead of two per 64.
constexpr int kUnroll = 4;

// The first kUnroll * kWave edges of a vertex, this lane's share: neighbour
// id, weight and (once loaded) the neighbour's community, kEmpty for
// self-loops and for neighbours that do not count.  Loading the ids of
// kUnroll wavefront-widths first and then all their communities keeps a
// vertex at two memory round trips per kUnroll * kWave edges.
struct EdgeBatch {
  int j[kUnroll];
  float x[kUnroll];
  int c[kUnroll];
};

__device__ __forceinline__ void batch_ids(EdgeBatch &eb, const int32_t *idx, const float *w, int i, int64_t e0,
                                          int64_t e1) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int64_t e = e0 + u * kWave + lane();
    eb.j[u] = i;
    eb.x[u] = 0.0f;
    if (e < e1) { eb.j[u] = idx[e]; eb.x[u] = w[e]; }
  }
}

// Communities of the batch's neighbours; with CB given only neighbours whose
// CB equals cb count (both loads issued together).
template <bool CA>
__device__ __forceinline__ void batch_comms(EdgeBatch &eb, const int32_t *C, const int32_t *CB, int cb, int i) {
  int bj[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    eb.c[u] = kEmpty;
    bj[u] = cb;
    if (eb.j[u] != i) {
      eb.c[u] = ld_c<CA>(&C[eb.j[u]]);
      if (CB) bj[u] = CB[eb.j[u]];
    }
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u)
    if (bj[u] != cb) eb.c[u] = kEmpty;
}

// Refinement: communities and bounds of the batch's neighbours from the
// packed words (bound << 32 | community), one 8-byte load per neighbour.
template <bool CA>
__device__ __forceinline__ void batch_comms_packed(EdgeBatch &eb, const unsigned long long *CP, int cb, int i) {
  unsigned long long pk[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) pk[u] = eb.j[u] != i ? ld_p<CA>(&CP[eb.j[u]]) : ~0ull;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u)
    eb.c[u] = (eb.j[u] != i && (int)(pk[u] >> 32) == cb) ? (int)(uint32_t)pk[u] : kEmpty;
}

// Adds the edges [e0, e1) of vertex i to table t, keyed by the neighbour's
// current community: the first kUnroll * kWave from the loaded batch, the
// rest loaded here.  Returns (in all lanes) the weight to community d.
template <bool CA>
__device__ __forceinline__ double table_edges(const WaveTable &t, const EdgeBatch &eb, const int32_t *idx,
                                              const float *w, const int32_t *C, const int32_t *CB, int cb,
                                              int i, int d, int64_t e0, int64_t e1,
                                              const unsigned long long *CP = nullptr) {
  double own = 0.0;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    if (eb.c[u] == kEmpty) continue;
    tab_add(t, eb.c[u], (double)eb.x[u]);
    if (eb.c[u] == d) own += (double)eb.x[u];
  }
  for (int64_t base = e0 + kUnroll * kWave; base < e1; base += kUnroll * kWave) {
    EdgeBatch r;
    batch_ids(r, idx, w, i, base, e1);
    if (CP) batch_comms_packed<CA>(r, CP, cb, i);
    else batch_comms<CA>(r, C, CB, cb, i);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (r.c[u] == kEmpty) continue;
      tab_add(t, r.c[u], (double)r.x[u]);
      if (r.c[u] == d) own += (double)r.x[u];
    }
  }
  return group_sum<kWave>(own);
}

// A flag set by many wavefronts (a neighbour of many moving vertices; on
// RMAT graphs the hubs are neighbours of nearly all): with WG the store
// stays in this XCD's L2 until the line is written back (at the latest when
// the sweep ends), instead of a device-scope store that goes through to
// memory, where stores to one line are performed one after another and
// every wavefront waits for its own.  The flag is only ever set to one
// value, so a late write-back can only make a vertex be evaluated once more.
template <bool WG>
__device__ __forceinline__ void set_flag(uint8_t *p) {
  if (WG) __hip_atomic_store(p, (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else st_u8(p, 1);
}

// Marks the neighbours of vertex i unprocessed after it moved.  WG: as in
// set_flag, for sweeps of many wavefronts (a mark then reaches the other
// XCDs by the end of the sweep at the latest, so a vertex marked after it
// was passed over is evaluated in the next iteration, as it would be if
// marked after its turn); one wavefront alone keeps device-scope stores and
// so the serial sweep's order exactly.
template <bool WG>
__device__ __forceinline__ void mark_edges(uint8_t *U, const int32_t *idx, int i, int64_t e0, int64_t e1,
                                           const EdgeBatch &eb) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u)
    if (eb.j[u] != i) set_flag<WG>(&U[eb.j[u]]);
  for (int64_t e = e0 + kUnroll * kWave + lane(); e < e1; e += kWave) {
    const int j = idx[e];
    if (j != i) set_flag<WG>(&U[j]);
  }
}

// Scores up to kUnroll (community, weight) pairs per lane with their Sigma
// loads in flight together, keeping the best positive gain and the Sigma it
// was scored with.
template <bool CA>
__device__ __forceinline__ void score_batch(const int (&c)[kUnroll], const double (&x)[kUnroll], double M2,
                                            double b, double Ki, double Sd, const double *Sig, double &bg,
                                            int &bc, double &bs) {
  double S[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) S[u] = c[u] != kEmpty ? ld_s<CA>(&Sig[c[u]]) : 0.0;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    if (c[u] == kEmpty) continue;
    const double g = move_score(M2, x[u], b, Ki, S[u], Sd);
    if (g > 0.0 && better(g, c[u], bg, bc)) { bg = g; bc = c[u]; bs = S[u]; }
  }
}

// Best positive-gain community other than d; (0, kNoComm) if none, with the
// Sigma of the best as read for its score (bs).  An LDS table is read
// through its list of taken slots, a global one slot by slot.
template <bool CA>
__device__ __forceinline__ void best_move(const WaveTable &t, double M2, int d, double b, double Ki, double Sd,
                                          const double *Sig, double &bg, int &bc, double &bs) {
  bg = 0.0;
  bc = kNoComm;
  bs = 0.0;
  const uint32_t n = t.global ? t.mask + 1 : (uint32_t)*t.cnt;
  for (uint32_t q0 = 0; q0 < n; q0 += kUnroll * kWave) {
    int c[kUnroll];
    double x[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t q = q0 + u * kWave + lane();
      c[u] = kEmpty;
      x[u] = 0.0;
      if (q < n) {
        if (t.global) {
          c[u] = ld_int(&t.keys[q]);
          if (c[u] != kEmpty && c[u] != d) x[u] = ld_dbl(&t.vals[q]);
        } else {
          const int s = t.list[q];
          c[u] = t.keys[s];
          x[u] = t.vals[s];
        }
        if (c[u] == d) c[u] = kEmpty;
      }
    }
    score_batch<CA>(c, x, M2, b, Ki, Sd, Sig, bg, bc, bs);
  }
  const int lc = bc;
  group_argmax<kWave>(bg, bc);
  // table keys are distinct, so exactly one lane scored the winner
  const unsigned long long wl = __ballot(bc != kNoComm && lc == bc);
  bs = __shfl(bs, wl ? __ffsll(wl) - 1 : 0);
}

// A wavefront takes kGrabChunks chunks of kAsyncChunk list positions at a
// time from the global counter (one atomic per 256 vertices: every wavefront
// of the sweep takes its work from this one address, so its atomics must stay
// rare) and handles them in order.  Returns the first position of the
// calling wavefront's next chunk (uniform value); chunks are taken in
// ascending order.
constexpr int kGrabChunks = 4;
struct Grab {
  int64_t base = 0;
  int left = 0;
};
__device__ __forceinline__ int64_t grab(unsigned long long *next, Grab &g) {
  if (g.left == 0) {
    unsigned long long b = 0;
    if (lane() == 0) b = atomicAdd(next, (unsigned long long)kAsyncChunk * kGrabChunks);
    g.base = (int64_t)__shfl(b, 0);
    g.left = kGrabChunks;
  }
  const int64_t r = g.base;
  g.base += kAsyncChunk;
  --g.left;
  return r;
}

template <int WPB, int LDSCAP, bool CA>
__global__ __launch_bounds__(256) void k_move_async(MoveArgs a) {
  __shared__ WaveLds<LDSCAP> lds[WPB];
  const int wv = threadIdx.x / kWave;
  lds_table_init(lds[wv]);
  const int64_t gw = (int64_t)blockIdx.x * WPB + wv;
  int *gk = a.akeys + gw * kHubDeg * 2;
  double *gv = a.avals + gw * kHubDeg * 2;
  double gsum = 0.0;
  long long mv = 0;
  unsigned long long nv = 0, ne = 0;  // vertices evaluated, edges scanned
  Pend &pd = lds[wv].pend;
  const double hot = a.defer ? a.M2 * kHotShare : __builtin_inf();
  const double eps = kHotEps / ((double)gridDim.x * (blockDim.x / kWave));
  Grab gr;
  for (;;) {
    if (gr.left == 0) pend_flush(pd, a.Sig);
    const int64_t base = grab(a.anext, gr);
    if (base >= a.alen) break;
    // each lane fetches the state of one vertex of the chunk; the chunk's
    // unprocessed vertices are then handled one after another by the whole
    // wavefront, in list order.  A vertex is marked processed at its turn, and
    // after a move the flags of the chunk's later vertices are read again, so
    // that one wavefront alone follows the serial sweep exactly (a vertex
    // re-marked by an earlier vertex of its chunk is handled in the same
    // iteration).
    const int64_t p = base + lane();
    int v = 0, dv = 0;
    int64_t e0v = 0, e1v = 0;
    double kv = 0.0;
    bool elig = false;
    if (p < a.alen) {
      v = a.alist[p];
      e0v = a.off[v];
      e1v = a.off[v + 1];
      elig = e1v - e0v <= a.hubdeg && a.rng[v];
      if (elig) {
        dv = a.C[v];  // only this wavefront writes C[v] during the sweep
        kv = a.K[v];
      }
    }
    unsigned long long m = __ballot(elig && ld_u8(&a.U[v]));
    while (m) {
      const int k = __ffsll(m) - 1;
      m &= ~((2ull << k) - 1ull);  // positions after k
      const int i = __shfl(v, k), d = __shfl(dv, k);
      const int64_t e0 = __shfl(e0v, k), e1 = __shfl(e1v, k);
      const double Ki = __shfl(kv, k);
      if (lane() == 0) st_u8(&a.U[i], 0);
      nv += 1;
      ne += (unsigned long long)(e1 - e0);
      EdgeBatch eb;
      batch_ids(eb, a.idx, a.w, i, e0, e1);
      batch_comms<CA>(eb, a.C, nullptr, 0, i);
      WaveTable t = wave_table(lds[wv], gk, gv, e1 - e0);
      const double b = table_edges<CA>(t, eb, a.idx, a.w, a.C, nullptr, 0, i, d, e0, e1);
      tab_sync(t);
      double bg, bs;
      int bc;
      const double Sd = ld_s<CA>(&a.Sig[d]);
      best_move<CA>(t, a.M2, d, b, Ki, Sd, a.Sig, bg, bc, bs);
      tab_release(t);
      if (bc == kNoComm) continue;
      if (lane() == 0) {
        st_int(&a.C[i], bc);
        if (Sd < hot) unsafeAtomicAdd(&a.Sig[d], -Ki);
        if (bs < hot) unsafeAtomicAdd(&a.Sig[bc], Ki);
        if (a.track) {
          if (a.defer) { set_flag<true>(&a.dC[d]); set_flag<true>(&a.dC[bc]); }
          else { st_u8(&a.dC[d], 1); st_u8(&a.dC[bc], 1); }
        }
        gsum += bg;
        mv += 1;
      }
      if (Sd >= hot) pend_add(pd, a.Sig, d, -Ki, Sd * eps);
      if (bs >= hot) pend_add(pd, a.Sig, bc, Ki, bs * eps);
      if (lane() == k) dv = bc;
      if (a.defer) mark_edges<true>(a.U, a.idx, i, e0, e1, eb);
      else mark_edges<false>(a.U, a.idx, i, e0, e1, eb);
      // the move may have marked later vertices of the chunk unprocessed
      wave_fence();
      m = __ballot(lane() > k && elig && ld_u8(&a.U[v]));
    }
  }
  pend_flush(pd, a.Sig);
  if (lane() == 0) {
    if (gsum != 0.0) unsafeAtomicAdd(a.gain, gsum);
    if (mv) atomicAdd(a.moves, (unsigned long long)mv);
    if (a.sweep_work && nv) {
      atomicAdd(&a.sweep_work[0], nv);
      atomicAdd(&a.sweep_work[1], ne);
    }
  }
}

// `waves` is rounded down to whole workgroups (at least one, possibly
// smaller); wide = the 2-wavefront, 2048-slot shape.
template <class Args, class K4, class K2>
static void launch_async(K4 k4, K2 k2, const Args &a, int waves, bool wide, hipStream_t s) {
  if (a.n <= 0 || waves <= 0) return;
  const int wpb = wide ? 2 : kAsyncWaves;
  const int per = waves < wpb ? waves : wpb;
  if (wide) hipLaunchKernelGGL(k2, waves / per, per * kWave, 0, s, a);
  else hipLaunchKernelGGL(k4, waves / per, per * kWave, 0, s, a);
}

void move_async(const MoveArgs &a, int waves, bool wide, hipStream_t s) {
  if (a.cached) launch_async(k_move_async<4, 512, true>, k_move_async<2, 2048, true>, a, waves, wide, s);
  else launch_async(k_move_async<4, 512, false>, k_move_async<2, 2048, false>, a, waves, wide, s);
}

constexpr int kRefineTries = 4;  // evaluations of a refinement candidate whose target emptied

// Sigma[target] += x unless the target community had become empty (Sigma
// 0: its last member left), in which case the addition is taken back; one
// atomic add (not a compare-and-swap loop, which would serialise on popular
// targets).  Returns whether the merge happened.
__device__ __forceinline__ bool join_nonempty(double *sig, double x) {
  const double old = unsafeAtomicAdd(sig, x);
  if (old != 0.0) return true;
  unsafeAtomicAdd(sig, -x);
  return false;
}

template <int WPB, int LDSCAP, bool CA>
__global__ __launch_bounds__(256) void k_refine_async(RefineArgs a) {
  __shared__ WaveLds<LDSCAP> lds[WPB];
  const int wv = threadIdx.x / kWave;
  lds_table_init(lds[wv]);
  const int64_t gw = (int64_t)blockIdx.x * WPB + wv;
  int *gk = a.akeys + gw * kHubDeg * 2;
  double *gv = a.avals + gw * kHubDeg * 2;
  Pend &pd = lds[wv].pend;
  const double hot = a.defer ? a.M2 * kHotShare : __builtin_inf();
  const double eps = kHotEps / ((double)gridDim.x * (blockDim.x / kWave));
  unsigned long long nv = 0, ne = 0;  // candidate evaluations, edges scanned
  Grab gr;
  for (;;) {
    if (gr.left == 0) pend_flush(pd, a.Sig);
    const int64_t base = grab(a.anext, gr);
    if (base >= a.alen) break;
    // each lane fetches one vertex of the chunk: isolated vertices of a
    // changed bound are candidates (their isolation is confirmed again by the
    // compare-and-swap when they move)
    const int64_t p = base + lane();
    int v = 0, cv = 0, cbv = 0;
    int64_t e0v = 0, e1v = 0;
    double kv = 0.0;
    bool cand = false;
    if (p < a.alen) {
      v = a.alist[p];
      e0v = a.off[v];
      e1v = a.off[v + 1];
      cbv = a.CB[v];
      cand = e1v - e0v <= a.hubdeg && a.dC[cbv];
      if (cand) {
        cv = a.C[v];  // only this wavefront moves vertex v
        kv = a.K[v];
        cand = ld_dbl(&a.Sig[cv]) == kv;
      }
    }
    unsigned long long m = __ballot(cand);
    while (m) {
      const int k = __ffsll(m) - 1;
      m &= m - 1;
      const int i = __shfl(v, k), c = __shfl(cv, k), cb = __shfl(cbv, k);
      const int64_t e0 = __shfl(e0v, k), e1 = __shfl(e1v, k);
      const double Ki = __shfl(kv, k);
      // A target chosen from communities read while other wavefronts move
      // may empty before the merge (its representative joined another
      // community); the vertex then looks again with fresh labels instead of
      // staying alone.  Alone (one wavefront) this never happens: a table
      // only holds communities that have members.
      for (int attempt = 0; attempt < kRefineTries; ++attempt) {
        nv += 1;
        ne += (unsigned long long)(e1 - e0);
        EdgeBatch eb;
        batch_ids(eb, a.idx, a.w, i, e0, e1);
        batch_comms_packed<CA>(eb, a.CP, cb, i);
        WaveTable t = wave_table(lds[wv], gk, gv, e1 - e0);
        const double b = table_edges<CA>(t, eb, a.idx, a.w, a.C, a.CB, cb, i, c, e0, e1, a.CP);
        tab_sync(t);
        double bg, bs;
        int bc;
        best_move<CA>(t, a.M2, c, b, Ki, Ki, a.Sig, bg, bc, bs);
        tab_release(t);
        if (bc == kNoComm) break;
        // Every vertex of a changed bound starts alone, so a neighbour other
        // than bc itself seen in bc has joined bc; then bc's representative
        // is no longer isolated, can never leave, and bc can never empty: the
        // join needs neither the representative check nor the old total.
        bool seen = false;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) seen |= eb.c[u] == bc && eb.j[u] != bc;
        const bool held = __ballot(seen) != 0;
        int again = 0, joined = 0;
        if (lane() == 0) {
          if (!held && ld_int(&a.C[bc]) != bc) {
            again = 1;
          } else {
            // claim the singleton: Sigma[c] K_i -> 0 fails if someone joined it
            unsigned long long *sc = (unsigned long long *)&a.Sig[c];
            const unsigned long long want = __double_as_longlong(Ki);
            if (atomicCAS(sc, want, 0ull) == want) {
              if (held) {
                if (bs < hot) unsafeAtomicAdd(&a.Sig[bc], Ki);
                joined = 1;
              } else if (join_nonempty(&a.Sig[bc], Ki)) {
                joined = 1;
              } else {
                unsafeAtomicAdd(&a.Sig[c], Ki);  // the target emptied meanwhile: stay, look again
                again = 1;
              }
              if (joined) {
                st_int(&a.C[i], bc);
                __hip_atomic_store(&a.CP[i], ((unsigned long long)(uint32_t)cb << 32) | (uint32_t)bc,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              }
            }
          }
        }
        if (held && bs >= hot && __shfl(joined, 0)) pend_add(pd, a.Sig, bc, Ki, bs * eps);
        if (!__shfl(again, 0)) break;
      }
    }
  }
  pend_flush(pd, a.Sig);
  if (lane() == 0 && a.sweep_work && nv) {
    atomicAdd(&a.sweep_work[0], nv);
    atomicAdd(&a.sweep_work[1], ne);
  }
}

__global__ void k_pack_cb(const int32_t *C, const int32_t *CB, int64_t n, unsigned long long *CP) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    CP[i] = ((unsigned long long)(uint32_t)CB[i] << 32) | (uint32_t)C[i];
}
void pack_cb(const int32_t *C, const int32_t *CB, int64_t n, unsigned long long *CP, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pack_cb, flat_grid(n), 256, 0, s, C, CB, n, CP);
}

void refine_async(const RefineArgs &a, int waves, bool wide, hipStream_t s) {
  if (a.cached) launch_async(k_refine_async<4, 512, true>, k_refine_async<2, 2048, true>, a, waves, wide, s);
  else launch_async(k_refine_async<4, 512, false>, k_refine_async<2, 2048, false>, a, waves, wide, s);
}

__global__ void k_edge_flags(const int64_t *off, int64_t n, int32_t *flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = off[i + 1] > off[i];
}
void edge_flags(const int64_t *off, int64_t n, int32_t *flags, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_edge_flags, flat_grid(n), 256, 0, s, off, n, flags);
}
__global__ void k_edge_list(const int64_t *off, int64_t n, const int32_t *pos, int32_t *list) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (off[i + 1] > off[i]) list[pos[i]] = (int32_t)i;
}
void edge_list(const int64_t *off, int64_t n, const int32_t *pos, int32_t *list, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_edge_list, flat_grid(n), 256, 0, s, off, n, pos, list);
}

}  // namespace lk

