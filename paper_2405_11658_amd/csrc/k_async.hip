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
// Sigma atomics, neighbours marked unprocessed.  Vertices of higher degree are
// handled before the sweep by the multi-workgroup hub kernels.
//
// Refinement follows the same scheme: an isolated vertex of a changed bound
// (Sigma of its community equal to its own K) looks for the best community
// inside its bound, claims its own community with a compare-and-swap of
// Sigma from K_i to 0, and joins the target if the target's representative
// still holds its label.
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
__device__ __forceinline__ uint8_t ld_u8(const uint8_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u8(uint8_t *p, uint8_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_int(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// completes this wavefront's outstanding memory operations before the next
// ones (the table is written and read by different lanes of the wavefront)
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t table_cap(int64_t deg) {
  uint32_t c = 2;
  while (c < 2 * (uint64_t)deg) c <<= 1;
  return c;
}

// One wavefront's table: LDS for small degrees, its global region otherwise.
struct WaveTable {
  int *keys;
  double *vals;
  uint32_t mask;
  bool global;
};

__device__ __forceinline__ WaveTable wave_table(int *lk, double *lv, int *gk, double *gv, int64_t deg,
                                                int ldscap) {
  WaveTable t;
  const uint32_t cap = table_cap(deg);
  t.global = cap > (uint32_t)ldscap;
  t.keys = t.global ? gk : lk;
  t.vals = t.global ? gv : lv;
  t.mask = cap - 1;
  for (uint32_t s = lane(); s < cap; s += kWave) { t.keys[s] = kEmpty; t.vals[s] = 0.0; }
  wave_fence();
  return t;
}

__device__ __forceinline__ int tkey(const WaveTable &t, uint32_t s) { return t.global ? ld_int(&t.keys[s]) : t.keys[s]; }
__device__ __forceinline__ double tval(const WaveTable &t, uint32_t s) {
  return t.global ? ld_dbl(&t.vals[s]) : t.vals[s];
}

// Weight to community d held in the table (0 if absent); all lanes return it.
__device__ __forceinline__ double own_weight(const WaveTable &t, int d) {
  double b = 0.0;
  for (uint32_t s = lane(); s <= t.mask; s += kWave)
    if (tkey(t, s) == d) b = tval(t, s);
  return group_sum<kWave>(b);  // at most one lane holds a non-zero term
}

// Best positive-gain community other than d; (0, kNoComm) if none.
__device__ __forceinline__ void best_move(const WaveTable &t, double M2, int d, double b, double Ki, double Sd,
                                          const double *Sig, double &bg, int &bc) {
  bg = 0.0;
  bc = kNoComm;
  for (uint32_t s = lane(); s <= t.mask; s += kWave) {
    const int c = tkey(t, s);
    if (c == kEmpty || c == d) continue;
    const double x = move_score(M2, tval(t, s), b, Ki, ld_dbl(&Sig[c]), Sd);
    if (x > 0.0 && better(x, c, bg, bc)) { bg = x; bc = c; }
  }
  group_argmax<kWave>(bg, bc);
}

// First position of the next chunk of kAsyncChunk list positions for the
// calling wavefront (uniform value); chunks are taken in ascending order.
__device__ __forceinline__ int64_t grab(unsigned long long *next) {
  unsigned long long base = 0;
  if (lane() == 0) base = atomicAdd(next, (unsigned long long)kAsyncChunk);
  return (int64_t)__shfl(base, 0);
}

template <int WPB, int LDSCAP>
__global__ __launch_bounds__(256) void k_move_async(MoveArgs a) {
  __shared__ int skeys[WPB][LDSCAP];
  __shared__ double svals[WPB][LDSCAP];
  const int wv = threadIdx.x / kWave;
  const int64_t gw = (int64_t)blockIdx.x * WPB + wv;
  int *gk = a.akeys + gw * kHubDeg * 2;
  double *gv = a.avals + gw * kHubDeg * 2;
  double gsum = 0.0;
  long long mv = 0;
  for (;;) {
    const int64_t base = grab(a.anext);
    if (base >= a.alen) break;
    // each lane fetches the state of one vertex of the chunk; unprocessed
    // candidates are claimed (marked processed) at once and then handled one
    // after another by the whole wavefront
    const int64_t p = base + lane();
    int v = 0, dv = 0;
    int64_t e0v = 0, e1v = 0;
    double kv = 0.0;
    bool cand = false;
    if (p < a.alen) {
      v = a.alist[p];
      e0v = a.off[v];
      e1v = a.off[v + 1];
      cand = e1v - e0v <= kHubDeg && a.rng[v] && ld_u8(&a.U[v]);
      if (cand) {
        st_u8(&a.U[v], 0);
        dv = a.C[v];  // only this wavefront writes C[v] during the sweep
        kv = a.K[v];
      }
    }
    unsigned long long m = __ballot(cand);
    while (m) {
      const int k = __ffsll(m) - 1;
      m &= m - 1;
      const int i = __shfl(v, k);
      const int64_t e0 = __shfl(e0v, k), e1 = __shfl(e1v, k);
      const int d = __shfl(dv, k);
      const double Ki = __shfl(kv, k);
      WaveTable t = wave_table(skeys[wv], svals[wv], gk, gv, e1 - e0, LDSCAP);
      for (int64_t e = e0 + lane(); e < e1; e += kWave) {
        const int j = a.idx[e];
        if (j != i) table_add(t.keys, t.vals, t.mask, ld_int(&a.C[j]), (double)a.w[e]);
      }
      wave_fence();
      const double b = own_weight(t, d);
      double bg;
      int bc;
      best_move(t, a.M2, d, b, Ki, ld_dbl(&a.Sig[d]), a.Sig, bg, bc);
      if (bc == kNoComm) continue;
      if (lane() == 0) {
        st_int(&a.C[i], bc);
        unsafeAtomicAdd(&a.Sig[d], -Ki);
        unsafeAtomicAdd(&a.Sig[bc], Ki);
        if (a.track) { st_u8(&a.dC[d], 1); st_u8(&a.dC[bc], 1); }
        gsum += bg;
        mv += 1;
      }
      for (int64_t e = e0 + lane(); e < e1; e += kWave) {
        const int j = a.idx[e];
        if (j != i) st_u8(&a.U[j], 1);
      }
    }
  }
  if (lane() == 0) {
    if (gsum != 0.0) unsafeAtomicAdd(a.gain, gsum);
    if (mv) atomicAdd(a.moves, (unsigned long long)mv);
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
  launch_async(k_move_async<4, 512>, k_move_async<2, 2048>, a, waves, wide, s);
}

template <int WPB, int LDSCAP>
__global__ __launch_bounds__(256) void k_refine_async(RefineArgs a) {
  __shared__ int skeys[WPB][LDSCAP];
  __shared__ double svals[WPB][LDSCAP];
  const int wv = threadIdx.x / kWave;
  const int64_t gw = (int64_t)blockIdx.x * WPB + wv;
  int *gk = a.akeys + gw * kHubDeg * 2;
  double *gv = a.avals + gw * kHubDeg * 2;
  for (;;) {
    const int64_t base = grab(a.anext);
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
      cand = e1v - e0v <= kHubDeg && a.dC[cbv];
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
      const int i = __shfl(v, k);
      const int c = __shfl(cv, k);
      const double Ki = __shfl(kv, k);
      const int cb = __shfl(cbv, k);
      const int64_t e0 = __shfl(e0v, k), e1 = __shfl(e1v, k);
      WaveTable t = wave_table(skeys[wv], svals[wv], gk, gv, e1 - e0, LDSCAP);
      for (int64_t e = e0 + lane(); e < e1; e += kWave) {
        const int j = a.idx[e];
        if (j != i && a.CB[j] == cb) table_add(t.keys, t.vals, t.mask, ld_int(&a.C[j]), (double)a.w[e]);
      }
      wave_fence();
      const double b = own_weight(t, c);
      double bg;
      int bc;
      best_move(t, a.M2, c, b, Ki, Ki, a.Sig, bg, bc);
      if (bc == kNoComm) continue;
      if (lane() == 0 && ld_int(&a.C[bc]) == bc) {
        // claim the singleton: Sigma[c] K_i -> 0 fails if someone joined it
        unsigned long long *sc = (unsigned long long *)&a.Sig[c];
        const unsigned long long want = __double_as_longlong(Ki);
        if (atomicCAS(sc, want, 0ull) == want) {
          unsafeAtomicAdd(&a.Sig[bc], Ki);
          st_int(&a.C[i], bc);
        }
      }
    }
  }
}

void refine_async(const RefineArgs &a, int waves, bool wide, hipStream_t s) {
  launch_async(k_refine_async<4, 512>, k_refine_async<2, 2048>, a, waves, wide, s);
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

// Hubs of slice a.s enter the frontier: processed flag cleared, proposal
// reset, in-range ones listed in bucket kNB-1 of the slice and flagged act.
__global__ void k_hub_frontier(MoveArgs a) {
  int32_t *cnt = a.counts + a.s * kNB + (kNB - 1);
  int32_t *list = a.lists + a.region[a.s * kNB + (kNB - 1)];
  for (int64_t h = a.hbeg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < a.hend;
       h += (int64_t)gridDim.x * blockDim.x) {
    const int i = a.hp.hubv[h];
    a.prop[i] = -1;
    const bool go = a.U[i] && a.rng[i];
    a.U[i] = 0;
    a.act[i] = go;
    if (go) list[atomicAdd(cnt, 1)] = i;
  }
}
void move_hub_frontier(const MoveArgs &a, hipStream_t s) {
  if (a.hend > a.hbeg) hipLaunchKernelGGL(k_hub_frontier, flat_grid(a.hend - a.hbeg), 256, 0, s, a);
}

}  // namespace lk
