// Local-moving phase (Alg. "leidenMove" with "scanCommunities", self=false),
// executed on the GPU as sweeps over S vertex slices (hash of the id); the
// slices of an iteration run in order, each synchronously:
//   frontier  - unprocessed in-range vertices of the slice are marked
//               processed (vertex pruning) and bucketed by degree;
//   propose   - each frontier vertex builds its neighbour-community weight
//               table and picks the community of best Eq. 2 gain (strictly
//               positive, ties to the smaller id);
//   apply     - a proposal d -> c is dropped when a neighbour of the same
//               slice proposes the exact reverse move c -> d with priority
//               (larger gain, then smaller id); accepted moves update C,
//               Sigma (atomics), flag
//               source and target communities as changed (dynamic runs) and
//               mark the mover's neighbours unprocessed; dropped proposers stay
//               unprocessed.
// Degree buckets pick the table: registers of a 4/8/32-lane group (all-pairs
// combine), an LDS table per wavefront or workgroup, or a global-memory table
// per workgroup for hubs.
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

__device__ __forceinline__ int bucket_of_d(int64_t deg, int64_t hubdeg) {
  return deg > hubdeg ? 5 : deg <= 4 ? 0 : deg <= 8 ? 1 : deg <= 32 ? 2 : deg <= 256 ? 3 : 4;
}

// Keyed appends are aggregated per workgroup: a tile of kTile vertices is
// counted into LDS counters, one global atomic per non-empty key reserves
// the workgroup's range, and a second pass places the items.
constexpr int kTile = 4096;
constexpr int kMaxKeys = 2048;  // >= 256 slices * (kNB + 1)

__global__ __launch_bounds__(256) void k_slice_hist(const int64_t *off, int64_t n, int S, int64_t hubdeg,
                                                    int32_t *counts, int32_t *slice_cnt) {
  __shared__ int cnt[kMaxKeys];
  const int K = S * kNB + S;  // bucket keys, then slice keys
  for (int k = threadIdx.x; k < K; k += blockDim.x) cnt[k] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t deg = off[i + 1] - off[i];
    const int sl = slice_of(i, S);
    atomicAdd(&cnt[S * kNB + sl], 1);
    if (deg > 0) atomicAdd(&cnt[sl * kNB + bucket_of_d(deg, hubdeg)], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const int c = cnt[k];
    if (c) atomicAdd(k < S * kNB ? &counts[k] : &slice_cnt[k - S * kNB], c);
  }
}
void slice_hist(const int64_t *off, int64_t n, int S, int64_t hubdeg, int32_t *counts, int32_t *slice_cnt,
                hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_slice_hist, flat_grid(n, 256, 1024), 256, 0, s, off, n, S, hubdeg, counts, slice_cnt);
}

__global__ __launch_bounds__(256) void k_slice_scatter(int64_t n, int S, const int32_t *slice_off,
                                                       int32_t *slice_fill, int32_t *vbyslice) {
  __shared__ int cnt[kMaxKeys];
  __shared__ int base[kMaxKeys];
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < n; t0 += (int64_t)gridDim.x * kTile) {
    const int64_t t1 = min(t0 + (int64_t)kTile, n);
    for (int k = threadIdx.x; k < S; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) atomicAdd(&cnt[slice_of(i, S)], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
      const int c = cnt[k];
      base[k] = c ? atomicAdd(&slice_fill[k], c) : 0;
      cnt[k] = 0;
    }
    __syncthreads();
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
      const int sl = slice_of(i, S);
      vbyslice[slice_off[sl] + base[sl] + atomicAdd(&cnt[sl], 1)] = (int32_t)i;
    }
    __syncthreads();
  }
}
void slice_scatter(int64_t n, int S, const int32_t *slice_off, int32_t *slice_fill, int32_t *vbyslice,
                   hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_slice_scatter, flat_grid(ceil_div(n, kTile), 1, 2048), 256, 0, s, n, S,
                                slice_off, slice_fill, vbyslice);
}

// Frontier of slice s: its unprocessed vertices become processed; in-range
// ones with edges are bucketed by degree.  Proposals of the slice are reset.
__device__ __forceinline__ int frontier_key(const MoveArgs &a, int i) {
  if (!a.U[i] || !a.rng[i]) return -1;
  const int64_t deg = a.off[i + 1] - a.off[i];
  return deg > 0 ? bucket_of_d(deg, a.hubdeg) : -1;
}

__global__ __launch_bounds__(256) void k_frontier(MoveArgs a) {
  __shared__ int cnt[kNB];
  __shared__ int base[kNB];
  int32_t *counts = a.counts + a.s * kNB;
  const int32_t *region = a.region + a.s * kNB;
  for (int64_t t0 = a.vbeg + (int64_t)blockIdx.x * kTile; t0 < a.vend; t0 += (int64_t)gridDim.x * kTile) {
    const int64_t t1 = min(t0 + (int64_t)kTile, a.vend);
    if (threadIdx.x < kNB) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
      const int key = frontier_key(a, a.vbyslice[t]);
      if (key >= 0) atomicAdd(&cnt[key], 1);
    }
    __syncthreads();
    if (threadIdx.x < kNB) {
      const int c = cnt[threadIdx.x];
      base[threadIdx.x] = c ? atomicAdd(&counts[threadIdx.x], c) : 0;
      cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
      const int i = a.vbyslice[t];
      const int key = frontier_key(a, i);
      a.prop[i] = -1;
      a.U[i] = 0;
      if (a.act && a.off[i + 1] - a.off[i] > a.hubdeg) a.act[i] = key >= 0;
      if (key >= 0) a.lists[region[key] + base[key] + atomicAdd(&cnt[key], 1)] = i;
    }
    __syncthreads();
  }
}

// ---- propose: small-degree groups (deg <= G), all-pairs combine in registers
template <int G>
__global__ __launch_bounds__(256) void k_propose_small(MoveArgs a, int b) {
  const int count = a.counts[a.s * kNB + b];
  const int32_t *list = a.lists + a.region[a.s * kNB + b];
  const int gl = threadIdx.x & (G - 1);
  // the loop runs in step for the whole wavefront (collectives stay uniform)
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwave = (int64_t)gridDim.x * blockDim.x / kWave;
  const int gin = lane() / G;
  for (int64_t v0 = wave * (kWave / G); v0 < count; v0 += nwave * (kWave / G)) {
    const int64_t v = v0 + gin;
    const bool valid = v < count;
    const int i = valid ? list[v] : 0;
    int deg = 0, d = 0;
    int64_t e0 = 0;
    if (valid) {
      e0 = a.off[i];
      deg = (int)(a.off[i + 1] - e0);
      d = a.C[i];
    }
    int key = -1;
    float wt = 0.0f;
    if (gl < deg) {
      const int j = a.idx[e0 + gl];
      if (j != i) { key = a.C[j]; wt = a.w[e0 + gl]; }
    }
    double sum = 0.0;
    bool first = true;
#pragma unroll
    for (int s = 0; s < G; ++s) {
      const int ks = __shfl(key, s, G);
      const float ws = __shfl(wt, s, G);
      if (ks == key) {
        sum += (double)ws;
        if (s < gl) first = false;
      }
    }
    const double bown = group_sum<G>((key == d && first) ? sum : 0.0);
    double g = 0.0;
    int c = kNoComm;
    if (key >= 0 && key != d && first) {
      const double x = move_score(a.M2, sum, bown, a.K[i], a.Sig[key], a.Sig[d]);
      if (x > 0.0) { g = x; c = key; }
    }
    group_argmax<G>(g, c);
    if (valid && gl == 0) {
      a.from[i] = d;
      a.prop[i] = (c == kNoComm) ? -1 : c;
      a.gp[i] = g;
    }
  }
}


__device__ __forceinline__ uint32_t pow2_at_least(uint64_t x) {
  uint32_t c = 2;
  while (c < x) c <<= 1;
  return c;
}

// Team argmax over TEAM threads (TEAM = 64 or a multiple); result in t == 0.

// ---- propose: a team (wavefront or workgroup) per vertex, hash table of T
// slots per team in LDS.
template <int TEAM, int T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_propose_team(MoveArgs a, int b) {
  constexpr int NT = BLOCK / TEAM;
  __shared__ int skeys[NT * T];
  __shared__ double svals[NT * T];
  __shared__ double sb[NT];
  __shared__ double rg[BLOCK / kWave];
  __shared__ int rc[BLOCK / kWave];
  const int team = threadIdx.x / TEAM;
  const int t = threadIdx.x % TEAM;
  const int count = a.counts[a.s * kNB + b];
  const int32_t *list = a.lists + a.region[a.s * kNB + b];
  for (int64_t base = (int64_t)blockIdx.x * NT; base < count; base += (int64_t)gridDim.x * NT) {
    const int64_t v = base + team;
    const bool valid = v < count;
    const int i = valid ? list[v] : 0;
    int64_t e0 = 0, e1 = 0;
    int d = 0;
    if (valid) { e0 = a.off[i]; e1 = a.off[i + 1]; d = a.C[i]; }
    int *keys = skeys + team * T;
    double *vals = svals + team * T;
    const uint32_t mask = T - 1;
    for (uint32_t s = t; s <= mask; s += TEAM) { keys[s] = kEmpty; vals[s] = 0.0; }
    if (t == 0) sb[team] = 0.0;
    __syncthreads();
    if (valid) {
      for (int64_t e = e0 + t; e < e1; e += TEAM) {
        const int j = a.idx[e];
        if (j != i) table_add(keys, vals, mask, a.C[j], (double)a.w[e]);
      }
    }
    __syncthreads();
    if (valid)
      for (uint32_t s = t; s <= mask; s += TEAM)
        if (keys[s] == d) sb[team] = vals[s];
    __syncthreads();
    double bg = 0.0;
    int bc = kNoComm;
    if (valid) {
      const double bown = sb[team];
      const double Ki = a.K[i];
      const double Sd = a.Sig[d];
      for (uint32_t s = t; s <= mask; s += TEAM) {
        const int c = keys[s];
        if (c == kEmpty || c == d) continue;
        const double x = move_score(a.M2, vals[s], bown, Ki, a.Sig[c], Sd);
        if (x > 0.0 && better(x, c, bg, bc)) { bg = x; bc = c; }
      }
    }
    team_argmax<TEAM, BLOCK>(bg, bc, rg, rc);
    if (valid && t == 0) {
      a.from[i] = d;
      a.prop[i] = (bc == kNoComm) ? -1 : bc;
      a.gp[i] = bg;
    }
    __syncthreads();
  }
}

// ---- propose: hubs, several workgroups per vertex --------------------------
// gather: a workgroup merges one edge chunk of a frontier hub in an LDS
// table, then adds its distinct communities into the hub's global table (the
// hub's own community into `own`).
__global__ __launch_bounds__(256) void k_hub_gather(MoveArgs a) {
  constexpr int T = 2 * kHubEC;
  constexpr int PER = kHubEC / 256;  // edges per thread
  static_assert(kHubEC % 256 == 0, "edge chunk must be a multiple of the workgroup size");
  __shared__ int keys[T];
  __shared__ double vals[T];
  __shared__ int used[kHubEC];  // slots taken (at most one per edge)
  __shared__ int nused;
  const int64_t q = a.qbeg + blockIdx.x;
  const int h = a.hp.chub[q];
  const int i = a.hp.hubv[h];
  if (a.hub_front) {
    // The hub enters the frontier of its slice: every chunk takes the same
    // decision from the processed flag, which k_hub_rev clears; the first
    // chunk records it and resets the proposal.
    const bool go = a.U[i] && a.rng[i];
    if (q == a.hp.hch[h] && threadIdx.x == 0) {
      a.prop[i] = -1;
      a.act[i] = go;
      if (go) a.lists[a.region[a.s * kNB + (kNB - 1)] + atomicAdd(a.counts + a.s * kNB + (kNB - 1), 1)] = i;
    }
    if (!go) return;
  } else if (!a.act[i]) {
    return;
  }
  const int64_t e0 = a.off[i] + (q - a.hp.hch[h]) * kHubEC;
  const int64_t e1 = min(e0 + (int64_t)kHubEC, a.off[i + 1]);
  if (a.hub_scanned && threadIdx.x == 0) atomicAdd(a.hub_scanned, (unsigned long long)(e1 - e0));
  for (int s = threadIdx.x; s < T; s += blockDim.x) { keys[s] = kEmpty; vals[s] = 0.0; }
  if (threadIdx.x == 0) nused = 0;
  // this thread's edges: all ids first, then all communities
  int j[PER], c[PER];
  float x[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t e = e0 + threadIdx.x + u * 256;
    j[u] = i;
    x[u] = 0.0f;
    if (e < e1) { j[u] = a.idx[e]; x[u] = a.w[e]; }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) c[u] = j[u] != i ? a.C[j[u]] : kEmpty;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (c[u] != kEmpty) table_add(keys, vals, T - 1, c[u], (double)x[u]);
  __syncthreads();
  // list the taken slots, so that the merge into the hub's global table is
  // spread evenly over the threads
  for (int s0 = 0; s0 < T; s0 += blockDim.x) {
    const int s = s0 + threadIdx.x;
    const bool taken = keys[s] != kEmpty;
    const unsigned long long m = __ballot(taken);
    int base = 0;
    if (lane() == 0 && m) base = atomicAdd(&nused, (int)__popcll(m));
    base = __shfl(base, 0);
    if (taken) used[base + (int)__popcll(m & ((1ull << lane()) - 1ull))] = s;
  }
  __syncthreads();
  const int nu = nused;
  const int d = a.C[i];
  const int64_t t0 = a.hp.htab[h];
  const uint32_t mask = (uint32_t)(a.hp.hcap[h] - 1);
  for (int k = threadIdx.x; k < nu; k += blockDim.x) {
    const int s = used[k];
    const int cs = keys[s];
    if (cs == d) unsafeAtomicAdd(&a.hp.own[h], vals[s]);
    else table_add(a.hp.keys + t0, a.hp.vals + t0, mask, cs, vals[s]);
  }
}

// score: a workgroup scans one table segment of a frontier hub, frees the
// slots it reads, and leaves the segment's best (gain, community).
__global__ __launch_bounds__(256) void k_hub_score(MoveArgs a) {
  __shared__ double rg[256 / kWave];
  __shared__ int rc[256 / kWave];
  const int64_t q = a.gbeg + blockIdx.x;
  const int h = a.hp.shub[q];
  const int i = a.hp.hubv[h];
  if (!a.act[i]) return;
  const int64_t s0 = a.hp.htab[h] + (q - a.hp.hsg[h]) * kHubSeg;
  const int64_t s1 = s0 + min((int64_t)kHubSeg, a.hp.hcap[h]);
  const int d = a.C[i];
  const double Ki = a.K[i], Sd = a.Sig[d], bown = a.hp.own[h];
  double bg = 0.0;
  int bc = kNoComm;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
    const int c = a.hp.keys[s];
    if (c == kEmpty) continue;
    const double v = a.hp.vals[s];
    a.hp.keys[s] = kEmpty;
    a.hp.vals[s] = 0.0;
    const double x = move_score(a.M2, v, bown, Ki, a.Sig[c], Sd);
    if (x > 0.0 && better(x, c, bg, bc)) { bg = x; bc = c; }
  }
  team_argmax<256, 256>(bg, bc, rg, rc);
  if (threadIdx.x == 0) { a.hp.pg[q] = bg; a.hp.pc[q] = bc; }
}

// final: a wavefront per hub of the slice reduces the segment results.
__global__ __launch_bounds__(256) void k_hub_final(MoveArgs a) {
  const int64_t h = a.hbeg + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (h >= a.hend) return;  // uniform per wavefront
  const int i = a.hp.hubv[h];
  if (!a.act[i]) return;
  double bg = 0.0;
  int bc = kNoComm;
  for (int64_t q = a.hp.hsg[h] + lane(); q < a.hp.hsg[h + 1]; q += kWave)
    if (better(a.hp.pg[q], a.hp.pc[q], bg, bc)) { bg = a.hp.pg[q]; bc = a.hp.pc[q]; }
  group_argmax<kWave>(bg, bc);
  if (lane() == 0) {
    a.from[i] = a.C[i];
    a.prop[i] = (bc == kNoComm) ? -1 : bc;
    a.gp[i] = bg;
    a.hp.own[h] = 0.0;
    a.hp.flag[h] = 0;
  }
}

// ---- hub plan -------------------------------------------------------------------
// Each workgroup takes a contiguous range of vertices, counts its hubs per
// slice in LDS, reserves each slice's places with one global atomic and then
// writes them: one atomic per workgroup and slice instead of one per hub (a
// level has up to millions of hubs but only S counters, and device-scope
// atomics on one address are performed one after another).  S <= 256.
constexpr int kHubFindBlocks = 1024;
__global__ __launch_bounds__(256) void k_hub_find(const int64_t *off, int64_t n, int S, int64_t hubdeg,
                                                  const int32_t *hub_soff, int32_t *hub_fill, int32_t *hubv) {
  __shared__ int cnt[256];
  __shared__ int base[256];
  const int64_t per = ceil_div(n, (int64_t)gridDim.x);
  const int64_t v0 = (int64_t)blockIdx.x * per;
  const int64_t v1 = min(v0 + per, n);
  for (int k = threadIdx.x; k < S; k += blockDim.x) cnt[k] = 0;
  __syncthreads();
  for (int64_t i = v0 + threadIdx.x; i < v1; i += blockDim.x)
    if (off[i + 1] - off[i] > hubdeg) atomicAdd(&cnt[slice_of(i, S)], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < S; k += blockDim.x) {
    base[k] = cnt[k] ? atomicAdd(&hub_fill[k], cnt[k]) : 0;
    cnt[k] = 0;
  }
  __syncthreads();
  for (int64_t i = v0 + threadIdx.x; i < v1; i += blockDim.x) {
    if (off[i + 1] - off[i] <= hubdeg) continue;
    const int sl = slice_of(i, S);
    hubv[hub_soff[sl] + base[sl] + atomicAdd(&cnt[sl], 1)] = (int32_t)i;
  }
}
void hub_find(const int64_t *off, int64_t n, int S, int64_t hubdeg, const int32_t *hub_soff, int32_t *hub_fill,
              int32_t *hubv, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_hub_find, (int)std::min<int64_t>(kHubFindBlocks, ceil_div(n, (int64_t)256)), 256, 0, s,
                       off, n, S, hubdeg, hub_soff, hub_fill, hubv);
}

__global__ void k_hub_sizes(const int64_t *off, const int32_t *hubv, int64_t nhub, int64_t *nch, int64_t *ncap,
                            int64_t *nseg) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h <= nhub; h += (int64_t)gridDim.x * blockDim.x) {
    if (h == nhub) { nch[h] = 0; ncap[h] = 0; nseg[h] = 0; continue; }
    const int i = hubv[h];
    const int64_t deg = off[i + 1] - off[i];
    int64_t cap = kHubMinCap;
    while (cap < 2 * deg) cap <<= 1;
    nch[h] = ceil_div(deg, (int64_t)kHubEC);
    ncap[h] = cap;
    nseg[h] = ceil_div(cap, (int64_t)kHubSeg);
  }
}
void hub_sizes(const int64_t *off, const int32_t *hubv, int64_t nhub, int64_t *nch, int64_t *ncap, int64_t *nseg,
               hipStream_t s) {
  hipLaunchKernelGGL(k_hub_sizes, flat_grid(nhub + 1), 256, 0, s, off, hubv, nhub, nch, ncap, nseg);
}

// Table offsets counted from the start of each hub's slice: the slices run
// one after another and scoring frees every slot it reads, so all slices
// share one table area of the largest slice's size.
__global__ void k_hub_rel(int64_t *htab, int64_t nhub, const int32_t *hub_soff, int S, const int64_t *slice_base) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < nhub; h += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = S;  // the slice s with hub_soff[s] <= h < hub_soff[s + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (hub_soff[mid] <= h) lo = mid;
      else hi = mid;
    }
    htab[h] -= slice_base[lo];
  }
}
void hub_rel(int64_t *htab, int64_t nhub, const int32_t *hub_soff, int S, const int64_t *slice_base, hipStream_t s) {
  if (nhub > 0) hipLaunchKernelGGL(k_hub_rel, flat_grid(nhub), 256, 0, s, htab, nhub, hub_soff, S, slice_base);
}

__global__ void k_hub_expand(HubPlan p, int64_t nhub) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < nhub; h += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t q = p.hch[h]; q < p.hch[h + 1]; ++q) p.chub[q] = (int32_t)h;
    for (int64_t q = p.hsg[h]; q < p.hsg[h + 1]; ++q) p.shub[q] = (int32_t)h;
  }
}
void hub_expand(const HubPlan &h, int64_t nhub, hipStream_t s) {
  if (nhub > 0) hipLaunchKernelGGL(k_hub_expand, flat_grid(nhub), 256, 0, s, h, nhub);
}

__global__ void k_gather_bounds(const int64_t *arr, const int32_t *at, int count, int64_t *out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) out[k] = arr[at[k]];
}
void gather_bounds(const int64_t *arr, const int32_t *at, int count, int64_t *out, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_gather_bounds, flat_grid(count), 256, 0, s, arr, at, count, out);
}

// ---- apply: reverse-move resolution and move application ------------------
__device__ __forceinline__ bool reverse_wins(const MoveArgs &a, int j, int i, int fi, int p, double gi) {
  const int pj = a.prop[j];
  return pj >= 0 && pj == fi && a.from[j] == p && slice_of(j, a.nsl) == a.s && better(a.gp[j], j, gi, i);
}

__device__ __forceinline__ void flush_gain(const MoveArgs &a, double gsum, long long mv) {
  __shared__ double sd[16];
  __shared__ long long sl[16];
  const double g = block_sum(gsum, sd);
  const long long m = block_sum_ll(mv, sl);
  if (threadIdx.x == 0) {
    if (g != 0.0 && a.gain) unsafeAtomicAdd(a.gain, g);
    if (m) atomicAdd(a.moves, (unsigned long long)m);
  }
}

__device__ __forceinline__ void do_move(const MoveArgs &a, int i, int fi, int p, double g, double &gsum,
                                        long long &mv) {
  a.C[i] = p;
  const double k = a.K[i];
  unsafeAtomicAdd(&a.Sig[fi], -k);
  unsafeAtomicAdd(&a.Sig[p], k);
  if (a.track) { a.dC[fi] = 1; a.dC[p] = 1; }
  if (a.gi) a.gi[i] = g;
  else gsum += g;
  mv += 1;
}

template <int G>
__global__ __launch_bounds__(256) void k_apply_small(MoveArgs a, int b) {
  const int count = a.counts[a.s * kNB + b];
  const int32_t *list = a.lists + a.region[a.s * kNB + b];
  const int gl = threadIdx.x & (G - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwave = (int64_t)gridDim.x * blockDim.x / kWave;
  const int gin = lane() / G;
  double gsum = 0.0;
  long long mv = 0;
  const unsigned long long gm =
      (G == kWave) ? ~0ull : (((1ull << G) - 1ull) << (unsigned)(lane() & ~(G - 1)));
  for (int64_t v0 = wave * (kWave / G); v0 < count; v0 += nwave * (kWave / G)) {
    const int64_t v = v0 + gin;
    const int i = v < count ? list[v] : 0;
    const int p = v < count ? a.prop[i] : -1;
    bool blocked = false;
    int j = -1;
    int fi = 0;
    double g = 0.0;
    int deg = 0;
    if (p >= 0) {
      fi = a.from[i];
      g = a.gp[i];
      const int64_t e0 = a.off[i];
      deg = (int)(a.off[i + 1] - e0);
      if (gl < deg) {
        j = a.idx[e0 + gl];
        if (j != i) blocked = reverse_wins(a, j, i, fi, p, g);
      }
    }
    const bool any = (__ballot(blocked) & gm) != 0ull;
    if (p >= 0) {
      if (!any) {
        if (gl < deg && j != i) a.U[j] = 1;
        if (gl == 0) do_move(a, i, fi, p, g, gsum, mv);
      } else if (gl == 0) {
        a.U[i] = 1;
      }
    }
  }
  flush_gain(a, gsum, mv);
}

template <int TEAM, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_apply_team(MoveArgs a, int b) {
  constexpr int NT = BLOCK / TEAM;
  __shared__ int sany[NT];
  const int team = threadIdx.x / TEAM;
  const int t = threadIdx.x % TEAM;
  const int count = a.counts[a.s * kNB + b];
  const int32_t *list = a.lists + a.region[a.s * kNB + b];
  double gsum = 0.0;
  long long mv = 0;
  for (int64_t base = (int64_t)blockIdx.x * NT; base < count; base += (int64_t)gridDim.x * NT) {
    const int64_t v = base + team;
    const bool valid = v < count;
    const int i = valid ? list[v] : 0;
    const int p = valid ? a.prop[i] : -1;
    int fi = 0;
    double g = 0.0;
    int64_t e0 = 0, e1 = 0;
    bool blocked = false;
    if (p >= 0) {
      fi = a.from[i];
      g = a.gp[i];
      e0 = a.off[i];
      e1 = a.off[i + 1];
      for (int64_t e = e0 + t; e < e1 && !blocked; e += TEAM) {
        const int j = a.idx[e];
        if (j != i && reverse_wins(a, j, i, fi, p, g)) blocked = true;
      }
    }
    bool any;
    if (TEAM == kWave) {
      any = __ballot(blocked) != 0ull;
    } else {
      if (t == 0) sany[team] = 0;
      __syncthreads();
      if (blocked) sany[team] = 1;
      __syncthreads();
      any = sany[team] != 0;
    }
    if (p >= 0) {
      if (!any) {
        for (int64_t e = e0 + t; e < e1; e += TEAM) {
          const int j = a.idx[e];
          if (j != i) a.U[j] = 1;
        }
        if (t == 0) do_move(a, i, fi, p, g, gsum, mv);
      } else if (t == 0) {
        a.U[i] = 1;
      }
    }
    if (TEAM != kWave) __syncthreads();
  }
  flush_gain(a, gsum, mv);
}

// ---- launchers -----------------------------------------------------------------
static int grid_for(int64_t cap, int per_block, int maxb = 4096) {
  int64_t g = ceil_div(cap, per_block);
  if (g < 1) g = 1;
  return (int)(g < maxb ? g : maxb);
}

void move_frontier(const MoveArgs &a, hipStream_t s) {
  if (a.vend > a.vbeg)
    hipLaunchKernelGGL(k_frontier, flat_grid(ceil_div(a.vend - a.vbeg, kTile), 1, 2048), 256, 0, s, a);
}

void move_propose(const MoveArgs &a, const int64_t *region_h, hipStream_t s) {
  for (int b = 0; b < kNB; ++b) move_propose_bucket(a, region_h, b, s);
}

void move_propose_bucket(const MoveArgs &a, const int64_t *region_h, int b, hipStream_t s) {
  {
    const int64_t cap = region_h[a.s * kNB + b + 1] - region_h[a.s * kNB + b];
    if (cap <= 0) return;
    switch (b) {
      case 0: hipLaunchKernelGGL(k_propose_small<4>, grid_for(cap, 64), 256, 0, s, a, b); break;
      case 1: hipLaunchKernelGGL(k_propose_small<8>, grid_for(cap, 32), 256, 0, s, a, b); break;
      case 2: hipLaunchKernelGGL(k_propose_small<32>, grid_for(cap, 8), 256, 0, s, a, b); break;
      case 3: hipLaunchKernelGGL((k_propose_team<64, 512, 256>), grid_for(cap, 4), 256, 0, s, a, b); break;
      case 4: hipLaunchKernelGGL((k_propose_team<256, 4096, 256>), grid_for(cap, 1, 2048), 256, 0, s, a, b); break;
      case 5:
        move_hub_gather(a, s);
        move_hub_score(a, s);
        break;
    }
  }
}

void move_hub_gather(const MoveArgs &a, hipStream_t s) {
  if (a.qend > a.qbeg) hipLaunchKernelGGL(k_hub_gather, (int)(a.qend - a.qbeg), 256, 0, s, a);
}

void move_hub_score(const MoveArgs &a, hipStream_t s) {
  if (a.qend > a.qbeg) {
    hipLaunchKernelGGL(k_hub_score, (int)(a.gend - a.gbeg), 256, 0, s, a);
    hipLaunchKernelGGL(k_hub_final, (int)ceil_div(a.hend - a.hbeg, (int64_t)4), 256, 0, s, a);
  }
}

void move_apply(const MoveArgs &a, const int64_t *region_h, hipStream_t s) {
  for (int b = 0; b < kNB; ++b) move_apply_bucket(a, region_h, b, s);
}

void move_hub_apply(const MoveArgs &a, hipStream_t s);

void move_apply_bucket(const MoveArgs &a, const int64_t *region_h, int b, hipStream_t s) {
  const int64_t cap = region_h[a.s * kNB + b + 1] - region_h[a.s * kNB + b];
  if (cap <= 0) return;
  switch (b) {
    case 0: hipLaunchKernelGGL(k_apply_small<4>, grid_for(cap, 64), 256, 0, s, a, b); break;
    case 1: hipLaunchKernelGGL(k_apply_small<8>, grid_for(cap, 32), 256, 0, s, a, b); break;
    case 2: hipLaunchKernelGGL(k_apply_small<32>, grid_for(cap, 8), 256, 0, s, a, b); break;
    case 3: hipLaunchKernelGGL((k_apply_team<64, 256>), grid_for(cap, 4), 256, 0, s, a, b); break;
    case 4: hipLaunchKernelGGL((k_apply_team<256, 256>), grid_for(cap, 1, 2048), 256, 0, s, a, b); break;
    case 5: move_hub_apply(a, s); break;
  }
}

// ---- apply for hubs, chunk-parallel --------------------------------------------
// The same rule as the other buckets, with the hub's edge chunks spread over
// workgroups: (1) a chunk that finds a same-slice neighbour proposing the
// exact reverse move with priority flags the hub blocked; (2) every chunk of
// an unblocked hub marks its neighbours unprocessed and the first one moves
// the hub, while the first chunk of a blocked hub leaves it unprocessed.
__global__ __launch_bounds__(256) void k_hub_rev(MoveArgs a) {
  const int64_t q = a.qbeg + blockIdx.x;
  const int h = a.hp.chub[q];
  const int i = a.hp.hubv[h];
  // the frontier read in the gather is complete: clear the processed flag
  if (a.hub_front && q == a.hp.hch[h] && threadIdx.x == 0) a.U[i] = 0;
  if (!a.act[i]) return;
  const int p = a.prop[i];
  if (p < 0) return;
  const int fi = a.from[i];
  const double g = a.gp[i];
  const int64_t e0 = a.off[i] + (q - a.hp.hch[h]) * kHubEC;
  const int64_t e1 = min(e0 + (int64_t)kHubEC, a.off[i + 1]);
  bool blocked = false;
  for (int64_t e = e0 + threadIdx.x; e < e1 && !blocked; e += blockDim.x) {
    const int j = a.idx[e];
    if (j != i && reverse_wins(a, j, i, fi, p, g)) blocked = true;
  }
  if (blocked) a.hp.flag[h] = 1;
}

__global__ __launch_bounds__(256) void k_hub_mark(MoveArgs a) {
  const int64_t q = a.qbeg + blockIdx.x;
  const int h = a.hp.chub[q];
  const int i = a.hp.hubv[h];
  if (!a.act[i]) return;
  const int p = a.prop[i];
  if (p < 0) return;
  const bool lead = q == a.hp.hch[h] && threadIdx.x == 0;
  if (a.hp.flag[h] == 1) {
    if (lead) a.U[i] = 1;
    return;
  }
  if (lead) {
    double gsum = 0.0;
    long long mv = 0;
    do_move(a, i, a.from[i], p, a.gp[i], gsum, mv);
    if (gsum != 0.0 && a.gain) unsafeAtomicAdd(a.gain, gsum);
    atomicAdd(a.moves, 1ull);
  }
  const int64_t e0 = a.off[i] + (q - a.hp.hch[h]) * kHubEC;
  const int64_t e1 = min(e0 + (int64_t)kHubEC, a.off[i + 1]);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int j = a.idx[e];
    if (j != i) a.U[j] = 1;
  }
}

void move_hub_apply(const MoveArgs &a, hipStream_t s) {
  if (a.qend <= a.qbeg) return;
  hipLaunchKernelGGL(k_hub_rev, (int)(a.qend - a.qbeg), 256, 0, s, a);
  hipLaunchKernelGGL(k_hub_mark, (int)(a.qend - a.qbeg), 256, 0, s, a);
}

// ---- fixed-order gain total (synchronous mode) ------------------------------------
__global__ void k_tile_sums(const double *x, int64_t n, double *tiles) {
  const int64_t ntiles = ceil_div(n, 256);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = t * 256;
    const int64_t b = min(n, a + 256);
    double s = 0.0;
    for (int64_t k = a; k < b; ++k) s += x[k];
    tiles[t] = s;
  }
}

__global__ __launch_bounds__(64) void k_tiles_total(const double *tiles, int64_t ntiles, double *out) {
  __shared__ double buf[64];
  double total = 0.0;
  for (int64_t base = 0; base < ntiles; base += 64) {
    const int64_t k = base + threadIdx.x;
    buf[threadIdx.x] = k < ntiles ? tiles[k] : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int64_t m = min((int64_t)64, ntiles - base);
      for (int64_t q = 0; q < m; ++q) total += buf[q];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = total;
}

void tiled_sum(const double *gi, int64_t n, double *tiles, double *out, hipStream_t s) {
  const int64_t ntiles = ceil_div(n, 256);
  if (ntiles > 0) hipLaunchKernelGGL(k_tile_sums, flat_grid(ntiles), 256, 0, s, gi, n, tiles);
  hipLaunchKernelGGL(k_tiles_total, 1, 64, 0, s, tiles, ntiles, out);
}

}  // namespace lk
