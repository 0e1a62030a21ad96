// Refinement side of a pass:
//   subset renumber (Alg. "leidenSubsetRenumber"): every community is
//     relabelled by its smallest member id, Sigma' and deltaC' re-keyed;
//   break (function "breakChangedCommunities" of Alg. "leiden"): vertices of
//     changed communities become singletons; the community bounds C'_B are
//     kept;
//   refine (Alg. "leidenRefine" with "scanBounded"): constrained merges of
//     isolated vertices inside their bound, one sweep over the vertex slices
//     in order - in a slice every isolated vertex of a changed bound proposes
//     its best target inside the bound from the current state; a proposal is
//     accepted when the target's representative is not proposing in the
//     slice, or when the two propose to each other and the proposer has
//     priority (larger gain, then smaller id).
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

__device__ __forceinline__ int bucket_of_r(int64_t deg, int64_t hubdeg) {
  return deg > hubdeg ? 5 : deg <= 4 ? 0 : deg <= 8 ? 1 : deg <= 32 ? 2 : deg <= 256 ? 3 : 4;
}

__global__ void k_rep_min(int64_t n, const int32_t *C, int32_t *rep) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = C[i];
    // a (possibly stale) value <= i means a smaller member already won
    if (rep[c] > (int32_t)i) atomicMin(&rep[c], (int32_t)i);
  }
}

__global__ void k_subset_remap(int64_t n, int32_t *C, const int32_t *rep, const double *Sig, double *Sig2,
                               const uint8_t *dC, uint8_t *dC2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = C[i];
    const int r = rep[c];
    if (r == (int32_t)i) { Sig2[i] = Sig[c]; dC2[i] = dC[c]; }
    else { Sig2[i] = 0.0; dC2[i] = 0; }
    C[i] = r;
  }
}

void subset_renumber(int64_t n, int32_t *C, int32_t *rep, const double *Sig, double *Sig2,
                     const uint8_t *dC, uint8_t *dC2, hipStream_t s) {
  if (n <= 0) return;
  fill_i32(rep, INT_MAX, n, s);
  hipLaunchKernelGGL(k_rep_min, flat_grid(n), 256, 0, s, n, C, rep);
  hipLaunchKernelGGL(k_subset_remap, flat_grid(n), 256, 0, s, n, C, rep, Sig, Sig2, dC, dC2);
}

// Break changed communities; keep the bounds; bucket the refine candidates
// by (slice, degree bucket), with per-workgroup reservation of list ranges.
constexpr int kRTile = 4096;
constexpr int kRMaxKeys = 2048;  // >= 256 slices * kNB

__device__ __forceinline__ int break_key(const RefineArgs &a, int64_t i, int cb) {
  if (!a.dC[cb]) return -2;  // not in a changed bound
  const int64_t deg = a.off[i + 1] - a.off[i];
  return deg > 0 ? slice_of(i, a.nsl) * kNB + bucket_of_r(deg, a.hubdeg) : -1;
}

__global__ __launch_bounds__(256) void k_break(RefineArgs a) {
  __shared__ int cnt[kRMaxKeys];
  __shared__ int base[kRMaxKeys];
  __shared__ long long sl_ref[16];
  const int K = a.nsl * kNB;
  long long nref = 0;
  for (int64_t t0 = (int64_t)blockIdx.x * kRTile; t0 < a.n; t0 += (int64_t)gridDim.x * kRTile) {
    const int64_t t1 = min(t0 + (int64_t)kRTile, a.n);
    for (int k = threadIdx.x; k < K; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
      const int key = break_key(a, i, a.C[i]);
      if (key >= 0) atomicAdd(&cnt[key], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const int c = cnt[k];
      base[k] = c ? atomicAdd(&a.counts[k], c) : 0;
      cnt[k] = 0;
    }
    __syncthreads();
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
      const int cb = a.C[i];
      const int key = break_key(a, i, cb);
      a.CB[i] = cb;
      if (key == -2) continue;
      a.C[i] = (int32_t)i;
      a.Sig[i] = a.K[i];
      a.S[i] = 1;
      a.prop[i] = -1;
      nref++;
      if (key >= 0) a.lists[a.region[key] + base[key] + atomicAdd(&cnt[key], 1)] = (int32_t)i;
    }
    __syncthreads();
  }
  const long long tot = block_sum_ll(nref, sl_ref);
  if (threadIdx.x == 0 && tot) atomicAdd(a.refined, (unsigned long long)tot);
}

void refine_break(const RefineArgs &a, hipStream_t s) {
  if (a.n > 0) hipLaunchKernelGGL(k_break, flat_grid(ceil_div(a.n, kRTile), 1, 2048), 256, 0, s, a);
}

// ---- refine propose ------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(256) void k_rprop_small(RefineArgs a, int b) {
  const int count = a.counts[a.s * kNB + b];
  const int32_t *list = a.lists + a.region[a.s * kNB + b];
  const int gl = threadIdx.x & (G - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwave = (int64_t)gridDim.x * blockDim.x / kWave;
  const int gin = lane() / G;
  for (int64_t v0 = wave * (kWave / G); v0 < count; v0 += nwave * (kWave / G)) {
    const int64_t v = v0 + gin;
    const bool valid = v < count;
    const int i = valid ? list[v] : 0;
    const bool active = valid && a.C[i] == i && a.S[i] == 1;
    int64_t e0 = 0;
    int deg = 0, cbi = 0;
    if (active) {
      e0 = a.off[i];
      deg = (int)(a.off[i + 1] - e0);
      cbi = a.CB[i];
    }
    int key = -1;
    float wt = 0.0f;
    if (gl < deg) {
      const int j = a.idx[e0 + gl];
      if (j != i && a.CB[j] == cbi) { key = a.C[j]; wt = a.w[e0 + gl]; }
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
    const double bown = group_sum<G>((key == i && first) ? sum : 0.0);
    double g = 0.0;
    int c = kNoComm;
    if (key >= 0 && key != i && first) {
      const double x = move_score(a.M2, sum, bown, a.K[i], a.Sig[key], a.Sig[i]);
      if (x > 0.0) { g = x; c = key; }
    }
    group_argmax<G>(g, c);
    if (valid && gl == 0) {
      a.prop[i] = (c == kNoComm) ? -1 : c;
      a.gp[i] = g;
    }
  }
}


template <int TEAM, int T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_rprop_team(RefineArgs a, int b) {
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
    const bool active = valid && a.C[i] == i && a.S[i] == 1;
    int64_t e0 = 0, e1 = 0;
    int cbi = 0;
    if (active) { e0 = a.off[i]; e1 = a.off[i + 1]; cbi = a.CB[i]; }
    int *keys = skeys + team * T;
    double *vals = svals + team * T;
    const uint32_t mask = T - 1;
    for (uint32_t s = t; s <= mask; s += TEAM) { keys[s] = kEmpty; vals[s] = 0.0; }
    if (t == 0) sb[team] = 0.0;
    __syncthreads();
    if (active) {
      for (int64_t e = e0 + t; e < e1; e += TEAM) {
        const int j = a.idx[e];
        if (j != i && a.CB[j] == cbi) table_add(keys, vals, mask, a.C[j], (double)a.w[e]);
      }
    }
    __syncthreads();
    if (active)
      for (uint32_t s = t; s <= mask; s += TEAM)
        if (keys[s] == i) sb[team] = vals[s];
    __syncthreads();
    double bg = 0.0;
    int bc = kNoComm;
    if (active) {
      const double bown = sb[team];
      const double Ki = a.K[i];
      const double Sd = a.Sig[i];
      for (uint32_t s = t; s <= mask; s += TEAM) {
        const int c = keys[s];
        if (c == kEmpty || c == i) continue;
        const double x = move_score(a.M2, vals[s], bown, Ki, a.Sig[c], Sd);
        if (x > 0.0 && better(x, c, bg, bc)) { bg = x; bc = c; }
      }
    }
    group_argmax<kWave>(bg, bc);
    if (TEAM > kWave) {
      const int w = threadIdx.x / kWave;
      if (lane() == 0) { rg[w] = bg; rc[w] = bc; }
      __syncthreads();
      if (t == 0)
        for (int k = 1; k < TEAM / kWave; ++k)
          if (better(rg[w + k], rc[w + k], bg, bc)) { bg = rg[w + k]; bc = rc[w + k]; }
      __syncthreads();
    }
    if (valid && t == 0) {
      a.prop[i] = (bc == kNoComm) ? -1 : bc;
      a.gp[i] = bg;
    }
    __syncthreads();
  }
}

static int rgrid(int64_t cap, int per_block, int maxb = 4096) {
  int64_t g = ceil_div(cap, per_block);
  if (g < 1) g = 1;
  return (int)(g < maxb ? g : maxb);
}

// ---- refine propose for hubs: several workgroups per candidate -------------------
// Same decomposition as the local-moving hub path (edge chunks merged in LDS,
// then a global table per hub; segments scored and cleared; a final
// wavefront reduces).  Candidates: hubs of the slice in a changed bound that
// are isolated at the start of the slice; only neighbours in the same bound
// count; the own community is the vertex itself.  Each gather chunk tests
// candidacy itself (nothing it reads changes during the launch) and the
// hub's first chunk records it for the later launches.
__global__ __launch_bounds__(256) void k_rhub_gather(RefineArgs a) {
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
  const bool go = a.dC[a.CB[i]] && a.C[i] == i && a.S[i] == 1;
  if (q == a.hp.hch[h] && threadIdx.x == 0) a.act[i] = go;
  if (!go) return;
  const int64_t e0 = a.off[i] + (q - a.hp.hch[h]) * kHubEC;
  const int64_t e1 = min(e0 + (int64_t)kHubEC, a.off[i + 1]);
  const int cbi = a.CB[i];
  for (int s = threadIdx.x; s < T; s += blockDim.x) { keys[s] = kEmpty; vals[s] = 0.0; }
  if (threadIdx.x == 0) nused = 0;
  // this thread's edges: all ids first, then communities and bounds together
  int j[PER], c[PER];
  float x[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t e = e0 + threadIdx.x + u * 256;
    j[u] = i;
    x[u] = 0.0f;
    if (e < e1) { j[u] = a.idx[e]; x[u] = a.w[e]; }
  }
  if (a.CP) {
    // packed (bound << 32 | community): one load per neighbour
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      c[u] = kEmpty;
      if (j[u] != i) {
        const unsigned long long pk = a.CP[j[u]];
        if ((int)(pk >> 32) == cbi) c[u] = (int)(uint32_t)pk;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      c[u] = kEmpty;
      if (j[u] != i) {
        const int cj = a.C[j[u]];
        if (a.CB[j[u]] == cbi) c[u] = cj;
      }
    }
  }
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
  const int64_t t0 = a.hp.htab[h];
  const uint32_t mask = (uint32_t)(a.hp.hcap[h] - 1);
  for (int k = threadIdx.x; k < nu; k += blockDim.x) {
    const int s = used[k];
    const int cs = keys[s];
    if (cs == i) unsafeAtomicAdd(&a.hp.own[h], vals[s]);
    else table_add(a.hp.keys + t0, a.hp.vals + t0, mask, cs, vals[s]);
  }
}

__global__ __launch_bounds__(256) void k_rhub_score(RefineArgs a) {
  __shared__ double rg[256 / kWave];
  __shared__ int rc[256 / kWave];
  const int64_t q = a.gbeg + blockIdx.x;
  const int h = a.hp.shub[q];
  const int i = a.hp.hubv[h];
  if (!a.act[i]) return;
  const int64_t s0 = a.hp.htab[h] + (q - a.hp.hsg[h]) * kHubSeg;
  const int64_t s1 = s0 + min((int64_t)kHubSeg, a.hp.hcap[h]);
  const double Ki = a.K[i], Sd = a.Sig[i], bown = a.hp.own[h];
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

__global__ __launch_bounds__(256) void k_rhub_final(RefineArgs a) {
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
    a.prop[i] = (bc == kNoComm) ? -1 : bc;
    a.gp[i] = bg;
    a.hp.own[h] = 0.0;
  }
}

static void refine_hubs(const RefineArgs &a, hipStream_t s) {
  if (a.hend <= a.hbeg || a.qend <= a.qbeg) return;  // every hub has edge chunks
  hipLaunchKernelGGL(k_rhub_gather, (int)(a.qend - a.qbeg), 256, 0, s, a);
  hipLaunchKernelGGL(k_rhub_score, (int)(a.gend - a.gbeg), 256, 0, s, a);
  hipLaunchKernelGGL(k_rhub_final, (int)ceil_div(a.hend - a.hbeg, (int64_t)4), 256, 0, s, a);
}

void refine_propose(const RefineArgs &a, const int64_t *region_h, hipStream_t s) {
  for (int b = 0; b < kNB; ++b) refine_propose_bucket(a, region_h, b, s);
}

void refine_propose_bucket(const RefineArgs &a, const int64_t *region_h, int b, hipStream_t s) {
  const int64_t cap = region_h[a.s * kNB + b + 1] - region_h[a.s * kNB + b];
  if (cap <= 0) return;
  switch (b) {
    case 0: hipLaunchKernelGGL(k_rprop_small<4>, rgrid(cap, 64), 256, 0, s, a, b); break;
    case 1: hipLaunchKernelGGL(k_rprop_small<8>, rgrid(cap, 32), 256, 0, s, a, b); break;
    case 2: hipLaunchKernelGGL(k_rprop_small<32>, rgrid(cap, 8), 256, 0, s, a, b); break;
    case 3: hipLaunchKernelGGL((k_rprop_team<64, 512, 256>), rgrid(cap, 4), 256, 0, s, a, b); break;
    case 4: hipLaunchKernelGGL((k_rprop_team<256, 4096, 256>), rgrid(cap, 1, 2048), 256, 0, s, a, b); break;
    case 5: refine_hubs(a, s); break;
  }
}

// Accept the proposals of slice s.  p "is proposing" only if p belongs to
// slice s and proposed in it.  One thread per list slot of the slice.
__global__ void k_raccept(RefineArgs a, int64_t beg, int64_t end) {
  for (int64_t t = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < end; t += (int64_t)gridDim.x * blockDim.x) {
    int b = 0;
    while (b + 1 < kNB && t >= a.region[a.s * kNB + b + 1]) ++b;
    if (t - a.region[a.s * kNB + b] >= a.counts[a.s * kNB + b]) continue;
    const int i = a.lists[t];
    const int p = a.prop[i];
    if (p < 0) continue;
    const int pp = (slice_of(p, a.nsl) == a.s) ? a.prop[p] : -1;
    const bool ok = pp < 0 || (pp == i && better(a.gp[i], i, a.gp[p], p));
    if (!ok) continue;
    a.C[i] = p;
    if (a.CP) a.CP[i] = ((unsigned long long)(uint32_t)a.CB[i] << 32) | (uint32_t)p;
    const double k = a.K[i];
    unsafeAtomicAdd(&a.Sig[i], -k);
    unsafeAtomicAdd(&a.Sig[p], k);
    a.S[i] = 0;
    atomicAdd(&a.S[p], 1);
  }
}

void refine_accept(const RefineArgs &a, const int64_t *region_h, hipStream_t s) {
  const int64_t beg = region_h[a.s * kNB], end = region_h[(a.s + 1) * kNB];
  if (end > beg) hipLaunchKernelGGL(k_raccept, flat_grid(end - beg), 256, 0, s, a, beg, end);
}

}  // namespace lk
