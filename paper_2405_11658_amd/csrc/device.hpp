// Device-side building blocks shared by the HIP kernels of the library:
// wave64 primitives, wave-aggregated atomics, an open-addressing
// community -> weight table (LDS or global memory), and the move score.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <limits.h>

namespace lk {

constexpr int kWave = 64;
constexpr int kNoComm = INT_MAX;  // "no candidate" in argmax reductions
constexpr int kEmpty = -1;        // empty table slot

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Eq. 2 scaled by 2m^2 (so Delta-Q = g / (M2^2 / 2)):
//   g = M2*(K_{i->c} - K_{i->d}) - K_i*(K_i + Sigma_c - Sigma_d),
// Sigma_d including K_i.  Exact parenthesisation, no contraction, so the
// value is bit-identical to any other IEEE evaluation of the same expression.
__device__ __forceinline__ double move_score(double M2, double a, double b, double Ki, double Sc,
                                             double Sd) {
#pragma clang fp contract(off)
  double t1 = M2 * (a - b);
  double t2 = Ki * ((Ki + Sc) - Sd);
  return t1 - t2;
}

// Total order used by every argmax: larger gain first, then smaller id.
__device__ __forceinline__ bool better(double g1, int c1, double g2, int c2) {
  return g1 > g2 || (g1 == g2 && c1 < c2);
}

template <int W>
__device__ __forceinline__ void group_argmax(double &g, int &c) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) {
    double og = __shfl_xor(g, off, W);
    int oc = __shfl_xor(c, off, W);
    if (better(og, oc, g, c)) { g = og; c = oc; }
  }
}

template <int W>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

template <int W>
__device__ __forceinline__ long long group_sum_ll(long long v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// 32-bit integer finaliser "lowbias32" (xorshift-multiply; constants from
// C. Wellons' published hash-prospector search).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ uint32_t mix64(uint64_t x) {
  return mix32((uint32_t)x ^ mix32((uint32_t)(x >> 32)));
}

// Argmax over a team of TEAM threads (TEAM a multiple of the wavefront or
// smaller); the result is valid in the team's first thread.  With TEAM >
// kWave every thread of the workgroup must call it.
template <int TEAM, int BLOCK>
__device__ __forceinline__ void team_argmax(double &g, int &c, double *rg, int *rc) {
  group_argmax<kWave>(g, c);
  if (TEAM > kWave) {
    const int w = threadIdx.x / kWave;
    if (lane() == 0) { rg[w] = g; rc[w] = c; }
    __syncthreads();
    if ((threadIdx.x % TEAM) == 0) {
      for (int k = 1; k < TEAM / kWave; ++k)
        if (better(rg[w + k], rc[w + k], g, c)) { g = rg[w + k]; c = rc[w + k]; }
    }
    __syncthreads();
  }
}

// Open addressing with linear probing.  keys[] holds kEmpty for free slots,
// vals[] starts at 0.  Capacity (mask+1) must exceed the number of distinct
// keys inserted; the probe loop is bounded by the capacity in any case.
__device__ __forceinline__ void table_add(int *keys, double *vals, uint32_t mask, int key,
                                          double w) {
  uint32_t h = mix32((uint32_t)key) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    int k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
    if (k == key) { atomicAdd(&vals[h], w); return; }
    if (k == kEmpty) {
      int old = atomicCAS(&keys[h], kEmpty, key);
      if (old == kEmpty || old == key) { atomicAdd(&vals[h], w); return; }
    }
    h = (h + 1) & mask;
  }
}

// Workgroup-level merge of (key, value) additions before they reach global
// memory: the block inserts into an LDS table (capacity above the number of
// distinct keys it inserts) and then issues one atomic per distinct key, so a
// key shared by many items (a giant community) costs one global atomic per
// workgroup instead of one per item.  Called by the whole block.
template <int SLOTS>
__device__ __forceinline__ void block_merge_clear(int *tk, double *tv) {
  for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) { tk[s] = kEmpty; tv[s] = 0.0; }
  __syncthreads();
}
template <int SLOTS>
__device__ __forceinline__ void block_merge_flush(int *tk, double *tv, double *out) {
  __syncthreads();
  for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
    if (tk[s] != kEmpty) {
      unsafeAtomicAdd(&out[tk[s]], tv[s]);
      tk[s] = kEmpty;
      tv[s] = 0.0;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double table_get(const int *keys, const double *vals, uint32_t mask,
                                            int key) {
  uint32_t h = mix32((uint32_t)key) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    int k = keys[h];
    if (k == key) return vals[h];
    if (k == kEmpty) return 0.0;
    h = (h + 1) & mask;
  }
  return 0.0;
}

// Wave-aggregated counter increment: lanes with equal keys share one atomic.
// Returns, for each active lane, old counter value + rank among equal keys.
// Must be called by the whole wave (inactive lanes pass active = false).
__device__ __forceinline__ int wave_peel_inc(int *ctr, int key, bool active) {
  unsigned long long pending = __ballot(active);
  int result = 0;
  const int ln = lane();
  while (pending) {
    int leader = __ffsll((unsigned long long)pending) - 1;
    int k = __shfl(key, leader);
    unsigned long long grp = __ballot(active && key == k) & pending;
    int base = 0;
    if (ln == leader) base = atomicAdd(&ctr[k], (int)__popcll(grp));
    base = __shfl(base, leader);
    if ((grp >> ln) & 1ull) result = base + (int)__popcll(grp & ((1ull << ln) - 1ull));
    pending &= ~grp;
  }
  return result;
}

// Wave-aggregated append to one of `nb` lists: lanes with equal bucket share
// one atomic on counts[bucket].  Returns the slot index inside the bucket.
__device__ __forceinline__ int wave_append(int *counts, int bucket, bool active) {
  return wave_peel_inc(counts, bucket, active);
}

// Wave-aggregated FP64 scatter-add arr[key] += v.  The most frequent keys of
// the wave are combined first (up to 4 rounds), the rest use direct atomics.
__device__ __forceinline__ void wave_peel_add_f64(double *arr, int key, double v, bool active) {
  unsigned long long pending = __ballot(active);
  const int ln = lane();
  for (int round = 0; round < 4 && pending; ++round) {
    int leader = __ffsll((unsigned long long)pending) - 1;
    int k = __shfl(key, leader);
    bool mine = ((pending >> ln) & 1ull) && key == k;
    unsigned long long grp = __ballot(mine);
    double s = group_sum<kWave>(mine ? v : 0.0);
    if (ln == leader) atomicAdd(&arr[k], s);
    pending &= ~grp;
  }
  if ((pending >> ln) & 1ull) atomicAdd(&arr[key], v);
}

// Block-wide sum (blockDim.x <= 1024, multiple of 64); result valid in all threads.
__device__ __forceinline__ double block_sum(double v, double *scratch /* >= 16 */) {
  v = group_sum<kWave>(v);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if (lane() == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += scratch[k];
  __syncthreads();
  return t;
}

__device__ __forceinline__ long long block_sum_ll(long long v, long long *scratch /* >= 16 */) {
  v = group_sum_ll<kWave>(v);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if (lane() == 0) scratch[w] = v;
  __syncthreads();
  long long t = 0;
  for (int k = 0; k < nw; ++k) t += scratch[k];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int64_t lower_bound_i32(const int32_t *a, int64_t lo, int64_t hi, int32_t x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Exclusive max-scan across the block (blockDim.x multiple of 64, <= 1024).
__device__ __forceinline__ int block_excl_max_scan(int v, int *sh /* >= 16 ints */) {
  int x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int y = __shfl_up(x, off);
    if (lane() >= off) x = max(x, y);
  }
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane() == kWave - 1) sh[w] = x;
  __syncthreads();
  int pre = -1;
  for (int k = 0; k < w; ++k) pre = max(pre, sh[k]);
  int incl = max(x, pre);
  int ex = __shfl_up(incl, 1);
  if (lane() == 0) ex = pre;
  __syncthreads();
  return ex;
}

// Row mapping for a chunk of CSR positions [q0, q0 + len), len <= CH:
// rowof[t] receives the row owning position q0 + t.  lo is the row owning q0
// and hi an upper bound on the row owning q0 + len - 1 (both precomputed by
// chunk_start_rows).  Empty rows are handled.  Called by the whole block.
template <int CH>
__device__ __forceinline__ void chunk_rows(const int64_t *off, int64_t q0, int len, int lo, int hi,
                                           int *rowof, int *sh) {
  for (int t = threadIdx.x; t < CH; t += blockDim.x) rowof[t] = -1;
  __syncthreads();
  // the start of every non-empty row (an empty row starts where the next
  // non-empty one does, and that one owns the slot): one plain store per
  // slot, no atomics
  for (int r = lo + (int)threadIdx.x; r <= hi; r += blockDim.x) {
    int64_t s = off[r] - q0;
    if (s < 0) s = 0;
    if (s < len && (r == hi || off[r + 1] > off[r])) rowof[s] = r;
  }
  __syncthreads();
  const int per = CH / (int)blockDim.x;
  const int t0 = threadIdx.x * per;
  int m = -1;
  for (int t = t0; t < t0 + per; ++t) m = max(m, rowof[t]);
  int acc = block_excl_max_scan(m, sh);
  for (int t = t0; t < t0 + per; ++t) {
    acc = max(acc, rowof[t]);
    rowof[t] = acc;
  }
  __syncthreads();
}

}  // namespace lk
