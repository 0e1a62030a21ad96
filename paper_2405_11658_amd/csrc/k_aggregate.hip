// Aggregation (Alg. "leidenAggregate"): the super-vertex graph of a level.
//
// GPU design.  Vertices with edges are counting-sorted by community (the
// community-vertex CSR of the algorithm); concatenating their rows in that
// order gives an "entry space" in which every community owns one contiguous
// range [toff[c], toff[c+1]).  The entry space is cut into fixed chunks of
// kChunk positions; each workgroup maps its positions to (member, entry) with
// an LDS max-scan, and merges (C[u], C[v]) pairs in an LDS hash table.  A
// community lying inside one chunk is emitted directly into its holey output
// row (capacity = its total degree).  Communities spanning several chunks
// leave per-chunk partial sums, which a second step merges in a global table
// per community sized from the known partial count.  Rows are then compacted
// and their weight sums (the next level's K' = Sigma') computed.
// Weights are summed in FP64 and stored rounded to float32.
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

__global__ void k_agg_count(int64_t n, const int64_t *off, const int32_t *C, int32_t *cnt) {
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    bool act = false;
    int c = 0;
    if (i < n) {
      act = off[i + 1] > off[i];
      c = C[i];
    }
    wave_peel_inc(cnt, c, act);
  }
}
void agg_count(const AggArgs &a, hipStream_t s) {
  if (a.n > 0) hipLaunchKernelGGL(k_agg_count, flat_grid(a.n), 256, 0, s, a.n, a.off, a.C, a.cnt);
}

__global__ void k_agg_scatter(int64_t n, const int64_t *off, const int32_t *C, const int32_t *coff,
                              int32_t *fill, int32_t *mem) {
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    bool act = false;
    int c = 0;
    if (i < n) {
      act = off[i + 1] > off[i];
      c = C[i];
    }
    const int pos = wave_peel_inc(fill, c, act);
    if (act) mem[coff[c] + pos] = (int32_t)i;
  }
}
void agg_scatter(const AggArgs &a, hipStream_t s) {
  if (a.n > 0) hipLaunchKernelGGL(k_agg_scatter, flat_grid(a.n), 256, 0, s, a.n, a.off, a.C, a.coff, a.cnt, a.mem);
}

__global__ void k_agg_mdeg(int64_t M, const int32_t *mem, const int64_t *off, int64_t *mdeg) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= M; k += (int64_t)gridDim.x * blockDim.x) {
    if (k == M) { mdeg[k] = 0; continue; }
    const int u = mem[k];
    mdeg[k] = off[u + 1] - off[u];
  }
}
void agg_mdeg(const AggArgs &a, int64_t M, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_mdeg, flat_grid(M + 1), 256, 0, s, M, a.mem, a.off, a.mdeg);
}

__global__ void k_agg_toff(int64_t ncomm, const int32_t *coff, const int64_t *mpos, int64_t *toff) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= ncomm; c += (int64_t)gridDim.x * blockDim.x)
    toff[c] = mpos[coff[c]];
}
void agg_toff(const AggArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_toff, flat_grid(a.ncomm + 1), 256, 0, s, a.ncomm, a.coff, a.mpos, a.toff);
}

// One workgroup per chunk of the entry space.
constexpr int kAggT = 2 * kChunk;  // LDS table slots (load factor <= 1/2)

__global__ __launch_bounds__(256) void k_agg_items(AggArgs a, int64_t M) {
  __shared__ unsigned long long tkeys[kAggT];
  __shared__ double tvals[kAggT];
  __shared__ int slotof[kChunk];
  __shared__ int sh[16];
  __shared__ int np;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, a.nnz - base);
  chunk_rows<kChunk>(a.mpos, base, len, a.mcrow[blockIdx.x], a.mcrow[blockIdx.x + 1], slotof, sh);
  for (int s = threadIdx.x; s < kAggT; s += blockDim.x) { tkeys[s] = ~0ull; tvals[s] = 0.0; }
  if (threadIdx.x == 0) np = 0;
  __syncthreads();
  for (int t0 = 0; t0 < len; t0 += blockDim.x) {
    const int t = t0 + threadIdx.x;
    const bool on = t < len;
    unsigned long long key = 0;
    double x = 0.0;
    if (on) {
      const int k = slotof[t];
      const int u = a.mem[k];
      const int64_t e = a.off[u] + (base + t - a.mpos[k]);
      const int v = a.idx[e];
      x = (double)a.w[e];
      key = ((unsigned long long)(uint32_t)a.C[u] << 32) | (uint32_t)a.C[v];
    }
    table_add64_wave(tkeys, tvals, kAggT - 1, key, x, on);
  }
  __syncthreads();
  for (int s0 = 0; s0 < kAggT; s0 += blockDim.x) {
    const int s = s0 + threadIdx.x;
    const unsigned long long key = tkeys[s];
    const bool used = key != ~0ull;
    const int c = used ? (int)(key >> 32) : 0;
    const int d = (int)(key & 0xffffffffull);
    bool inside = false;
    if (used) inside = a.toff[c] >= base && a.toff[c + 1] <= base + len;
    const int pos = wave_peel_inc(a.rowlen, c, used && inside);
    if (used && inside) {
      a.hidx[a.toff[c] + pos] = d;
      a.hw[a.toff[c] + pos] = (float)tvals[s];
    }
    const bool part = used && !inside;
    const unsigned long long pm = __ballot(part);
    int pbase = 0;
    if (lane() == 0 && pm) pbase = atomicAdd(&np, (int)__popcll(pm));
    pbase = __shfl(pbase, 0);
    if (part) {
      const int r = pbase + (int)__popcll(pm & ((1ull << lane()) - 1ull));
      a.pkey[base + r] = key;
      a.pval[base + r] = tvals[s];
    }
    wave_peel_inc(a.pcnt, c, part);
  }
  __syncthreads();
  if (threadIdx.x == 0) a.pcnt_item[blockIdx.x] = np;
}
void agg_items(const AggArgs &a, int64_t M, hipStream_t s) {
  if (a.nnz > 0) hipLaunchKernelGGL(k_agg_items, (int)ceil_div(a.nnz, kChunk), 256, 0, s, a, M);
}

__global__ void k_agg_caps(int64_t ncomm, const int32_t *pcnt, int64_t *tcap) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= ncomm; c += (int64_t)gridDim.x * blockDim.x) {
    int64_t cap = 0;
    if (c < ncomm && pcnt[c] > 0) {
      cap = 16;
      while (cap < 2 * (int64_t)pcnt[c]) cap <<= 1;
    }
    tcap[c] = cap;
  }
}
void agg_caps(const AggArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_caps, flat_grid(a.ncomm + 1), 256, 0, s, a.ncomm, a.pcnt, a.tcap);
}

__global__ __launch_bounds__(256) void k_agg_part_insert(AggArgs a, int *tkeys, double *tvals) {
  const int np = a.pcnt_item[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  for (int t = threadIdx.x; t < np; t += blockDim.x) {
    const unsigned long long key = a.pkey[base + t];
    const int c = (int)(key >> 32);
    const int d = (int)(key & 0xffffffffull);
    const int64_t ts = a.tstart[c];
    const uint32_t mask = (uint32_t)(a.tstart[c + 1] - ts - 1);
    table_add(tkeys + ts, tvals + ts, mask, d, a.pval[base + t]);
  }
}
void agg_part_insert(const AggArgs &a, int *tkeys, double *tvals, hipStream_t s) {
  if (a.nnz > 0) hipLaunchKernelGGL(k_agg_part_insert, (int)ceil_div(a.nnz, kChunk), 256, 0, s, a, tkeys, tvals);
}

// Emission of the merged partials: the table slots (community c owns
// [tstart[c], tstart[c+1])) are cut into chunks; each workgroup maps its
// slots to communities with an LDS max-scan, counts its used slots per
// community, reserves their output range with one atomic per community and
// writes them.
__global__ __launch_bounds__(256) void k_agg_part_emit(AggArgs a, const int *tkeys, const double *tvals,
                                                      int64_t tc, const int32_t *crow) {
  __shared__ int rowof[kChunk];
  __shared__ int cnt[kChunk];
  __shared__ int base[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, tc - q0);
  chunk_rows<kChunk>(a.tstart, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < kChunk; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    if (tkeys[q0 + t] == kEmpty) continue;
    int64_t s0 = a.tstart[rowof[t]] - q0;
    if (s0 < 0) s0 = 0;
    atomicAdd(&cnt[s0], 1);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int c = cnt[t];
    if (c > 0) {
      base[t] = atomicAdd(&a.rowlen[rowof[t]], c);
      cnt[t] = 0;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int d = tkeys[q0 + t];
    if (d == kEmpty) continue;
    const int r = rowof[t];
    int64_t s0 = a.tstart[r] - q0;
    if (s0 < 0) s0 = 0;
    const int pos = base[s0] + atomicAdd(&cnt[s0], 1);
    a.hidx[a.toff[r] + pos] = d;
    a.hw[a.toff[r] + pos] = (float)tvals[q0 + t];
  }
}
void agg_part_emit(const AggArgs &a, const int *tkeys, const double *tvals, int64_t tc, const int32_t *crow,
                   hipStream_t s) {
  if (tc > 0) hipLaunchKernelGGL(k_agg_part_emit, (int)ceil_div(tc, (int64_t)kChunk), 256, 0, s, a, tkeys, tvals, tc,
                                 crow);
}

// Compaction of the holey rows into the output CSR plus row sums.
__global__ __launch_bounds__(256) void k_agg_compact(AggArgs a, int64_t nnz2) {
  __shared__ int rowof[kChunk];
  __shared__ double ksum[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, nnz2 - q0);
  chunk_rows<kChunk>(a.out_off, q0, len, a.out_crow[blockIdx.x], a.out_crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < kChunk; t += blockDim.x) ksum[t] = 0.0;
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int r = rowof[t];
    const int64_t q = q0 + t;
    const int64_t src = a.toff[r] + (q - a.out_off[r]);
    const float x = a.hw[src];
    a.out_idx[q] = a.hidx[src];
    a.out_w[q] = x;
    int64_t s0 = a.out_off[r] - q0;
    if (s0 < 0) s0 = 0;
    atomicAdd(&ksum[s0], (double)x);
  }
  __syncthreads();
  if (a.out_K)
    for (int t = threadIdx.x; t < len; t += blockDim.x)
      if (t == 0 || rowof[t] != rowof[t - 1]) unsafeAtomicAdd(&a.out_K[rowof[t]], ksum[t]);
}
void agg_compact(const AggArgs &a, int64_t nnz_out, hipStream_t s) {
  if (nnz_out > 0) hipLaunchKernelGGL(k_agg_compact, (int)ceil_div(nnz_out, kChunk), 256, 0, s, a, nnz_out);
}

}  // namespace lk
