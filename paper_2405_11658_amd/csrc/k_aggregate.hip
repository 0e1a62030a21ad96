// Aggregation (Alg. "leidenAggregate"): the super-vertex graph of a level.
//
// GPU design.  Instead of one hash table per community (the paper's per-thread
// tables), every CSR entry (u, v, w) becomes the 64-bit key
// C[u] * ncomm + C[v] with value w (one coalesced pass, one gather of C[v]);
// a radix sort over the key bits in use (2 * ceil(log2 ncomm)) and a
// deterministic reduce-by-key (FP64 sums of the float weights, fixed order)
// leave the distinct (community, community) pairs sorted, i.e. the output
// entries already in CSR order with rows sorted by neighbour id.  On large
// levels the communities that own entries are first relabelled densely (in
// increasing order, so the sorted order is kept), which drops the edgeless
// singletons from the key space and saves radix passes.  A last pass
// splits the keys into (row, id), stores the weights rounded to float32 and
// accumulates the row lengths and row sums (the next level's K' = Sigma');
// a scan of the lengths gives the offsets.  All work is streaming except the C[v] gather, and the
// result does not depend on scheduling.
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

__global__ __launch_bounds__(256) void k_agg_keys(AggArgs a, const int32_t *crow, unsigned long long *keys,
                                                  float *vals) {
  __shared__ int rowof[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, a.nnz - q0);
  chunk_rows<kChunk>(a.off, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int64_t e = q0 + t;
    const int u = rowof[t];
    keys[e] = (unsigned long long)(uint32_t)a.C[u] * (unsigned long long)a.ncomm + (uint32_t)a.C[a.idx[e]];
    vals[e] = a.w[e];
  }
}
void agg_keys(const AggArgs &a, const int32_t *crow, unsigned long long *keys, float *vals, hipStream_t s) {
  if (a.nnz > 0) hipLaunchKernelGGL(k_agg_keys, (int)ceil_div(a.nnz, kChunk), 256, 0, s, a, crow, keys, vals);
}

// Dense relabelling of the communities that own entries (on large levels, so
// that the keys need fewer bits): flag[C[u]] = 1 for every u with edges; after
// an exclusive scan cmap of flag, Cc[u] = cmap[C[u]] and inv[cmap[c]] = c.
__global__ void k_agg_flag(int64_t n, const int64_t *off, const int32_t *C, int32_t *flag) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    if (off[u + 1] > off[u]) flag[C[u]] = 1;
}
__global__ void k_agg_relabel(int64_t n, const int64_t *off, const int32_t *C, const int32_t *cmap, int32_t *Cc) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    Cc[u] = off[u + 1] > off[u] ? cmap[C[u]] : 0;
}
__global__ void k_agg_inv(int64_t ncomm, const int32_t *flag, const int32_t *cmap, int32_t *inv) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncomm; c += (int64_t)gridDim.x * blockDim.x)
    if (flag[c]) inv[cmap[c]] = (int32_t)c;
}
void agg_flag(int64_t n, const int64_t *off, const int32_t *C, int32_t *flag, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_agg_flag, flat_grid(n), 256, 0, s, n, off, C, flag);
}
void agg_relabel(int64_t n, const int64_t *off, const int32_t *C, const int32_t *cmap, int32_t *Cc, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_agg_relabel, flat_grid(n), 256, 0, s, n, off, C, cmap, Cc);
}
void agg_inv(int64_t ncomm, const int32_t *flag, const int32_t *cmap, int32_t *inv, hipStream_t s) {
  if (ncomm > 0) hipLaunchKernelGGL(k_agg_inv, flat_grid(ncomm), 256, 0, s, ncomm, flag, cmap, inv);
}

// Distinct sorted keys -> output entries (in place: position k of the sorted
// distinct keys is the CSR position), row lengths and, with K given, row sums
// of the stored float weights (the next level's K').  Rows are contiguous
// runs, so each wavefront adds one count and one sum per run it holds.
__global__ void k_agg_rows(const unsigned long long *ukeys, const double *sums, int64_t nu, int64_t ncomm,
                           const int32_t *inv, int32_t *out_idx, float *out_w, int32_t *rowlen, double *K) {
  for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < nu; k0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    const bool act = k < nu;
    int r = 0;
    double x = 0.0;
    if (act) {
      const unsigned long long key = ukeys[k];
      r = (int)(key / (unsigned long long)ncomm);
      int col = (int)(key % (unsigned long long)ncomm);
      if (inv) {
        r = inv[r];
        col = inv[col];
      }
      const float wf = (float)sums[k];
      out_idx[k] = (int32_t)col;
      out_w[k] = wf;
      x = (double)wf;
    }
    unsigned long long pending = __ballot(act);
    while (pending) {
      const int leader = __ffsll(pending) - 1;
      const int rk = __shfl(r, leader);
      const bool mine = ((pending >> lane()) & 1ull) && r == rk;
      const unsigned long long grp = __ballot(mine);
      const double sum = group_sum<kWave>(mine ? x : 0.0);
      if (lane() == leader) {
        atomicAdd(&rowlen[rk], (int)__popcll(grp));
        if (K) unsafeAtomicAdd(&K[rk], sum);
      }
      pending &= ~grp;
    }
  }
}
void agg_rows(const unsigned long long *ukeys, const double *sums, int64_t nu, int64_t ncomm, const int32_t *inv,
              int32_t *out_idx, float *out_w, int32_t *rowlen, double *K, hipStream_t s) {
  if (nu > 0)
    hipLaunchKernelGGL(k_agg_rows, flat_grid(nu), 256, 0, s, ukeys, sums, nu, ncomm, inv, out_idx, out_w, rowlen,
                       K);
}

}  // namespace lk
