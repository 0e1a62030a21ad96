// Modularity, Eq. 1: Q = sum_c [sigma_c / 2m - (Sigma_c / 2m)^2], with sigma_c the
// weight of stored entries inside c and Sigma_c the total weight of c.  One
// chunked pass over the CSR accumulates the internal weight and the per-row
// sums, merged by community within the chunk before they are added to
// Sigma (FP64); a second pass over communities sums Sigma_c and
// (Sigma_c / 2m)^2.
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

__global__ __launch_bounds__(256) void k_mod_edges(const int64_t *off, const int32_t *idx, const float *w,
                                                   const int32_t *crow, int64_t nnz, const int32_t *C,
                                                   double *acc, double *S) {
  __shared__ int rowof[kChunk];
  __shared__ double ksum[kChunk];
  __shared__ int tk[2 * kChunk];
  __shared__ double tv[2 * kChunk];
  __shared__ int sh[16];
  __shared__ double sd[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, nnz - q0);
  chunk_rows<kChunk>(off, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < kChunk; t += blockDim.x) ksum[t] = 0.0;
  block_merge_clear<2 * kChunk>(tk, tv);
  double sig = 0.0;
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int r = rowof[t];
    const int64_t q = q0 + t;
    const double x = (double)w[q];
    if (C[idx[q]] == C[r]) sig += x;
    int64_t s0 = off[r] - q0;
    if (s0 < 0) s0 = 0;
    atomicAdd(&ksum[s0], x);
  }
  sig = block_sum(sig, sd);
  if (threadIdx.x == 0 && sig != 0.0) unsafeAtomicAdd(&acc[0], sig);
  // row sums -> Sigma of the row's community, merged per chunk (at most
  // kChunk distinct communities in the 2 * kChunk-slot table)
  for (int t = threadIdx.x; t < len; t += blockDim.x)
    if ((t == 0 || rowof[t] != rowof[t - 1]) && ksum[t] != 0.0)
      table_add(tk, tv, 2 * kChunk - 1, C[rowof[t]], ksum[t]);
  block_merge_flush<2 * kChunk>(tk, tv, S);
}

// Internal weight only (acc[0] += sum of entries inside a community): used
// when Sigma and 2m are already known.  W: float for a stored graph, double
// for the FP64 weights of an aggregated level.
template <class W>
__global__ __launch_bounds__(256) void k_mod_intra(const int64_t *off, const int32_t *idx, const W *w,
                                                   const int32_t *crow, int64_t nnz, const int32_t *C,
                                                   double *acc) {
  __shared__ int rowof[kChunk];
  __shared__ int sh[16];
  __shared__ double sd[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, nnz - q0);
  chunk_rows<kChunk>(off, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  // loads in two rounds, each issued together: ids, weights and row ids;
  // then both communities
  constexpr int PER = kChunk / 256;
  int j[PER], r[PER];
  W x[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * 256;
    j[k] = 0;
    r[k] = 0;
    x[k] = W(0);
    if (t < len) {
      j[k] = idx[q0 + t];
      x[k] = w[q0 + t];
      r[k] = rowof[t];
    }
  }
  double sig = 0.0;
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (threadIdx.x + k * 256 < len && C[j[k]] == C[r[k]]) sig += (double)x[k];
  sig = block_sum(sig, sd);
  if (threadIdx.x == 0 && sig != 0.0) unsafeAtomicAdd(&acc[0], sig);
}
void modularity_intra(const int64_t *off, const int32_t *idx, const float *w, const int32_t *crow, int64_t nnz,
                      const int32_t *C, double *acc, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_mod_intra<float>, (int)ceil_div(nnz, kChunk), 256, 0, s, off, idx, w, crow, nnz, C, acc);
}
void modularity_intra64(const int64_t *off, const int32_t *idx, const double *w, const int32_t *crow, int64_t nnz,
                        const int32_t *C, double *acc, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_mod_intra<double>, (int)ceil_div(nnz, kChunk), 256, 0, s, off, idx, w, crow, nnz, C, acc);
}

__global__ void k_scatter_labels(const int32_t *to, const int32_t *val, int64_t n, int32_t *out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[to[v]] = val[v];
}
void scatter_labels(const int32_t *to, const int32_t *val, int64_t n, int32_t *out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_labels, flat_grid(n), 256, 0, s, to, val, n, out);
}

void modularity_edges(const int64_t *off, const int32_t *idx, const float *w, const int32_t *crow,
                      int64_t n, int64_t nnz, const int32_t *C, double *acc, double *S, hipStream_t s) {
  (void)n;
  if (nnz > 0) hipLaunchKernelGGL(k_mod_edges, (int)ceil_div(nnz, kChunk), 256, 0, s, off, idx, w, crow, nnz, C, acc, S);
}

__global__ __launch_bounds__(256) void k_mod_comm(const double *S, int64_t n, double *acc) {
  __shared__ double sd[16];
  double t = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) t += S[c];
  t = block_sum(t, sd);
  if (threadIdx.x == 0 && t != 0.0) unsafeAtomicAdd(&acc[1], t);
}
void modularity_comm(const double *S, int64_t n, double *acc, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mod_comm, flat_grid(n, 256, 1024), 256, 0, s, S, n, acc);
}

__global__ __launch_bounds__(256) void k_mod_comm_sq(const double *S, int64_t n, double M2, double *acc) {
  __shared__ double sd[16];
  double t = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const double a = S[c] / M2;
    t += a * a;
  }
  t = block_sum(t, sd);
  if (threadIdx.x == 0 && t != 0.0) unsafeAtomicAdd(&acc[2], t);
}
void modularity_comm_sq(const double *S, int64_t n, double M2, double *acc, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mod_comm_sq, flat_grid(n, 256, 1024), 256, 0, s, S, n, M2, acc);
}

}  // namespace lk
