// Utility kernels: fills, label maps, CSR chunk mapping, row sums, checks,
// degree buckets.

#include "device.hpp"
#include "kernels.hpp"

namespace lk {

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill<int32_t>, flat_grid(n), 256, 0, s, p, v, n);
}
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill<uint8_t>, flat_grid(n), 256, 0, s, p, v, n);
}
void fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill<double>, flat_grid(n), 256, 0, s, p, v, n);
}
void fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill<unsigned long long>, flat_grid(n), 256, 0, s, p, v, n);
}

__global__ void k_iota(int32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}
void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_iota, flat_grid(n), 256, 0, s, p, n);
}

__global__ void k_chunk_start_rows(const int64_t *off, int64_t nrows, int64_t nnz, int32_t *out) {
  const int64_t nchunks = ceil_div(nnz, kChunk);
  if (blockIdx.x == 0 && threadIdx.x == 0) out[nchunks] = (int32_t)(nrows > 0 ? nrows - 1 : 0);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = off[r], b = off[r + 1];
    if (a == b) continue;
    int64_t q = ceil_div(a, kChunk) * kChunk;
    for (; q < b; q += kChunk) out[q / kChunk] = (int32_t)r;
  }
}
void chunk_start_rows(const int64_t *off, int64_t nrows, int64_t nnz, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_start_rows, flat_grid(nrows), 256, 0, s, off, nrows, nnz, out);
}

// Row sums over CSR chunks: each block owns kChunk consecutive positions,
// accumulates per-row partial sums in LDS and adds them to K once per row.
__global__ __launch_bounds__(256) void k_row_sums(const int64_t *off, const float *w, int64_t nnz,
                                                  const int32_t *crow, double *K) {
  __shared__ int rowof[kChunk];
  __shared__ double ksum[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, nnz - q0);
  chunk_rows<kChunk>(off, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < kChunk; t += blockDim.x) ksum[t] = 0.0;
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int r = rowof[t];
    int64_t s0 = off[r] - q0;
    if (s0 < 0) s0 = 0;
    atomicAdd(&ksum[s0], (double)w[q0 + t]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    if (t == 0 || rowof[t] != rowof[t - 1]) unsafeAtomicAdd(&K[rowof[t]], ksum[t]);
  }
}
void row_sums(const int64_t *off, const float *w, int64_t nrows, int64_t nnz, const int32_t *crow,
              double *K, hipStream_t s) {
  (void)nrows;
  if (nnz > 0) hipLaunchKernelGGL(k_row_sums, (int)ceil_div(nnz, kChunk), 256, 0, s, off, w, nnz, crow, K);
}

// out[C[i]] += v[i] (zero values skipped), merged per workgroup by key.
constexpr int kScatterItems = 1024;
__global__ __launch_bounds__(256) void k_scatter_add(const double *v, const int32_t *C, int64_t n, double *out) {
  __shared__ int tk[2 * kScatterItems];
  __shared__ double tv[2 * kScatterItems];
  block_merge_clear<2 * kScatterItems>(tk, tv);
  for (int64_t i0 = (int64_t)blockIdx.x * kScatterItems; i0 < n; i0 += (int64_t)gridDim.x * kScatterItems) {
    for (int t = threadIdx.x; t < kScatterItems; t += blockDim.x) {
      const int64_t i = i0 + t;
      if (i < n && v[i] != 0.0) table_add(tk, tv, 2 * kScatterItems - 1, C[i], v[i]);
    }
    block_merge_flush<2 * kScatterItems>(tk, tv, out);
  }
}
void scatter_add(const double *v, const int32_t *C, int64_t n, double *out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_add, (int)std::min<int64_t>(ceil_div(n, kScatterItems), 2048), 256, 0, s, v, C, n, out);
}

__global__ void k_gather_map(int32_t *C, const int32_t *map, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    C[i] = map[C[i]];
}
void gather_map(int32_t *C, const int32_t *map, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gather_map, flat_grid(n), 256, 0, s, C, map, n);
}

__global__ void k_gather_map_bounded(int32_t *C, const int32_t *map, int64_t n, int64_t bound) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = C[i];
    if (c < bound) C[i] = map[c];
  }
}
void gather_map_bounded(int32_t *C, const int32_t *map, int64_t n, int64_t bound, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gather_map_bounded, flat_grid(n), 256, 0, s, C, map, n, bound);
}

__global__ void k_mark_used_active(const int32_t *C, const int64_t *off, int64_t n, int32_t *used, int32_t *act) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = C[i];
    used[c] = 1;
    if (off[i + 1] > off[i]) act[c] = 1;
  }
}
void mark_used_active(const int32_t *C, const int64_t *off, int64_t n, int32_t *used, int32_t *act, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mark_used_active, flat_grid(n), 256, 0, s, C, off, n, used, act);
}
__global__ void k_flags_inactive(int32_t *used, const int32_t *act, int64_t n) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    used[c] = used[c] && !act[c];
}
void flags_inactive(int32_t *used, const int32_t *act, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_flags_inactive, flat_grid(n), 256, 0, s, used, act, n);
}
__global__ void k_active_first_map(const int32_t *act, const int32_t *pa, const int32_t *pi, int64_t na, int64_t n,
                                   int32_t *map) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    map[c] = act[c] ? pa[c] : (int32_t)(na + pi[c]);
}
void active_first_map(const int32_t *act, const int32_t *pa, const int32_t *pi, int64_t na, int64_t n, int32_t *map,
                      hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_active_first_map, flat_grid(n), 256, 0, s, act, pa, pi, na, n, map);
}

__global__ void k_mark_used(const int32_t *C, int64_t n, int32_t *flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flags[C[i]] = 1;
}
void mark_used(const int32_t *C, int64_t n, int32_t *flags, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mark_used, flat_grid(n), 256, 0, s, C, n, flags);
}



__global__ void k_check_labels(const int32_t *C, int64_t n, int64_t bound, int32_t *err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (C[i] < 0 || (int64_t)C[i] >= bound) atomicOr(err, 1);
}
void check_labels(const int32_t *C, int64_t n, int64_t bound, int32_t *err, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_check_labels, flat_grid(n), 256, 0, s, C, n, bound, err);
}

__global__ void k_check_offsets(const int64_t *off, int64_t n, int64_t nnz, int32_t *err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (off[i] > off[i + 1] || off[i] < 0 || off[i + 1] > nnz) atomicOr(err, 1);
  if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != nnz)) atomicOr(err, 1);
}
void check_offsets(const int64_t *off, int64_t n, int64_t nnz, int32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(k_check_offsets, flat_grid(n > 0 ? n : 1), 256, 0, s, off, n, nnz, err);
}

// Rows must be strictly ascending (sorted, no duplicate entries), ids in
// range, weights finite and > 0.  Chunked over positions.
__global__ __launch_bounds__(256) void k_check_rows(const int64_t *off, const int32_t *idx, const float *w,
                                                    int64_t n, int64_t nnz, const int32_t *crow,
                                                    int32_t *err) {
  __shared__ int rowof[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, nnz - q0);
  chunk_rows<kChunk>(off, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int64_t q = q0 + t;
    const int r = rowof[t];
    const int j = idx[q];
    const float x = w[q];
    bool bad = j < 0 || (int64_t)j >= n || !(x > 0.0f) || !isfinite(x);
    if (q > off[r] && idx[q - 1] >= j) bad = true;
    if (bad) atomicOr(err, 1);
  }
}
void check_rows_chunked(const int64_t *off, const int32_t *idx, const float *w, int64_t n, int64_t nnz,
                        const int32_t *crow, int32_t *err, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_check_rows, (int)ceil_div(nnz, kChunk), 256, 0, s, off, idx, w, n, nnz, crow, err);
}

}  // namespace lk

namespace lk {
__global__ __launch_bounds__(256) void k_count_nz(const uint8_t *p, int64_t n, unsigned long long *out) {
  __shared__ long long sl[16];
  long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += p[i] != 0;
  c = block_sum_ll(c, sl);
  if (threadIdx.x == 0 && c) atomicAdd(out, (unsigned long long)c);
}
void count_nonzero_u8(const uint8_t *p, int64_t n, unsigned long long *out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_count_nz, flat_grid(n, 256, 1024), 256, 0, s, p, n, out);
}
__global__ void k_copy_bytes(const uint8_t *src, uint8_t *dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
// Per-iteration counters cleared in one launch: n ints and up to three
// scalars (each nullable).
__global__ void k_reset_iter(int32_t *counts, int n, double *d0, unsigned long long *u0, unsigned long long *u1) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) counts[i] = 0;
  if (threadIdx.x == 0) {
    if (d0) *d0 = 0.0;
    if (u0) *u0 = 0ull;
    if (u1) *u1 = 0ull;
  }
}
void reset_iter(int32_t *counts, int n, double *d0, unsigned long long *u0, unsigned long long *u1, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_iter, 1, 256, 0, s, counts, n, d0, u0, u1);
}
void copy_u8(const uint8_t *src, uint8_t *dst, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy_bytes, flat_grid(n), 256, 0, s, src, dst, n);
}
}  // namespace lk
