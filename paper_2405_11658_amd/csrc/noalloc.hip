// leiden_modularity_noalloc (include/leiden.h): Eq. 1 for callers that cannot
// allocate (code under stream capture, tight serving loops).  The working
// arrays live in one fixed device array of this library; nothing is
// allocated or freed, and the result stays on the device (no host wait).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "device.hpp"
#include "leiden.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // per device, held until the process ends
constexpr int kMaxDevices = 64;
constexpr size_t kHead = 256;                        // acc[4] + error flag, then S[n]

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device.
hipError_t scratch_ptr(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

// acc[0]: sum of intra-community entries; acc[1]: 2m; acc[2]: sum of
// (S_c / 2m)^2; err: bit 1 = a label or neighbour id out of range.
struct Head {
  double acc[4];
  int err;
};

__global__ void k_na_clear(Head *h, double *S, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    for (int k = 0; k < 4; ++k) h->acc[k] = 0.0;
    h->err = 0;
  }
  for (int64_t c = t; c < n; c += (int64_t)gridDim.x * blockDim.x) S[c] = 0.0;
}

// One thread per row: S[C[u]] += K_u, intra-community weight into acc[0].
__global__ void k_na_rows(const int64_t *off, const int32_t *idx, const float *w, const int32_t *C, int64_t n,
                          Head *h, double *S) {
  __shared__ double red[16];
  double in = 0.0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int cu = C[u];
    if (cu < 0 || cu >= n) {
      atomicOr(&h->err, 1);
      continue;
    }
    double k = 0.0;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int v = idx[e];
      const double x = (double)w[e];
      k += x;
      if (v < 0 || v >= n) {
        atomicOr(&h->err, 1);
        continue;
      }
      if (C[v] == cu) in += x;
    }
    if (k != 0.0) unsafeAtomicAdd(&S[cu], k);
  }
  const double b = lk::block_sum(in, red);
  if (threadIdx.x == 0 && b != 0.0) unsafeAtomicAdd(&h->acc[0], b);
}

// acc[1] = sum of S (= 2m)
__global__ void k_na_total(const double *S, int64_t n, Head *h) {
  __shared__ double red[16];
  double t = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    t += S[c];
  const double b = lk::block_sum(t, red);
  if (threadIdx.x == 0 && b != 0.0) unsafeAtomicAdd(&h->acc[1], b);
}

// acc[2] = sum of (S_c / 2m)^2, 2m read from acc[1]
__global__ void k_na_squares(const double *S, int64_t n, Head *h) {
  __shared__ double red[16];
  const double M2 = __hip_atomic_load(&h->acc[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double t = 0.0;
  if (M2 > 0.0)
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
      const double a = S[c] / M2;
      t += a * a;
    }
  const double b = lk::block_sum(t, red);
  if (threadIdx.x == 0 && b != 0.0) unsafeAtomicAdd(&h->acc[2], b);
}

__global__ void k_na_final(Head *h, double *q) {
  const double M2 = h->acc[1];
  double r = M2 > 0.0 ? h->acc[0] / M2 - h->acc[2] : 0.0;
  if (h->err) r = NAN;
  *q = r;
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : g > 2048 ? 2048 : g);
}

}  // namespace

extern "C" leiden_status leiden_modularity_noalloc(int64_t n, int64_t nnz, const int64_t *offsets,
                                                   const int32_t *indices, const float *weights,
                                                   const int32_t *membership, double *q_out, void *stream) {
  if (n < 0 || nnz < 0 || !q_out || (n > 0 && (!offsets || !membership)) || (nnz > 0 && (!indices || !weights)))
    return LEIDEN_EINVAL;
  if (kHead + (size_t)n * sizeof(double) > kScratchBytes) return LEIDEN_EINVAL;
  void *base = nullptr;
  if (scratch_ptr(&base) != hipSuccess) return LEIDEN_EHIP;
  hipStream_t s = (hipStream_t)stream;
  Head *h = (Head *)base;
  double *S = (double *)((char *)base + kHead);
  hipLaunchKernelGGL(k_na_clear, grid_for(n), 256, 0, s, h, S, n);
  if (n > 0) {
    hipLaunchKernelGGL(k_na_rows, grid_for(n), 256, 0, s, offsets, indices, weights, membership, n, h, S);
    hipLaunchKernelGGL(k_na_total, grid_for(n), 256, 0, s, S, n, h);
    hipLaunchKernelGGL(k_na_squares, grid_for(n), 256, 0, s, S, n, h);
  }
  hipLaunchKernelGGL(k_na_final, 1, 1, 0, s, h, q_out);
  return hipGetLastError() == hipSuccess ? LEIDEN_OK : LEIDEN_EHIP;
}

extern "C" int64_t leiden_modularity_noalloc_max_vertices(void) {
  return (int64_t)((kScratchBytes - kHead) / sizeof(double));
}
