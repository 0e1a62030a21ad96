// Batch updates (Sec. 3.5, Sec. 5.1.4) and the dynamic front-ends.
//   build/validate: each undirected batch edge becomes two directed entries
//     keyed (src, dst); a deletion must exist in G^{t-1} (its weight is read
//     there), an insertion must not; ids, self-loops and weights are checked;
//   the entries are radix-sorted (rocPRIM) so duplicates are adjacent and
//     every row's batch entries form one segment ordered by dst;
//   apply: the new CSR keeps rows sorted - every surviving old entry and every
//     insertion gets its merged position from binary searches in the row's
//     segment and a prefix count of deletions;
//   marking: Alg. "dynamicFrontier", "deltaScreening", "naiveDynamic" and the
//     function "changedCommunities" of Alg. "leiden";
//   Alg. "updateWeights": K and Sigma of the previous membership (atomics).
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

__device__ __forceinline__ int64_t lower_bound_u64(const unsigned long long *a, int64_t lo, int64_t hi,
                                                   unsigned long long x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_batch_build(BatchArgs a) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.E; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e >> 1;
    const bool rev = (e & 1) != 0;
    const bool del = k < a.nd;
    int u, v;
    float x = 0.0f;
    if (del) { u = a.du[k]; v = a.dv[k]; }
    else { u = a.iu[k - a.nd]; v = a.iv[k - a.nd]; x = a.iw[k - a.nd]; }
    if (rev) { int t = u; u = v; v = t; }
    int errf = 0;
    if (u < 0 || (int64_t)u >= a.n || v < 0 || (int64_t)v >= a.n) {
      errf |= 1;
    } else if (u == v) {
      errf |= 2;
    } else {
      const int64_t lo = a.off[u], hi = a.off[u + 1];
      const int64_t pos = lower_bound_i32(a.idx, lo, hi, v);
      const bool found = pos < hi && a.idx[pos] == v;
      if (del) {
        if (!found) errf |= 8;
        else x = a.w[pos];
      } else {
        if (found) errf |= 16;
        if (!(x > 0.0f) || !isfinite(x)) errf |= 32;
      }
    }
    if (errf) atomicOr(a.err, errf);
    a.keys[e] = errf ? ~0ull : (((unsigned long long)(uint32_t)u << 32) | (uint32_t)v);
    a.vals[e] = (int32_t)e;
    a.ew[e] = x;
  }
}
void batch_build(const BatchArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_batch_build, flat_grid(a.E), 256, 0, s, a);
}

__global__ void k_batch_dups_rows(BatchArgs a) {
  const int64_t nd2 = 2 * a.nd;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= a.E; p += (int64_t)gridDim.x * blockDim.x) {
    if (p == a.E) { a.isdel[p] = 0; continue; }
    const unsigned long long key = a.skeys[p];
    const bool del = a.svals[p] < nd2;
    a.isdel[p] = del ? 1 : 0;
    const unsigned long long u = key >> 32;
    if (u >= (unsigned long long)a.n) { atomicOr(a.err, 64); continue; }
    if (p > 0 && a.skeys[p - 1] == key) atomicOr(a.err, 4);
    if (p == 0 || (a.skeys[p - 1] >> 32) != u) a.bstart[u] = p;
    atomicAdd(&a.bcnt[u], 1);
    atomicAdd(del ? &a.dcnt[u] : &a.icnt[u], 1);
  }
}
void batch_dups_rows(const BatchArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_dups_rows, flat_grid(a.E + 1), 256, 0, s, a);
}

__global__ void k_batch_newdeg(BatchArgs a) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= a.n; r += (int64_t)gridDim.x * blockDim.x) {
    if (r == a.n) { a.newdeg[r] = 0; continue; }
    a.newdeg[r] = (a.off[r + 1] - a.off[r]) - a.dcnt[r] + a.icnt[r];
  }
}
void batch_newdeg(const BatchArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_newdeg, flat_grid(a.n + 1), 256, 0, s, a);
}

__global__ __launch_bounds__(256) void k_batch_apply_old(BatchArgs a) {
  __shared__ int rowof[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, a.nnz - q0);
  chunk_rows<kChunk>(a.off, q0, len, a.crow[blockIdx.x], a.crow[blockIdx.x + 1], rowof, sh);
  // the thread's entries in two rounds of loads, each round's loads issued
  // together: ids, weights and the rows' batch counts and offsets; then the
  // places (a binary search in the row's sorted batch entries where it has
  // any) and the stores
  constexpr int PER = kChunk / 256;
  int x[PER], bc[PER], r[PER];
  float wv[PER];
  int64_t base[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * 256;
    x[k] = 0;
    bc[k] = 0;
    r[k] = 0;
    wv[k] = 0.0f;
    base[k] = 0;
    if (t < len) {
      r[k] = rowof[t];
      x[k] = a.idx[q0 + t];
      wv[k] = a.w[q0 + t];
      bc[k] = a.bcnt[r[k]];
      base[k] = a.newoff[r[k]] - a.off[r[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * 256;
    if (t >= len) continue;
    const int64_t q = q0 + t;
    int64_t pos = base[k] + q;
    if (bc[k] != 0) {
      const int64_t s0 = a.bstart[r[k]];
      const int64_t s1 = s0 + bc[k];
      const unsigned long long key = ((unsigned long long)(uint32_t)r[k] << 32) | (uint32_t)x[k];
      const int64_t p = lower_bound_u64(a.skeys, s0, s1, key);
      if (p < s1 && a.skeys[p] == key) continue;  // deleted
      const int64_t dl = a.delpre[p] - a.delpre[s0];
      const int64_t il = (p - s0) - dl;
      pos += il - dl;
    }
    a.nidx[pos] = x[k];
    a.nw[pos] = wv[k];
  }
}

__global__ void k_batch_apply_ins(BatchArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    if (a.isdel[p]) continue;
    const unsigned long long key = a.skeys[p];
    const int r = (int)(key >> 32);
    const int y = (int)(key & 0xffffffffull);
    const int64_t s0 = a.bstart[r];
    const int64_t old_lt = lower_bound_i32(a.idx, a.off[r], a.off[r + 1], y) - a.off[r];
    const int64_t dl = a.delpre[p] - a.delpre[s0];
    const int64_t il = (p - s0) - dl;
    const int64_t pos = a.newoff[r] + old_lt - dl + il;
    a.nidx[pos] = y;
    a.nw[pos] = a.ew[a.svals[p]];
  }
}

void batch_apply_old(const BatchArgs &a, hipStream_t s) {
  if (a.nnz > 0) hipLaunchKernelGGL(k_batch_apply_old, (int)ceil_div(a.nnz, kChunk), 256, 0, s, a);
}
void batch_apply_ins(const BatchArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_batch_apply_ins, flat_grid(a.E), 256, 0, s, a);
}

// ---- marking ---------------------------------------------------------------------
__global__ void k_mark_df(MarkArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = a.skeys[p];
    const int u = (int)(key >> 32), v = (int)(key & 0xffffffffull);
    const bool del = a.svals[p] < a.nd2;
    const int cu = a.C[u], cv = a.C[v];
    if (del ? (cu == cv) : (cu != cv)) a.dV[u] = 1;
    if (cu == cv) a.dC[cu] = 1;
  }
}
void mark_df(const MarkArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_mark_df, flat_grid(a.E), 256, 0, s, a);
}

__global__ void k_mark_changed(MarkArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = a.skeys[p];
    const int u = (int)(key >> 32), v = (int)(key & 0xffffffffull);
    const int cu = a.C[u];
    if (cu == a.C[v]) a.dC[cu] = 1;
  }
}
void mark_changed(const MarkArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_mark_changed, flat_grid(a.E), 256, 0, s, a);
}

__global__ void k_mark_ds_del(MarkArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = a.skeys[p];
    const int u = (int)(key >> 32), v = (int)(key & 0xffffffffull);
    const bool del = a.svals[p] < a.nd2;
    const int cu = a.C[u], cv = a.C[v];
    if (cu == cv) {
      a.dC[cu] = 1;
      if (del) { a.dV[u] = 1; a.dE[u] = 1; a.dCm[cv] = 1; }
    }
  }
}
void mark_ds_del(const MarkArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_mark_ds_del, flat_grid(a.E), 256, 0, s, a);
}

__global__ void k_mark_ds_keys(MarkArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = a.skeys[p];
    const int u = (int)(key >> 32), v = (int)(key & 0xffffffffull);
    const bool del = a.svals[p] < a.nd2;
    const int cu = a.C[u], cv = a.C[v];
    if (!del && cu != cv) {
      a.k2[p] = ((unsigned long long)(uint32_t)u << 32) | (uint32_t)cv;
      a.v2[p] = (double)a.ew[a.svals[p]];
    } else {
      a.k2[p] = ~0ull;
      a.v2[p] = 0.0;
    }
  }
}
void mark_ds_keys(const MarkArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_mark_ds_keys, flat_grid(a.E), 256, 0, s, a);
}

// Eq. 2 with the terms independent of the target community dropped.
__device__ __forceinline__ double ds_score(double M2, double h, double Ku, double Sc) {
#pragma clang fp contract(off)
  const double t1 = M2 * h;
  const double t2 = Ku * Sc;
  return t1 - t2;
}

// Per insertion source u (leader = first sorted (u, c) entry): sum inserted
// weight per community c, best c by M2*H[c] - K_u*Sigma_c (previous values),
// ties to the smaller c (keys ascend by c, strict comparison keeps the first).
__global__ void k_mark_ds_best(MarkArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = a.k2s[p];
    if (key == ~0ull) continue;
    const unsigned long long u = key >> 32;
    if (p > 0 && (a.k2s[p - 1] >> 32) == u) continue;
    const double Ku = a.K[u];
    int best = -1;
    double bestg = 0.0;
    int64_t q = p;
    while (q < a.E && a.k2s[q] != ~0ull && (a.k2s[q] >> 32) == u) {
      const unsigned long long kc = a.k2s[q];
      const int c = (int)(kc & 0xffffffffull);
      double h = 0.0;
      while (q < a.E && a.k2s[q] == kc) { h += a.v2s[q]; ++q; }
      const double g = ds_score(a.M2, h, Ku, a.Sig[c]);
      if (best < 0 || g > bestg) { best = c; bestg = g; }
    }
    a.dV[u] = 1;
    a.dE[u] = 1;
    a.dCm[best] = 1;
  }
}
void mark_ds_best(const MarkArgs &a, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_mark_ds_best, flat_grid(a.E), 256, 0, s, a);
}

__global__ void k_mark_ds_collect(MarkArgs a) {
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < a.n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    bool e = false;
    if (i < a.n) {
      e = a.dE[i] != 0;
      if (a.dCm[a.C[i]]) a.dV[i] = 1;
    }
    const int pos = wave_peel_inc(a.count, 0, e);
    if (e) a.list[pos] = (int32_t)i;
  }
}

__global__ __launch_bounds__(256) void k_mark_ds_nbrs(MarkArgs a) {
  const int count = *a.count;
  const int wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int k = wv; k < count; k += nw) {
    const int i = a.list[k];
    for (int64_t e = a.off[i] + lane(); e < a.off[i + 1]; e += kWave) a.dV[a.idx[e]] = 1;
  }
}

__global__ void k_copy_u8(const uint8_t *src, uint8_t *dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void mark_ds_expand(const MarkArgs &a, hipStream_t s) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_mark_ds_collect, flat_grid(a.n), 256, 0, s, a);
  hipLaunchKernelGGL(k_mark_ds_nbrs, flat_grid(a.E > 0 ? a.E * kWave : kWave, 256, 2048), 256, 0, s, a);
  hipLaunchKernelGGL(k_copy_u8, flat_grid(a.n), 256, 0, s, a.dV, a.rng, a.n);
}

__global__ __launch_bounds__(256) void k_update_weights(MarkArgs a, double *K, double *Sig, double *m2delta) {
  __shared__ double sd[16];
  double t = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.E; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = a.skeys[p];
    const int u = (int)(key >> 32);
    const bool del = a.svals[p] < a.nd2;
    const double x = (double)a.ew[a.svals[p]];
    const double dx = del ? -x : x;
    unsafeAtomicAdd(&K[u], dx);
    unsafeAtomicAdd(&Sig[a.C[u]], dx);
    t += dx;
  }
  t = block_sum(t, sd);
  if (threadIdx.x == 0 && t != 0.0) unsafeAtomicAdd(m2delta, t);
}
void update_weights(const MarkArgs &a, double *K, double *Sig, double *m2delta, hipStream_t s) {
  if (a.E > 0) hipLaunchKernelGGL(k_update_weights, flat_grid(a.E, 256, 1024), 256, 0, s, a, K, Sig, m2delta);
}

}  // namespace lk
