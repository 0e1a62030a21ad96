// Aggregation (Alg. "leidenAggregate"): the super-vertex graph of a level.
//
// GPU design.  The paper merges each community's edges in a per-thread hash
// table.  Here the entries are first grouped by the community of their
// source, then each group is sorted by the community of the neighbour and
// equal neighbours are summed, so every group becomes one row of the output
// CSR, sorted by neighbour id:
//   1. vertices ordered by community (stable radix sort of (C[u], u));
//   2. a scan of the degrees in that order gives every vertex's place in the
//      grouped entry array, and every community's segment [seg[c], seg[c+1]);
//   3. one streaming pass writes (C[v], w) of every entry to its place;
//   4. segments of at most kAggSmall entries: a workgroup takes the segments
//      that start in one kAggSmall-entry window (at most 2 * kAggSmall
//      entries), sorts them in LDS by (segment, neighbour) with a bitonic
//      network, and sums the runs of equal keys;
//   5. larger segments: a segmented radix sort by neighbour (tiles of 4096
//      entries that never cross a segment), then the runs are summed with a
//      segmented scan per tile plus the continuation pieces of the following
//      tiles, all in a fixed order;
//   6. a scan of the row lengths gives the offsets, and the rows are copied
//      into place.
// Weights are summed in FP64 and stored rounded to float32; the next level's
// K' is the FP64 sum of the stored row weights.  Every sum is taken in an
// order fixed by the input, so results do not depend on scheduling.
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

constexpr int kSmallCap = 2 * kAggSmall;  // entries of one small-segment window

// ---- 1-3: community order and grouped entries ---------------------------------
__global__ void k_agg_vkeys(int64_t n, const int32_t *C, uint32_t *keys, int32_t *vals) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    keys[u] = (uint32_t)C[u];
    vals[u] = (int32_t)u;
  }
}
void agg_vkeys(int64_t n, const int32_t *C, uint32_t *keys, int32_t *vals, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_agg_vkeys, flat_grid(n), 256, 0, s, n, C, keys, vals);
}

// deg[i] = degree of the i-th vertex in community order (deg[n] = 0), pos = inverse order
__global__ void k_agg_vdeg(int64_t n, const int64_t *off, const int32_t *vs, int64_t *deg, int32_t *pos) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {
      deg[n] = 0;
      continue;
    }
    const int u = vs[i];
    deg[i] = off[u + 1] - off[u];
    pos[u] = (int32_t)i;
  }
}
void agg_vdeg(int64_t n, const int64_t *off, const int32_t *vs, int64_t *deg, int32_t *pos, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_vdeg, flat_grid(n + 1), 256, 0, s, n, off, vs, deg, pos);
}

// Entries per community: hpos[c] = first place of c's entries (at c's first
// member in community order), then cdeg[c] = end of c's last member - hpos[c].
__global__ void k_agg_heads(int64_t n, const uint32_t *Cs, const int64_t *eoff, int64_t *hpos) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (i == 0 || Cs[i] != Cs[i - 1]) hpos[Cs[i]] = eoff[i];
}
__global__ void k_agg_tails(int64_t n, const uint32_t *Cs, const int64_t *eoff, const int64_t *hpos, int64_t *cdeg) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (i == n - 1 || Cs[i + 1] != Cs[i]) cdeg[Cs[i]] = eoff[i + 1] - hpos[Cs[i]];
}
void agg_cdeg(int64_t n, const uint32_t *Cs, const int64_t *eoff, int64_t *hpos, int64_t *cdeg, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_agg_heads, flat_grid(n), 256, 0, s, n, Cs, eoff, hpos);
  hipLaunchKernelGGL(k_agg_tails, flat_grid(n), 256, 0, s, n, Cs, eoff, (const int64_t *)hpos, cdeg);
}

// (C[v], w) of entry e of row u to its place eoff[pos[u]] + (e - off[u]).
__global__ __launch_bounds__(256) void k_agg_group(AggArgs a, const int32_t *crow, const int32_t *pos,
                                                   const int64_t *eoff, uint32_t *gkey, float *gval) {
  __shared__ int rowof[kChunk];
  __shared__ int sh[16];
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, a.nnz - q0);
  chunk_rows<kChunk>(a.off, q0, len, crow[blockIdx.x], crow[blockIdx.x + 1], rowof, sh);
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int64_t e = q0 + t;
    const int u = rowof[t];
    const int64_t dst = eoff[pos[u]] + (e - a.off[u]);
    gkey[dst] = (uint32_t)a.C[a.idx[e]];
    gval[dst] = a.w[e];
  }
}
void agg_group(const AggArgs &a, const int32_t *crow, const int32_t *pos, const int64_t *eoff, uint32_t *gkey,
               float *gval, hipStream_t s) {
  if (a.nnz > 0)
    hipLaunchKernelGGL(k_agg_group, (int)ceil_div(a.nnz, kChunk), 256, 0, s, a, crow, pos, eoff, gkey, gval);
}

// ---- 4: small segments -------------------------------------------------------
// tfc[t] = first community whose segment starts at or after t * kAggSmall
// (t in [0, nst]); window t holds the communities [tfc[t], tfc[t + 1]).
__global__ void k_agg_windows(const int64_t *seg, int64_t ncomm, int64_t nst, int32_t *tfc) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= nst; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t at = t * kAggSmall;
    int64_t lo = 0, hi = ncomm;  // first c in [0, ncomm] with seg[c] >= at (seg[ncomm] = nnz)
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (seg[mid] >= at) hi = mid;
      else lo = mid + 1;
    }
    tfc[t] = (int32_t)(t == nst ? ncomm : lo);
  }
}
void agg_windows(const int64_t *seg, int64_t ncomm, int64_t nst, int32_t *tfc, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_windows, flat_grid(nst + 1), 256, 0, s, seg, ncomm, nst, tfc);
}

__device__ __forceinline__ int blk_excl_int(int x, int *tot, int *sw) {
  int incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane() >= o) incl += y;
  }
  const int w = (int)threadIdx.x / kWave;
  if (lane() == kWave - 1) sw[w] = incl;
  __syncthreads();
  int pre = 0, all = 0;
  for (int k = 0; k < (int)blockDim.x / kWave; ++k) {
    if (k < w) pre += sw[k];
    all += sw[k];
  }
  __syncthreads();
  *tot = all;
  return pre + incl - x;
}

__global__ __launch_bounds__(256) void k_agg_small(const int64_t *seg, const int32_t *tfc, int cb,
                                                   const uint32_t *gkey, const float *gval, uint32_t *ukey,
                                                   float *uval, int32_t *rowlen, double *K) {
  __shared__ unsigned long long ck[kSmallCap];
  __shared__ float cv[kSmallCap];
  __shared__ int lo[kSmallCap + 1];   // window place of each small segment, then the end
  __shared__ int com[kSmallCap];      // community of each small segment
  __shared__ int hr[kSmallCap + 1];   // exclusive rank of each run head
  __shared__ int sw[16];
  __shared__ int tot_s, tot_m;
  const int64_t t = blockIdx.x;
  const int c0 = tfc[t], c1 = tfc[t + 1];
  if (threadIdx.x == 0) { tot_s = 0; tot_m = 0; }
  __syncthreads();
  // the window's small, non-empty segments, in community order
  for (int b = c0; b < c1; b += blockDim.x) {
    const int c = b + (int)threadIdx.x;
    int64_t len = 0;
    if (c < c1) len = seg[c + 1] - seg[c];
    const bool small = len > 0 && len <= kAggSmall;
    int ts, tm;
    const int is = blk_excl_int(small ? 1 : 0, &ts, sw);
    const int im = blk_excl_int(small ? (int)len : 0, &tm, sw);
    const int s0 = tot_s, m0 = tot_m;
    if (small) {
      com[s0 + is] = c;
      lo[s0 + is] = m0 + im;
    }
    __syncthreads();
    if (threadIdx.x == 0) { tot_s = s0 + ts; tot_m = m0 + tm; }
    __syncthreads();
  }
  const int ns = tot_s, m = tot_m;
  if (ns == 0) return;  // uniform
  if (threadIdx.x == 0) lo[ns] = m;
  __syncthreads();
  int P = 2;
  while (P < m) P <<= 1;
  const uint32_t kmask = cb >= 32 ? 0xffffffffu : ((1u << cb) - 1u);
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    if (p >= m) {
      ck[p] = ~0ull;
      cv[p] = 0.0f;
      continue;
    }
    int l = 0, h = ns;  // lo[l] <= p < lo[h]
    while (h - l > 1) {
      const int mid = (l + h) >> 1;
      if (lo[mid] <= p) l = mid;
      else h = mid;
    }
    const int64_t src = seg[com[l]] + (p - lo[l]);
    ck[p] = ((unsigned long long)l << cb) | (unsigned long long)(gkey[src] & kmask);
    cv[p] = gval[src];
  }
  __syncthreads();
  // bitonic sort of the window by (segment, neighbour): a fixed network, so
  // equal keys end in an order fixed by the input
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int ix = i ^ j;
        if (ix > i) {
          const unsigned long long a = ck[i], bk = ck[ix];
          const bool up = (i & k) == 0;
          if ((a > bk) == up) {
            ck[i] = bk;
            ck[ix] = a;
            const float va = cv[i];
            cv[i] = cv[ix];
            cv[ix] = va;
          }
        }
      }
      __syncthreads();
    }
  }
  // run heads and their ranks
  int carry = 0;
  for (int b = 0; b < m; b += blockDim.x) {
    const int p = b + (int)threadIdx.x;
    const bool head = p < m && (p == 0 || ck[p] != ck[p - 1]);
    int tt;
    const int r = blk_excl_int(head ? 1 : 0, &tt, sw);
    if (p < m) hr[p] = carry + r;
    carry += tt;
  }
  if (threadIdx.x == 0) hr[m] = carry;
  __syncthreads();
  // run sums (sequential within the run) ...
  double rs[kSmallCap / 256];
  int rp[kSmallCap / 256];
  int nr = 0;
  for (int p = threadIdx.x; p < m; p += blockDim.x) {
    if (!(p == 0 || ck[p] != ck[p - 1])) continue;
    double x = 0.0;
    for (int q = p; q < m && ck[q] == ck[p]; ++q) x += (double)cv[q];
    rs[nr] = x;
    rp[nr] = p;
    ++nr;
  }
  __syncthreads();
  // ... stored at the run's rank in the segment's row, and kept in LDS for K'
  for (int k = 0; k < nr; ++k) {
    const int p = rp[k];
    const int l = (int)(ck[p] >> cb);
    const int c = com[l];
    const int j = hr[p] - hr[lo[l]];
    const float wf = (float)rs[k];
    ukey[seg[c] + j] = (uint32_t)(ck[p] & kmask);
    uval[seg[c] + j] = wf;
    cv[hr[p]] = wf;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < ns; l += blockDim.x) {
    const int c = com[l];
    const int r0 = hr[lo[l]], r1 = hr[lo[l + 1]];
    rowlen[c] = r1 - r0;
    if (K) {
      double x = 0.0;
      for (int r = r0; r < r1; ++r) x += (double)cv[r];
      K[c] = x;
    }
  }
}
void agg_small(const int64_t *seg, const int32_t *tfc, int64_t nst, int cb, const uint32_t *gkey, const float *gval,
               uint32_t *ukey, float *uval, int32_t *rowlen, double *K, hipStream_t s) {
  if (nst > 0)
    hipLaunchKernelGGL(k_agg_small, (int)nst, 256, 0, s, seg, tfc, cb, gkey, gval, ukey, uval, rowlen, K);
}

// ---- 5: large segments ----------------------------------------------------------
__global__ void k_agg_lflag(const int64_t *seg, int64_t ncomm, int32_t *flag) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= ncomm; c += (int64_t)gridDim.x * blockDim.x)
    flag[c] = c < ncomm && seg[c + 1] - seg[c] > kAggSmall;
}
// lc[l] = community of large segment l, [lsb, lse) its entries, ltn[l] its tile count (ltn[nl] = 0)
__global__ void k_agg_llist(const int64_t *seg, int64_t ncomm, const int32_t *flag, const int32_t *lidx, int32_t *lc,
                            int64_t *lsb, int64_t *lse, int64_t *ltn) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= ncomm;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (c == ncomm) {
      ltn[lidx[ncomm]] = 0;
      continue;
    }
    if (!flag[c]) continue;
    const int l = lidx[c];
    lc[l] = (int32_t)c;
    lsb[l] = seg[c];
    lse[l] = seg[c + 1];
    ltn[l] = ceil_div(seg[c + 1] - seg[c], kPTile);
  }
}
__global__ void k_agg_tseg(const int64_t *tfirst, int64_t nl, int32_t *tseg) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nl; l += (int64_t)gridDim.x * blockDim.x)
    for (int64_t t = tfirst[l]; t < tfirst[l + 1]; ++t) tseg[t] = (int32_t)l;
}
void agg_large_list(const int64_t *seg, int64_t ncomm, int32_t *flag, const int32_t *lidx, int32_t *lc, int64_t *lsb,
                    int64_t *lse, int64_t *ltn, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_llist, flat_grid(ncomm + 1), 256, 0, s, seg, ncomm, (const int32_t *)flag, lidx, lc, lsb,
                     lse, ltn);
}
void agg_large_flags(const int64_t *seg, int64_t ncomm, int32_t *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_lflag, flat_grid(ncomm + 1), 256, 0, s, seg, ncomm, flag);
}
void agg_tile_seg(const int64_t *tfirst, int64_t nl, int32_t *tseg, hipStream_t s) {
  if (nl > 0) hipLaunchKernelGGL(k_agg_tseg, flat_grid(nl), 256, 0, s, tfirst, nl, tseg);
}

// Runs of equal neighbours in the sorted large segments.  A segmented
// inclusive scan (FP64, fixed order) over each tile gives at every run end the
// sum of the run's piece inside the tile.
//   pass 0: hc[t] = run heads in tile t, tin[t] = the tile's leading piece of
//           a run that started in an earlier tile (0 if the tile starts with a
//           head);
//   pass 1: (hc scanned) each run whose head lies in tile t is written at its
//           rank in the segment's row: its piece plus the leading pieces of the
//           following tiles it covers.
template <int PASS>
__global__ __launch_bounds__(256) void k_agg_lruns(const uint32_t *gkey, const float *gval, RsSeg g, int64_t *hc,
                                                   double *tin, uint32_t *ukey, float *uval, double *tks) {
  __shared__ double wv[4];
  __shared__ int wf[4];
  __shared__ int sw[16];
  __shared__ double cvv;
  __shared__ int cff;
  const int64_t t = blockIdx.x;
  const TileSpan ts = tile_span(g, t);
  const int64_t se = g.send[g.tseg[t]];
  if (PASS == 0 && threadIdx.x == 0) tin[t] = 0.0;
  if (threadIdx.x == 0) { cvv = 0.0; cff = 0; }
  __syncthreads();
  const int wid = (int)threadIdx.x / kWave;
  int heads = 0;  // heads in earlier rounds
  double kacc = 0.0;  // this thread's stored run weights (pass 1)
  const int64_t base_rank = PASS == 1 ? hc[t] - hc[ts.f0] : 0;
  for (int64_t b = ts.lo; b < ts.hi; b += blockDim.x) {
    const int64_t p = b + threadIdx.x;
    const bool act = p < ts.hi;
    uint32_t key = 0;
    double v = 0.0;
    bool head = false, rend = false;
    if (act) {
      key = gkey[p];
      v = (double)gval[p];
      head = p == ts.sb || gkey[p - 1] != key;
      rend = p + 1 == se || gkey[p + 1] != key;
    }
    // segmented inclusive scan: wavefront, then the earlier wavefronts and rounds
    double x = v;
    int f = head ? 1 : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const double yx = __shfl_up(x, o);
      const int yf = __shfl_up(f, o);
      if (lane() >= o) {
        if (!f) x += yx;
        f |= yf;
      }
    }
    if (lane() == kWave - 1) { wv[wid] = x; wf[wid] = f; }
    int ht;
    const int hx = blk_excl_int(head ? 1 : 0, &ht, sw);  // has a barrier after the stores above
    double ax = cvv;
    int af = cff;
    for (int k = 0; k < wid; ++k) {
      if (!wf[k]) ax += wv[k];
      else ax = wv[k];
      af |= wf[k];
    }
    if (!f) x += ax;
    f |= af;
    const int seen = heads + hx + (head ? 1 : 0);  // heads up to and including p in this tile
    if (act && (rend || p == ts.hi - 1)) {
      if (seen == 0) {
        if (PASS == 0) tin[t] = x;  // the leading piece ends here
      } else if (PASS == 1) {
        double sum = x;
        if (!rend) {
          // the run goes on past this tile: add the leading pieces it covers
          for (int64_t u = t + 1; u < ts.f0 + ts.nt; ++u) {
            sum += tin[u];
            if (hc[u + 1] - hc[u] > 0) break;
          }
        }
        const int64_t r = base_rank + seen - 1;
        const float wf = (float)sum;
        ukey[ts.sb + r] = key;
        uval[ts.sb + r] = wf;
        kacc += (double)wf;
      }
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) { cvv = x; cff = f; }
    heads += ht;
    __syncthreads();
  }
  if (PASS == 0 && threadIdx.x == 0) hc[t] = heads;
  if (PASS == 1 && tks) {
    // the tile's part of K', summed in a fixed order
    kacc = group_sum<kWave>(kacc);
    if (lane() == 0) wv[wid] = kacc;
    __syncthreads();
    if (threadIdx.x == 0) tks[t] = ((wv[0] + wv[1]) + wv[2]) + wv[3];
  }
}
void agg_large_runs(int pass, const uint32_t *gkey, const float *gval, const RsSeg &g, int64_t *hc, double *tin,
                    uint32_t *ukey, float *uval, double *tks, hipStream_t s) {
  if (g.ntiles <= 0) return;
  if (pass == 0)
    hipLaunchKernelGGL(k_agg_lruns<0>, (int)g.ntiles, 256, 0, s, gkey, gval, g, hc, tin, ukey, uval, tks);
  else
    hipLaunchKernelGGL(k_agg_lruns<1>, (int)g.ntiles, 256, 0, s, gkey, gval, g, hc, tin, ukey, uval, tks);
}

// rowlen and K' of the large segments (K' from the tiles' parts): a
// wavefront per segment
__global__ void k_agg_lrows(int64_t nl, const int32_t *lc, const int64_t *tfirst, const int64_t *hc,
                            const double *tks, int32_t *rowlen, double *K) {
  const int64_t l = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (l >= nl) return;
  const int c = lc[l];
  const int64_t U = hc[tfirst[l + 1]] - hc[tfirst[l]];
  if (lane() == 0) rowlen[c] = (int32_t)U;
  if (!K) return;
  double x = 0.0;
  for (int64_t t = tfirst[l] + lane(); t < tfirst[l + 1]; t += kWave) x += tks[t];
  x = group_sum<kWave>(x);
  if (lane() == 0) K[c] = x;
}
void agg_large_rows(int64_t nl, const int32_t *lc, const int64_t *tfirst, const int64_t *hc, const double *tks,
                    int32_t *rowlen, double *K, hipStream_t s) {
  if (nl > 0)
    hipLaunchKernelGGL(k_agg_lrows, (int)ceil_div(nl * kWave, 256), 256, 0, s, nl, lc, tfirst, hc, tks, rowlen, K);
}

// ---- 6: rows into place ------------------------------------------------------------
__global__ __launch_bounds__(256) void k_agg_csmall(const int64_t *seg, const int32_t *tfc, const int32_t *rowlen,
                                                    const int64_t *out_off, const uint32_t *ukey, const float *uval,
                                                    int32_t *out_idx, float *out_w) {
  const int64_t t = blockIdx.x;
  const int c0 = tfc[t], c1 = tfc[t + 1];
  for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
    const int64_t len = seg[c + 1] - seg[c];
    if (len <= 0 || len > kAggSmall) continue;
    const int64_t s0 = seg[c], d0 = out_off[c];
    const int r = rowlen[c];
    for (int j = 0; j < r; ++j) {
      out_idx[d0 + j] = (int32_t)ukey[s0 + j];
      out_w[d0 + j] = uval[s0 + j];
    }
  }
}
__global__ __launch_bounds__(256) void k_agg_clarge(const int32_t *lc, const int64_t *lsb, const int32_t *rowlen,
                                                    const int64_t *out_off, const uint32_t *ukey, const float *uval,
                                                    int32_t *out_idx, float *out_w) {
  const int64_t l = blockIdx.x;
  const int c = lc[l];
  const int64_t s0 = lsb[l], d0 = out_off[c];
  const int r = rowlen[c];
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    out_idx[d0 + j] = (int32_t)ukey[s0 + j];
    out_w[d0 + j] = uval[s0 + j];
  }
}
void agg_compact(const int64_t *seg, const int32_t *tfc, int64_t nst, const int32_t *lc, const int64_t *lsb,
                 int64_t nl, const int32_t *rowlen, const int64_t *out_off, const uint32_t *ukey, const float *uval,
                 int32_t *out_idx, float *out_w, hipStream_t s) {
  if (nst > 0)
    hipLaunchKernelGGL(k_agg_csmall, (int)nst, 256, 0, s, seg, tfc, rowlen, out_off, ukey, uval, out_idx, out_w);
  if (nl > 0)
    hipLaunchKernelGGL(k_agg_clarge, (int)nl, 256, 0, s, lc, lsb, rowlen, out_off, ukey, uval, out_idx, out_w);
}

}  // namespace lk
