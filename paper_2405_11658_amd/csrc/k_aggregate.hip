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
//   4. segments of at most kAggSmall entries: a wavefront per segment sorts
//      it by neighbour with a bitonic network (in registers up to 64 entries,
//      else in the wavefront's LDS area) and sums the runs of equal keys;
//   5. larger segments: a segmented radix sort by neighbour (tiles of 4096
//      entries that never cross a segment, digits of up to 9 bits), then the
//      runs are summed with a segmented scan per tile plus the continuation
//      pieces of the following tiles, all in a fixed order;
//   6. a scan of the row lengths gives the offsets, and the rows are copied
//      into place.
// Weights are summed in FP64 and stored rounded to float32; the next level's
// K' is the FP64 sum of the stored row weights.  Every sum is taken in an
// order fixed by the input, so results do not depend on scheduling.
#include "device.hpp"
#include "kernels.hpp"

namespace lk {

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
  // the thread's entries in three rounds of loads, each round's loads issued
  // together: ids, weights and row data; then communities and places; then
  // the stores
  constexpr int PER = kChunk / 256;
  int j[PER], pu[PER];
  float x[PER];
  int64_t ru[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * 256;
    j[k] = 0;
    pu[k] = 0;
    x[k] = 0.0f;
    ru[k] = 0;
    if (t < len) {
      const int u = rowof[t];
      j[k] = a.idx[q0 + t];
      x[k] = a.w[q0 + t];
      pu[k] = pos[u];
      ru[k] = a.off[u];
    }
  }
  int c[PER];
  int64_t d[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * 256;
    c[k] = 0;
    d[k] = 0;
    if (t < len) {
      c[k] = a.C[j[k]];
      d[k] = eoff[pu[k]] + (q0 + t - ru[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (threadIdx.x + k * 256 < len) {
      gkey[d[k]] = (uint32_t)c[k];
      gval[d[k]] = x[k];
    }
  }
}
void agg_group(const AggArgs &a, const int32_t *crow, const int32_t *pos, const int64_t *eoff, uint32_t *gkey,
               float *gval, hipStream_t s) {
  if (a.nnz > 0)
    hipLaunchKernelGGL(k_agg_group, (int)ceil_div(a.nnz, kChunk), 256, 0, s, a, crow, pos, eoff, gkey, gval);
}

// ---- 4: small segments -------------------------------------------------------
// A wavefront per segment of at most kAggSmall entries (the wavefronts take
// 64 communities at a time, spread over the whole id range, since costly
// segments cluster in id order): up to 64 entries are sorted in registers with a
// bitonic network over the lanes, up to 256 with the same network over R = 2
// or 4 registers per lane, larger ones (up to 1024) in the wavefront's LDS
// area (more registers per lane would spill).
// The network is data-oblivious and exchanges only strictly ordered pairs,
// so equal keys end in an order fixed by the input.  Runs of equal keys are
// summed with a segmented scan (fixed tree), each run written at its rank in
// the row; K' is the sum of the stored row weights (fixed tree).
constexpr uint32_t kKeyPad = 0xffffffffu;  // above every community id

// Orders a wavefront's own LDS accesses (one wavefront's LDS operations
// execute in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
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

__device__ __forceinline__ void seg_scan(double &x, int &f) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double yx = __shfl_up(x, o);
    const int yf = __shfl_up(f, o);
    if (lane() >= o) {
      if (!f) x += yx;
      f |= yf;
    }
  }
}

__device__ __forceinline__ void small_regs(const uint32_t *gkey, const float *gval, int64_t sb, int sl, int c,
                                           uint32_t *ukey, float *uval, double *u64, int32_t *rowlen, double *K) {
  uint32_t key = kKeyPad;
  float v = 0.0f;
  if (lane() < sl) {
    key = gkey[sb + lane()];
    v = gval[sb + lane()];
  }
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t ok = __shfl_xor(key, j);
      const float ov = __shfl_xor(v, j);
      const bool up = (lane() & k) == 0;
      const bool low = (lane() & j) == 0;
      // ascending pairs: the lower lane keeps the smaller key
      const bool take = (low == up) ? ok < key : ok > key;
      if (take) {
        key = ok;
        v = ov;
      }
    }
  }
  const bool act = lane() < sl;
  const uint32_t pk = __shfl_up(key, 1), nk = __shfl_down(key, 1);
  const bool head = act && (lane() == 0 || pk != key);
  const bool rend = act && (lane() == sl - 1 || nk != key);
  double x = act ? (double)v : 0.0;
  int f = head ? 1 : 0;
  seg_scan(x, f);
  const unsigned long long hm = __ballot(head);
  const int rank = __popcll(hm & ((2ull << lane()) - 1ull)) - 1;
  double kx = 0.0;
  if (rend) {
    const float wf = (float)x;
    ukey[sb + rank] = key;
    uval[sb + rank] = wf;
    if (u64) u64[sb + rank] = x;
    kx = (double)wf;
  }
  kx = group_sum<kWave>(kx);
  if (lane() == 0) {
    rowlen[c] = __popcll(hm);
    if (K) K[c] = kx;
  }
}

// One exchange step (block size K, distance J) of the bitonic network over
// the blocked layout of small_wide, then the following steps of the block.
template <int R, int K, int J>
__device__ __forceinline__ void bitonic_step(uint32_t (&key)[R], float (&v)[R]) {
  if constexpr (J >= R) {
    constexpr int LJ = J / R;
    const bool low = (lane() & LJ) == 0;
    const bool up = ((lane() * R) & K) == 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t ok = __shfl_xor(key[r], LJ);
      const float ov = __shfl_xor(v[r], LJ);
      const bool take = (low == up) ? ok < key[r] : ok > key[r];
      if (take) {
        key[r] = ok;
        v[r] = ov;
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r & J) continue;
      const int q = r | J;
      const bool up = K < R ? (r & K) == 0 : ((lane() * R) & K) == 0;
      if (up ? key[r] > key[q] : key[r] < key[q]) {
        const uint32_t tk = key[r];
        key[r] = key[q];
        key[q] = tk;
        const float tv = v[r];
        v[r] = v[q];
        v[q] = tv;
      }
    }
  }
  if constexpr (J > 1) bitonic_step<R, K, J / 2>(key, v);
}
// Blocks of size K, 2K, ... up to the whole 64 * R positions.
template <int R, int K>
__device__ __forceinline__ void bitonic_regs(uint32_t (&key)[R], float (&v)[R]) {
  bitonic_step<R, K, K / 2>(key, v);
  if constexpr (K < kWave * R) bitonic_regs<R, 2 * K>(key, v);
}

// Segments of 65 .. 64 * R entries in registers: lane L holds the R
// consecutive positions L * R .. L * R + R - 1 (keys padded with kKeyPad).
// The bitonic network's exchanges at distance j < R stay inside a lane (the
// register indices are compile-time constants once the loops are unrolled);
// at distance j >= R the partner is lane L ^ (j / R), same register.  As
// above, only strictly ordered pairs are exchanged.  The runs are then
// summed in position order: each lane in order over its registers, the run
// open at a lane's start taken from the lanes before it by a segmented scan
// over the lanes (fixed tree).
template <int R>
__device__ __forceinline__ void small_wide(const uint32_t *gkey, const float *gval, int64_t sb, int sl, int c,
                                           uint32_t *ukey, float *uval, double *u64, int32_t *rowlen, double *K) {
  uint32_t key[R];
  float v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = lane() * R + r;
    key[r] = kKeyPad;
    v[r] = 0.0f;
    if (e < sl) {
      key[r] = gkey[sb + e];
      v[r] = gval[sb + e];
    }
  }
  bitonic_regs<R, 2>(key, v);
  // heads and run ends; position e = lane * R + r is valid below sl
  const uint32_t prevk = __shfl_up(key[R - 1], 1);
  const uint32_t nextk = __shfl_down(key[0], 1);
  bool head[R], rend[R];
  int nh = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = lane() * R + r;
    const bool act = e < sl;
    const uint32_t pk = r == 0 ? prevk : key[r - 1];
    const uint32_t nk = r == R - 1 ? nextk : key[r + 1];
    head[r] = act && (e == 0 || pk != key[r]);
    rend[r] = act && (e == sl - 1 || nk != key[r]);
    nh += head[r] ? 1 : 0;
  }
  // the lane's open run: sum after its last head (all of it without a head)
  double tail = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double x = lane() * R + r < sl ? (double)v[r] : 0.0;
    tail = head[r] ? x : tail + x;
  }
  double t = tail;
  int f = nh > 0 ? 1 : 0;
  seg_scan(t, f);  // t: run open at the end of this lane
  double carry = __shfl_up(t, 1);
  if (lane() == 0) carry = 0.0;
  // ranks: heads before this lane, then in register order
  int hb = nh;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(hb, o);
    if (lane() >= o) hb += y;
  }
  const int total = __shfl(hb, kWave - 1);
  hb -= nh;
  double acc = carry, kx = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double x = lane() * R + r < sl ? (double)v[r] : 0.0;
    acc = head[r] ? x : acc + x;
    hb += head[r] ? 1 : 0;
    if (rend[r]) {
      const float wf = (float)acc;
      ukey[sb + hb - 1] = key[r];
      uval[sb + hb - 1] = wf;
      if (u64) u64[sb + hb - 1] = acc;
      kx += (double)wf;
    }
  }
  kx = group_sum<kWave>(kx);
  if (lane() == 0) {
    rowlen[c] = total;
    if (K) K[c] = kx;
  }
}

__device__ __forceinline__ void small_lds(const uint32_t *gkey, const float *gval, int64_t sb, int sl, int c,
                                          uint32_t *sk, float *sv, uint32_t *ukey, float *uval, double *u64,
                                          int32_t *rowlen, double *K) {
  int P = 2 * kWave;
  while (P < sl) P <<= 1;
  wave_lds_fence();  // the previous segment's reads of this area are done
  for (int p = lane(); p < P; p += kWave) {
    sk[p] = p < sl ? gkey[sb + p] : kKeyPad;
    sv[p] = p < sl ? gval[sb + p] : 0.0f;
  }
  wave_lds_fence();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      // pair p: lower position i (bit j clear), upper i + j; every lane
      // takes a pair in every round
      for (int p = lane(); p < P / 2; p += kWave) {
        const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
        const int ix = i + j;
        const uint32_t a = sk[i], b = sk[ix];
        const bool up = (i & k) == 0;
        if (up ? a > b : a < b) {
          sk[i] = b;
          sk[ix] = a;
          const float t = sv[i];
          sv[i] = sv[ix];
          sv[ix] = t;
        }
      }
      wave_lds_fence();
    }
  }
  double carry = 0.0, kx = 0.0;
  int heads = 0;
  for (int base = 0; base < sl; base += kWave) {
    const int p = base + lane();
    const bool act = p < sl;
    const uint32_t key = act ? sk[p] : kKeyPad;
    const bool head = act && (p == 0 || sk[p - 1] != key);
    const bool rend = act && (p == sl - 1 || sk[p + 1] != key);
    double x = act ? (double)sv[p] : 0.0;
    int f = head ? 1 : 0;
    seg_scan(x, f);
    if (!f) x += carry;  // the run open at the end of the previous chunk
    const unsigned long long hm = __ballot(head);
    const int rank = heads + __popcll(hm & ((2ull << lane()) - 1ull)) - 1;
    if (rend) {
      const float wf = (float)x;
      ukey[sb + rank] = key;
      uval[sb + rank] = wf;
      if (u64) u64[sb + rank] = x;
      kx += (double)wf;
    }
    carry = __shfl(x, kWave - 1);
    heads += __popcll(hm);
  }
  kx = group_sum<kWave>(kx);
  if (lane() == 0) {
    rowlen[c] = heads;
    if (K) K[c] = kx;
  }
}

__global__ __launch_bounds__(256) void k_agg_small(const int64_t *seg, int64_t ncomm, const uint32_t *gkey,
                                                   const float *gval, uint32_t *ukey, float *uval, double *u64,
                                                   int32_t *rowlen, double *K) {
  constexpr int W = 256 / kWave;
  __shared__ uint32_t sk[W][kAggSmall];
  __shared__ float sv[W][kAggSmall];
  const int wid = (int)threadIdx.x / kWave;
  // round r, wavefront w, lane q: community r * 64 * nw + q * nw + w
  const int64_t nw = (int64_t)gridDim.x * W;
  const int64_t w = (int64_t)blockIdx.x * W + wid;
  for (int64_t base = 0; base < ncomm; base += nw * kWave) {
    const int64_t c = base + (int64_t)lane() * nw + w;
    int64_t b = 0, len = 0;
    if (c < ncomm) {
      b = seg[c];
      len = seg[c + 1] - b;
    }
    unsigned long long todo = __ballot(len > 0 && len <= kAggSmall);
    while (todo) {
      const int k = __ffsll(todo) - 1;
      todo &= todo - 1ull;
      const int64_t sb = __shfl(b, k);
      const int sl = (int)__shfl(len, k);
      const int ck = (int)__shfl(c, k);
      if (sl <= kWave) small_regs(gkey, gval, sb, sl, ck, ukey, uval, u64, rowlen, K);
      else if (sl <= 2 * kWave) small_wide<2>(gkey, gval, sb, sl, ck, ukey, uval, u64, rowlen, K);
      else if (sl <= 4 * kWave) small_wide<4>(gkey, gval, sb, sl, ck, ukey, uval, u64, rowlen, K);
      else small_lds(gkey, gval, sb, sl, ck, sk[wid], sv[wid], ukey, uval, u64, rowlen, K);
    }
  }
}
void agg_small(const int64_t *seg, int64_t ncomm, const uint32_t *gkey, const float *gval, uint32_t *ukey,
               float *uval, double *u64, int32_t *rowlen, double *K, hipStream_t s) {
  if (ncomm > 0)
    hipLaunchKernelGGL(k_agg_small, flat_grid(ceil_div(ncomm, kWave), 4, 8192), 256, 0, s, seg, ncomm, gkey, gval,
                       ukey, uval, u64, rowlen, K);
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
// tseg[t] = the large segment of tile t: one thread per tile, a binary search
// in the segments' first tiles (strictly increasing; a thread per segment
// left the giant segment's hundreds of thousands of tiles to one thread).
__global__ void k_agg_tseg(const int64_t *tfirst, int64_t nl, int64_t ntl, int32_t *tseg) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntl; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nl;  // tfirst[lo] <= t < tfirst[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (tfirst[mid] <= t) lo = mid;
      else hi = mid;
    }
    tseg[t] = (int32_t)lo;
  }
}
void agg_large_list(const int64_t *seg, int64_t ncomm, int32_t *flag, const int32_t *lidx, int32_t *lc, int64_t *lsb,
                    int64_t *lse, int64_t *ltn, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_llist, flat_grid(ncomm + 1), 256, 0, s, seg, ncomm, (const int32_t *)flag, lidx, lc, lsb,
                     lse, ltn);
}
void agg_large_flags(const int64_t *seg, int64_t ncomm, int32_t *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_agg_lflag, flat_grid(ncomm + 1), 256, 0, s, seg, ncomm, flag);
}
void agg_tile_seg(const int64_t *tfirst, int64_t nl, int64_t ntl, int32_t *tseg, hipStream_t s) {
  if (nl > 0 && ntl > 0) hipLaunchKernelGGL(k_agg_tseg, flat_grid(ntl), 256, 0, s, tfirst, nl, ntl, tseg);
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
                                                   double *tin, uint32_t *ukey, float *uval, double *l64,
                                                   double *tks) {
  // The tile is loaded with coalesced loads into LDS (one pad word per kPR
  // items, so that each thread then reads its kPR consecutive items without
  // bank conflicts) and scanned in one round: each thread sums its items in
  // order, the threads' open runs are joined by a segmented scan over the
  // block (fixed tree), and heads are counted the same way.
  constexpr int E = kPR;
  constexpr int W = 256 / kWave;
  __shared__ uint32_t sk[kPTile + kPTile / E];
  __shared__ float sv[kPTile + kPTile / E];
  __shared__ double wx[W];
  __shared__ int wfl[W], wh[W];
  __shared__ uint32_t edge[2];
  const int64_t t = blockIdx.x;
  const TileSpan ts = tile_span(g, t);
  const int64_t se = g.send[g.tseg[t]];
  const int n = (int)(ts.hi - ts.lo);
  const int tid = (int)threadIdx.x, wid = tid / kWave;
  if (PASS == 0 && tid == 0) tin[t] = 0.0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = r * 256 + tid;
    if (e < n) {
      sk[e + e / E] = gkey[ts.lo + e];
      sv[e + e / E] = gval[ts.lo + e];
    }
  }
  if (tid == 0) {
    edge[0] = ts.lo > ts.sb ? gkey[ts.lo - 1] : 0u;  // compared only inside a segment
    edge[1] = ts.hi < se ? gkey[ts.hi] : 0u;
  }
  __syncthreads();
  const int e0 = tid * E;
  uint32_t key[E];
  double v[E];
  bool head[E], rend[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = e0 + r;
    key[r] = e < n ? sk[e + tid] : 0u;
    v[r] = e < n ? (double)sv[e + tid] : 0.0;
  }
  const uint32_t before = e0 == 0 ? edge[0] : sk[(e0 - 1) + (e0 - 1) / E];
  const uint32_t after = e0 + E < n ? sk[(e0 + E) + (e0 + E) / E] : edge[1];
  int nh = 0;
  double tail = 0.0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = e0 + r;
    const bool act = e < n;
    const int64_t p = ts.lo + e;
    const uint32_t pk = r == 0 ? before : key[r - 1];
    const uint32_t nk = r == E - 1 ? after : key[r + 1];
    head[r] = act && (p == ts.sb || pk != key[r]);
    rend[r] = act && (p + 1 == se || nk != key[r]);
    nh += head[r] ? 1 : 0;
    tail = head[r] ? v[r] : tail + v[r];
  }
  // open run at the end of each thread (inclusive), then exclusive carries
  double x = tail;
  int f = nh > 0 ? 1 : 0;
  seg_scan(x, f);
  int hi = nh;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(hi, o);
    if (lane() >= o) hi += y;
  }
  if (lane() == kWave - 1) {
    wx[wid] = x;
    wfl[wid] = f;
    wh[wid] = hi;
  }
  __syncthreads();
  double ax = 0.0;
  int hw = 0, ht = 0;
  for (int k = 0; k < W; ++k) {
    if (k < wid) {
      ax = wfl[k] ? wx[k] : ax + wx[k];
      hw += wh[k];
    }
    ht += wh[k];
  }
  double carry = __shfl_up(x, 1);
  const int fprev = __shfl_up(f, 1);
  if (lane() == 0) carry = ax;
  else if (!fprev) carry += ax;
  if (tid == 0) carry = 0.0;
  int seen = hw + hi - nh;  // heads before this thread's items
  double acc = carry, kacc = 0.0;
  const int64_t base_rank = PASS == 1 ? hc[t] - hc[ts.f0] : 0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = e0 + r;
    acc = head[r] ? v[r] : acc + v[r];
    seen += head[r] ? 1 : 0;
    if (e < n && (rend[r] || e == n - 1)) {
      if (seen == 0) {
        if (PASS == 0) tin[t] = acc;  // the leading piece ends here
      } else if (PASS == 1) {
        double sum = acc;
        if (!rend[r]) {
          // the run goes on past this tile: add the leading pieces it covers
          for (int64_t u = t + 1; u < ts.f0 + ts.nt; ++u) {
            sum += tin[u];
            if (hc[u + 1] - hc[u] > 0) break;
          }
        }
        const int64_t rk = base_rank + seen - 1;
        const float wf = (float)sum;
        ukey[ts.sb + rk] = key[r];
        uval[ts.sb + rk] = wf;
        if (l64) l64[ts.sb + rk] = sum;
        kacc += (double)wf;
      }
    }
  }
  if (PASS == 0 && tid == 0) hc[t] = ht;
  if (PASS == 1 && tks) {
    // the tile's part of K', summed in a fixed order
    kacc = group_sum<kWave>(kacc);
    __syncthreads();  // wx is reused
    if (lane() == 0) wx[wid] = kacc;
    __syncthreads();
    if (tid == 0) tks[t] = ((wx[0] + wx[1]) + wx[2]) + wx[3];
  }
}
void agg_large_runs(int pass, const uint32_t *gkey, const float *gval, const RsSeg &g, int64_t *hc, double *tin,
                    uint32_t *ukey, float *uval, double *l64, double *tks, hipStream_t s) {
  if (g.ntiles <= 0) return;
  if (pass == 0)
    hipLaunchKernelGGL(k_agg_lruns<0>, (int)g.ntiles, 256, 0, s, gkey, gval, g, hc, tin, ukey, uval, l64, tks);
  else
    hipLaunchKernelGGL(k_agg_lruns<1>, (int)g.ntiles, 256, 0, s, gkey, gval, g, hc, tin, ukey, uval, l64, tks);
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
__global__ __launch_bounds__(256) void k_agg_csmall(const int64_t *seg, int64_t ncomm, const int32_t *rowlen,
                                                    const int64_t *out_off, const uint32_t *ukey, const float *uval,
                                                    const double *v64, int32_t *out_idx, float *out_w,
                                                    double *out_w64) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave * kWave; c0 < ncomm; c0 += stride) {
    const int64_t c = c0 + lane();
    int64_t s0 = 0, d0 = 0, len = 0;
    int r = 0;
    if (c < ncomm) {
      s0 = seg[c];
      len = seg[c + 1] - s0;
      r = rowlen[c];
      d0 = out_off[c];
    }
    unsigned long long todo = __ballot(len > 0 && len <= kAggSmall && r > 0);
    while (todo) {
      const int k = __ffsll(todo) - 1;
      todo &= todo - 1ull;
      const int64_t src = __shfl(s0, k), dst = __shfl(d0, k);
      const int rk = __shfl(r, k);
      for (int j = lane(); j < rk; j += kWave) {
        out_idx[dst + j] = (int32_t)ukey[src + j];
        out_w[dst + j] = uval[src + j];
        if (out_w64) out_w64[dst + j] = v64[src + j];
      }
    }
  }
}
// One workgroup per input tile of the large segments: tile k of segment l
// copies row entries [k * kPTile, (k + 1) * kPTile) of the segment's row (a
// row is never longer than its segment, so the tiles cover it and no
// workgroup copies more than one tile's worth, however large the segment).
__global__ __launch_bounds__(256) void k_agg_clarge(const int32_t *lc, const int64_t *lsb, const int32_t *tseg,
                                                    const int64_t *tfirst, const int32_t *rowlen,
                                                    const int64_t *out_off, const uint32_t *ukey, const float *uval,
                                                    const double *v64, int32_t *out_idx, float *out_w,
                                                    double *out_w64) {
  const int64_t t = blockIdx.x;
  const int l = tseg[t];
  const int c = lc[l];
  const int64_t s0 = lsb[l], d0 = out_off[c];
  const int64_t j0 = (t - tfirst[l]) * kPTile;
  const int64_t j1 = min(j0 + kPTile, (int64_t)rowlen[c]);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    out_idx[d0 + j] = (int32_t)ukey[s0 + j];
    out_w[d0 + j] = uval[s0 + j];
    if (out_w64) out_w64[d0 + j] = v64[s0 + j];
  }
}
void agg_compact(const int64_t *seg, int64_t ncomm, const int32_t *lc, const int64_t *lsb, const int32_t *tseg,
                 const int64_t *tfirst, int64_t ntl, const int32_t *rowlen, const int64_t *out_off,
                 const uint32_t *ukey, const float *uval, const uint32_t *lkey, const float *lval,
                 const double *v64, int32_t *out_idx, float *out_w, double *out_w64, hipStream_t s) {
  if (ncomm > 0)
    hipLaunchKernelGGL(k_agg_csmall, flat_grid(ncomm, 256, 8192), 256, 0, s, seg, ncomm, rowlen, out_off, ukey, uval,
                       v64, out_idx, out_w, out_w64);
  if (ntl > 0)
    hipLaunchKernelGGL(k_agg_clarge, (int)ntl, 256, 0, s, lc, lsb, tseg, tfirst, rowlen, out_off, lkey, lval,
                       v64, out_idx, out_w, out_w64);
}

}  // namespace lk
