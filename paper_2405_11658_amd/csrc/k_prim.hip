// Device-wide primitives of the library: exclusive prefix scans and a stable
// least-significant-digit radix sort of (key, value) pairs over independent
// segments.  Both work in tiles of 4096 items (256 threads x 16 rounds); no
// vendor primitive library is used.
//
// Scan: tile totals (one workgroup per tile), a scan of the totals (the same
// routine, recursively), then each tile scans its items in 16 rounds of 256
// with the tile's prefix as carry.  In-place use (in == out) is allowed.
//
// Radix sort: per pass (digits of at most 9 bits) a digit histogram per tile,
// an exclusive scan of the histograms laid out segment-major, digit-major,
// tile-minor (so the scanned value of (segment, digit, tile) is where the
// tile's items of that digit go), and a stable scatter that ranks the items of
// each 256-item round with wavefront ballots (lanes with the same digit) plus
// per-wavefront counts into a digit-sorted copy of the tile in LDS, written
// out in order (coalesced runs per digit).  Tiles never cross a segment.
#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace lk {

// exclusive prefix over the workgroup of one value per thread, in thread
// order; *tot receives the workgroup total.  All threads must call it.
template <class T>
__device__ __forceinline__ T blk_excl(T x, T *tot, T *sw /* >= kPT / kWave */) {
  T incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const T y = __shfl_up(incl, o);
    if (lane() >= o) incl += y;
  }
  const int w = (int)threadIdx.x / kWave;
  if (lane() == kWave - 1) sw[w] = incl;
  __syncthreads();
  T pre = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kPT / kWave; ++k) {
    if (k < w) pre += sw[k];
    all += sw[k];
  }
  __syncthreads();
  *tot = all;
  return pre + incl - x;
}

// ---- scan ----------------------------------------------------------------------
template <class I, class O>
__global__ __launch_bounds__(kPT) void k_scan_reduce(const I *in, int64_t n, O *tsum) {
  __shared__ O sw[kPT / kWave];
  const int64_t b = (int64_t)blockIdx.x * kPTile;
  O s = 0;
  for (int k = threadIdx.x; k < kPTile; k += kPT) {
    const int64_t p = b + k;
    if (p < n) s += (O)in[p];
  }
  O tot;
  (void)blk_excl<O>(s, &tot, sw);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

template <class I, class O>
__global__ __launch_bounds__(kPT) void k_scan_apply(const I *in, O *out, int64_t n, const O *tpre) {
  __shared__ O sw[kPT / kWave];
  const int64_t b = (int64_t)blockIdx.x * kPTile;
  O carry = tpre ? tpre[blockIdx.x] : (O)0;
  for (int r = 0; r < kPR; ++r) {
    const int64_t p = b + (int64_t)r * kPT + threadIdx.x;
    if (b + (int64_t)r * kPT >= n) break;  // uniform
    const O x = p < n ? (O)in[p] : (O)0;
    O tot;
    const O ex = blk_excl<O>(x, &tot, sw);
    if (p < n) out[p] = carry + ex;
    carry += tot;
  }
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t t = 0;
  while (n > kPTile) {
    n = ceil_div(n, kPTile);
    t += n;
  }
  return t;
}

template <class I, class O>
void scan_rec(const I *in, O *out, int64_t n, O *tmp, hipStream_t s) {
  if (n <= 0) return;
  if (n <= kPTile) {
    hipLaunchKernelGGL((k_scan_apply<I, O>), 1, kPT, 0, s, in, out, n, (const O *)nullptr);
    return;
  }
  const int64_t nt = ceil_div(n, kPTile);
  hipLaunchKernelGGL((k_scan_reduce<I, O>), (int)nt, kPT, 0, s, in, n, tmp);
  scan_rec<O, O>(tmp, tmp, nt, tmp + nt, s);
  hipLaunchKernelGGL((k_scan_apply<I, O>), (int)nt, kPT, 0, s, in, out, n, (const O *)tmp);
}

static size_t scan_bytes(int64_t n, size_t osize) {
  return std::max<size_t>(256, (size_t)scan_tmp_elems(n) * osize);
}
size_t scan_excl_i32(void *temp, size_t tbytes, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  const size_t need = scan_bytes(n, sizeof(int32_t));
  if (temp && tbytes >= need) scan_rec<int32_t, int32_t>(in, out, n, (int32_t *)temp, s);
  return need;
}
size_t scan_excl_i64(void *temp, size_t tbytes, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  const size_t need = scan_bytes(n, sizeof(int64_t));
  if (temp && tbytes >= need) scan_rec<int64_t, int64_t>(in, out, n, (int64_t *)temp, s);
  return need;
}
size_t scan_excl_i32_to_i64(void *temp, size_t tbytes, const int32_t *in, int64_t *out, int64_t n,
                            hipStream_t s) {
  const size_t need = scan_bytes(n, sizeof(int64_t));
  if (temp && tbytes >= need) scan_rec<int32_t, int64_t>(in, out, n, (int64_t *)temp, s);
  return need;
}

// ---- radix sort ------------------------------------------------------------------
constexpr int kRadixBits = 9;            // digits of at most 9 bits
constexpr int kDig = 1 << kRadixBits;    // 512 digit values
constexpr int kDPT = kDig / kPT;         // digits per thread

// hist: scan layout (segment, digit, tile) over the pass's 2^bits digits.
template <class K>
__global__ __launch_bounds__(kPT) void k_rs_hist(const K *keys, RsSeg g, int shift, int bits, int64_t *hist) {
  __shared__ int h[kDig];
  const int64_t t = blockIdx.x;
  const TileSpan ts = tile_span(g, t);
  for (int d = threadIdx.x; d < kDig; d += kPT) h[d] = 0;
  __syncthreads();
  const K mask = (K)((1u << bits) - 1u);
  // all of the thread's loads issued together, then the counts
  K kr[kPR];
#pragma unroll
  for (int r = 0; r < kPR; ++r) {
    const int64_t p = ts.lo + r * kPT + threadIdx.x;
    kr[r] = p < ts.hi ? keys[p] : (K)0;
  }
#pragma unroll
  for (int r = 0; r < kPR; ++r)
    if (ts.lo + r * kPT + threadIdx.x < ts.hi) atomicAdd(&h[(int)((kr[r] >> shift) & mask)], 1);
  __syncthreads();
  const int nd = 1 << bits;
  for (int d = threadIdx.x; d < nd; d += kPT) hist[nd * ts.f0 + (int64_t)d * ts.nt + (t - ts.f0)] = h[d];
}

// Each tile ranks its items stably by digit into a local digit-sorted copy in
// LDS, then writes it out in order: the items of one digit go to consecutive
// places, so consecutive threads write consecutive addresses.  Each
// wavefront ranks its own contiguous quarter of the tile (16 rounds of 64
// items, in order) against digit counters that only it uses, so the rounds
// need no workgroup barrier; one prefix over the digits and the four
// wavefronts' counts then gives every item its place.  Items are ordered by
// (wavefront, round, lane), which is their order in the tile: stable.
template <class K, class V>
__global__ __launch_bounds__(kPT) void k_rs_scatter(const K *ki, const V *vi, K *ko, V *vo, RsSeg g, int shift,
                                                    int bits, const int64_t *hs) {
  constexpr int W = kPT / kWave;
  constexpr int QW = kPTile / W;  // items per wavefront
  __shared__ K sk[kPTile];
  __shared__ V sv[kPTile];
  __shared__ int64_t gbase[kDig];
  __shared__ int cnt[W][kDig];
  __shared__ int sw[W];
  const int64_t t = blockIdx.x;
  const TileSpan ts = tile_span(g, t);
  const int nd = 1 << bits;
  const int64_t seg0 = hs[nd * ts.f0];
  const int wid = (int)threadIdx.x / kWave;
  for (int d = threadIdx.x; d < kDig; d += kPT) {
#pragma unroll
    for (int w = 0; w < W; ++w) cnt[w][d] = 0;
  }
  // the wavefront's items in registers first (all loads in flight together)
  const int64_t q0 = ts.lo + (int64_t)wid * QW;
  K kr[kPR];
  V vr[kPR];
#pragma unroll
  for (int r = 0; r < kPR; ++r) {
    const int64_t p = q0 + r * kWave + lane();
    kr[r] = (K)0;
    vr[r] = V();
    if (p < ts.hi) {
      kr[r] = ki[p];
      vr[r] = vi[p];
    }
  }
  __syncthreads();  // counters cleared
  const K mask = (K)((1u << bits) - 1u);
  const unsigned long long below = lane() == 0 ? 0ull : (~0ull >> (64 - lane()));
  int rk[kPR];
#pragma unroll
  for (int r = 0; r < kPR; ++r) {
    const int64_t p = q0 + r * kWave + lane();
    const bool act = p < ts.hi;
    const int dg = act ? (int)((kr[r] >> shift) & mask) : 0;
    unsigned long long same = __ballot(act);
    for (int bit = 0; bit < bits; ++bit) {
      const unsigned long long on = __ballot(act && ((dg >> bit) & 1));
      same &= ((dg >> bit) & 1) ? on : ~on;
    }
    const int rank_w = __popcll(same & below);
    // every lane reads the count before the group's first lane adds to it
    // (one wavefront's LDS operations execute in order)
    const int old = act ? cnt[wid][dg] : 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (act && rank_w == 0) cnt[wid][dg] = old + __popcll(same);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    rk[r] = old + rank_w;
  }
  __syncthreads();
  {
    // digit d's items start at the total of the smaller digits; wavefront w's
    // after those of the wavefronts before it.  Each thread owns kDPT digits.
    int c[kDPT][W], sum = 0;
#pragma unroll
    for (int k = 0; k < kDPT; ++k) {
      const int d = threadIdx.x * kDPT + k;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        c[k][w] = cnt[w][d];
        sum += c[k][w];
      }
    }
    int tot;
    int pre = blk_excl<int>(sum, &tot, sw);  // barriers: every count read above
#pragma unroll
    for (int k = 0; k < kDPT; ++k) {
      const int d = threadIdx.x * kDPT + k;
      if (d < nd) gbase[d] = ts.sb + (hs[nd * ts.f0 + (int64_t)d * ts.nt + (t - ts.f0)] - seg0) - pre;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        cnt[w][d] = pre;
        pre += c[k][w];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPR; ++r) {
    const int64_t p = q0 + r * kWave + lane();
    if (p < ts.hi) {
      const int dg = (int)((kr[r] >> shift) & mask);
      const int q = cnt[wid][dg] + rk[r];
      sk[q] = kr[r];
      sv[q] = vr[r];
    }
  }
  __syncthreads();
  const int m = (int)(ts.hi - ts.lo);
  for (int j = threadIdx.x; j < m; j += kPT) {
    const K key = sk[j];
    const int dg = (int)((key >> shift) & mask);
    const int64_t q = gbase[dg] + j;
    ko[q] = key;
    vo[q] = sv[j];
  }
}

int rs_passes(int bits) { return bits <= 0 ? 0 : (bits + kRadixBits - 1) / kRadixBits; }

size_t rs_tmp_bytes(int64_t ntiles) {
  const int64_t nh = (int64_t)kDig * std::max<int64_t>(ntiles, 1);
  return (size_t)nh * sizeof(int64_t) + scan_bytes(nh, sizeof(int64_t));
}

template <class K, class V>
int rsort(K *k0, V *v0, K *k1, V *v1, const RsSeg &g, int bits, void *tmp, hipStream_t s) {
  const int np = rs_passes(bits);
  if (np == 0 || g.ntiles <= 0) return 0;
  const int wd = (bits + np - 1) / np;
  const int64_t nhmax = (int64_t)kDig * g.ntiles;
  int64_t *hist = (int64_t *)tmp;
  int64_t *stmp = hist + nhmax;
  K *ks = k0, *kd = k1;
  V *vs = v0, *vd = v1;
  int shift = 0;
  for (int p = 0; p < np; ++p) {
    const int b = std::min(wd, bits - shift);
    const int64_t nh = ((int64_t)1 << b) * g.ntiles;
    hipLaunchKernelGGL((k_rs_hist<K>), (int)g.ntiles, kPT, 0, s, (const K *)ks, g, shift, b, hist);
    scan_rec<int64_t, int64_t>(hist, hist, nh, stmp, s);
    hipLaunchKernelGGL((k_rs_scatter<K, V>), (int)g.ntiles, kPT, 0, s, (const K *)ks, (const V *)vs, kd, vd, g,
                       shift, b, (const int64_t *)hist);
    std::swap(ks, kd);
    std::swap(vs, vd);
    shift += b;
  }
  return np & 1;
}

template int rsort<uint32_t, int32_t>(uint32_t *, int32_t *, uint32_t *, int32_t *, const RsSeg &, int, void *,
                                      hipStream_t);
template int rsort<uint32_t, float>(uint32_t *, float *, uint32_t *, float *, const RsSeg &, int, void *,
                                    hipStream_t);

RsSeg rs_plain(int64_t n) {
  RsSeg g;
  g.ntiles = ceil_div(n, kPTile);
  g.n = n;
  g.tseg = nullptr;
  g.tfirst = nullptr;
  g.sbeg = nullptr;
  g.send = nullptr;
  return g;
}

int key_bits(unsigned long long x) {
  int b = 0;
  while (b < 64 && (x >> b) != 0ull) ++b;
  return b;
}

// Sorted copies (kout, vout) of (kin, vin) by the low `bits` key bits.  The
// temporary area holds the second key / value buffers, the histograms and the
// scan space.
template <class K, class V>
static size_t sort_copy(void *temp, size_t tbytes, const K *kin, K *kout, const V *vin, V *vout, int64_t n,
                        int bits, hipStream_t s) {
  const RsSeg g = rs_plain(n);
  const size_t kb = ((size_t)std::max<int64_t>(n, 1) * sizeof(K) + 255) & ~(size_t)255;
  const size_t vb = ((size_t)std::max<int64_t>(n, 1) * sizeof(V) + 255) & ~(size_t)255;
  const size_t need = kb + vb + rs_tmp_bytes(g.ntiles);
  if (!temp || tbytes < need || n <= 0) return need;
  char *t = (char *)temp;
  K *tk = (K *)t;
  V *tv = (V *)(t + kb);
  // an odd number of passes ends in the second buffers: start there
  const bool odd = rs_passes(bits) & 1;
  (void)hipMemcpyAsync(odd ? tk : kout, kin, sizeof(K) * n, hipMemcpyDeviceToDevice, s);
  (void)hipMemcpyAsync(odd ? tv : vout, vin, sizeof(V) * n, hipMemcpyDeviceToDevice, s);
  if (odd) rsort<K, V>(tk, tv, kout, vout, g, bits, t + kb + vb, s);
  else rsort<K, V>(kout, vout, tk, tv, g, bits, t + kb + vb, s);
  return need;
}
template int rsort<unsigned long long, int32_t>(unsigned long long *, int32_t *, unsigned long long *, int32_t *,
                                                 const RsSeg &, int, void *, hipStream_t);
template int rsort<unsigned long long, double>(unsigned long long *, double *, unsigned long long *, double *,
                                                const RsSeg &, int, void *, hipStream_t);
template int rsort<unsigned long long, float>(unsigned long long *, float *, unsigned long long *, float *,
                                               const RsSeg &, int, void *, hipStream_t);

size_t sort_pairs_u64_i32(void *temp, size_t tbytes, const unsigned long long *kin, unsigned long long *kout,
                          const int32_t *vin, int32_t *vout, int64_t n, hipStream_t s) {
  return sort_copy<unsigned long long, int32_t>(temp, tbytes, kin, kout, vin, vout, n, 64, s);
}
size_t sort_pairs_u64_f64(void *temp, size_t tbytes, const unsigned long long *kin, unsigned long long *kout,
                          const double *vin, double *vout, int64_t n, hipStream_t s) {
  return sort_copy<unsigned long long, double>(temp, tbytes, kin, kout, vin, vout, n, 64, s);
}

// Rows sorted by column id: (row << 32 | column) keys over the bits in use.
__global__ void k_row_keys(const int64_t *off, int64_t nrows, const int32_t *col, unsigned long long *keys) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x)
    for (int64_t e = off[r]; e < off[r + 1]; ++e)
      keys[e] = ((unsigned long long)r << 32) | (unsigned long long)(uint32_t)col[e];
}
__global__ void k_low_words(const unsigned long long *keys, int64_t n, int32_t *col) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    col[e] = (int32_t)(uint32_t)keys[e];
}
size_t seg_sort_i32_f32(void *temp, size_t tbytes, const int32_t *kin, int32_t *kout, const float *vin, float *vout,
                        int64_t nnz, int64_t nseg, const int64_t *off, hipStream_t s) {
  const RsSeg g = rs_plain(nnz);
  const size_t kb = ((size_t)std::max<int64_t>(nnz, 1) * 8 + 255) & ~(size_t)255;
  const size_t vb = ((size_t)std::max<int64_t>(nnz, 1) * 4 + 255) & ~(size_t)255;
  const size_t need = 2 * kb + vb + rs_tmp_bytes(g.ntiles);
  if (!temp || tbytes < need || nnz <= 0) return need;
  char *t = (char *)temp;
  unsigned long long *k0 = (unsigned long long *)t, *k1 = (unsigned long long *)(t + kb);
  float *v1 = (float *)(t + 2 * kb);
  hipLaunchKernelGGL(k_row_keys, flat_grid(nseg), 256, 0, s, off, nseg, kin, k0);
  const int bits = 32 + key_bits((unsigned long long)std::max<int64_t>(nseg - 1, 0));
  const bool odd = rs_passes(bits) & 1;  // values end in vout either way
  (void)hipMemcpyAsync(odd ? v1 : vout, vin, sizeof(float) * nnz, hipMemcpyDeviceToDevice, s);
  const int r = odd ? rsort<unsigned long long, float>(k0, v1, k1, vout, g, bits, t + 2 * kb + vb, s)
                    : rsort<unsigned long long, float>(k0, vout, k1, v1, g, bits, t + 2 * kb + vb, s);
  hipLaunchKernelGGL(k_low_words, flat_grid(nnz), 256, 0, s, r ? k1 : k0, nnz, kout);
  return need;
}

}  // namespace lk
