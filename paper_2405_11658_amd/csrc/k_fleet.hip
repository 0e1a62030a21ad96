// Fused many-graph engine (see fleet_kernels.hpp): one persistent launch in
// which each workgroup runs whole graph updates, one job after another.
#include "device.hpp"
#include "fleet_kernels.hpp"

#pragma clang fp contract(off)

namespace lk {
namespace {

// Loads of words that other threads of the workgroup update with atomics
// (performed in L2): read past the CU's L1.
template <class V>
__device__ __forceinline__ V ldx(const V *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr unsigned long long kNoKey = ~0ull;

// LDS of one workgroup.
template <int T, int SLOTS>
struct FSh {
  static constexpr int W = T / kWave;
  // reductions and broadcasts
  double rd[W];
  int ri[W];
  long long rl[W];
  int flag;
  int cnt;
  int list[T];          // candidate positions of a tile
  // radix sort
  int hist[256];
  int base[256];
  int wcnt[W][256];
  // neighbour-community table
  int tkeys[SLOTS];
  double tvals[SLOTS];
  int tlist[SLOTS];
  int tcnt;
  // job state broadcast
  FleetJob job;
  FleetGraph g;
};

template <int T, int SLOTS>
struct Blk {
  using Sh = FSh<T, SLOTS>;
  static constexpr int W = T / kWave;

  static __device__ int tid() { return (int)threadIdx.x; }
  static __device__ int wid() { return (int)threadIdx.x / kWave; }

  static __device__ double sum_d(double v, Sh &s) {
    v = group_sum<kWave>(v);
    __syncthreads();
    if (lane() == 0) s.rd[wid()] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < W; ++k) t += s.rd[k];
    __syncthreads();
    return t;
  }
  static __device__ long long sum_l(long long v, Sh &s) {
    v = group_sum_ll<kWave>(v);
    __syncthreads();
    if (lane() == 0) s.rl[wid()] = v;
    __syncthreads();
    long long t = 0;
    for (int k = 0; k < W; ++k) t += s.rl[k];
    __syncthreads();
    return t;
  }
  static __device__ int or_i(int v, Sh &s) {
    __syncthreads();
    if (tid() == 0) s.flag = 0;
    __syncthreads();
    if (v) atomicOr(&s.flag, v);
    __syncthreads();
    const int r = s.flag;
    __syncthreads();
    return r;
  }
  // best (larger gain, then smaller id) over the block; valid in all threads
  static __device__ void argmax(double &g, int &c, Sh &s) {
    group_argmax<kWave>(g, c);
    __syncthreads();
    if (lane() == 0) {
      s.rd[wid()] = g;
      s.ri[wid()] = c;
    }
    __syncthreads();
    g = s.rd[0];
    c = s.ri[0];
    for (int k = 1; k < W; ++k)
      if (better(s.rd[k], s.ri[k], g, c)) { g = s.rd[k]; c = s.ri[k]; }
    __syncthreads();
  }
  // exclusive prefix of x over the block (tile order); total in *tot
  static __device__ long long excl(long long x, long long *tot, Sh &s) {
    long long incl = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const long long y = __shfl_up(incl, off);
      if (lane() >= off) incl += y;
    }
    __syncthreads();
    if (lane() == kWave - 1) s.rl[wid()] = incl;
    __syncthreads();
    long long pre = 0, all = 0;
    for (int k = 0; k < W; ++k) {
      if (k < wid()) pre += s.rl[k];
      all += s.rl[k];
    }
    __syncthreads();
    *tot = all;
    return pre + incl - x;
  }
  // out[k] = sum of in[0..k) for k in [0, n]; returns the total.  in and out
  // may be the same array.
  template <class I, class O>
  static __device__ long long scan(const I *in, O *out, int64_t n, Sh &s) {
    long long carry = 0;
    for (int64_t b = 0; b < n + 1; b += T) {
      const int64_t k = b + tid();
      const long long x = (k < n) ? (long long)ldx(&in[k]) : 0;
      long long tot;
      const long long ex = excl(x, &tot, s);
      if (k <= n) out[k] = (O)(carry + ex);
      carry += tot;
      __syncthreads();
    }
    return carry;
  }

  // Stable LSD radix sort of (key, payload) pairs by the low `bits` key bits;
  // returns the buffer (0 / 1) holding the result.
  static __device__ int sort(unsigned long long *key[2], int32_t *pay[2], int64_t n, int bits, Sh &s) {
    int src = 0;
    for (int shift = 0; shift < bits; shift += 8) {
      const unsigned long long *ki = key[src];
      const int32_t *pi = pay[src];
      unsigned long long *ko = key[src ^ 1];
      int32_t *po = pay[src ^ 1];
      for (int d = tid(); d < 256; d += T) s.hist[d] = 0;
      __syncthreads();
      for (int64_t k = tid(); k < n; k += T) atomicAdd(&s.hist[(int)((ki[k] >> shift) & 255ull)], 1);
      __syncthreads();
      if (tid() == 0) {
        int acc = 0;
        for (int d = 0; d < 256; ++d) {
          s.base[d] = acc;
          acc += s.hist[d];
        }
      }
      for (int d = tid(); d < 256 * W; d += T) (&s.wcnt[0][0])[d] = 0;
      __syncthreads();
      for (int64_t b = 0; b < n; b += T) {
        const int64_t k = b + tid();
        const bool act = k < n;
        unsigned long long key = 0;
        int32_t p = 0;
        int dg = 0;
        if (act) {
          key = ki[k];
          p = pi[k];
          dg = (int)((key >> shift) & 255ull);
        }
        // lanes of this wavefront with the same digit
        unsigned long long same = __ballot(act);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
          const unsigned long long on = __ballot(act && ((dg >> bit) & 1));
          same &= ((dg >> bit) & 1) ? on : ~on;
        }
        const unsigned long long below = (lane() == 0) ? 0ull : (~0ull >> (64 - lane()));
        const int rank_w = __popcll(same & below);
        if (act && rank_w == 0) s.wcnt[wid()][dg] = __popcll(same);
        __syncthreads();
        if (act) {
          int before = 0;
          for (int w = 0; w < wid(); ++w) before += s.wcnt[w][dg];
          const int64_t pos = s.base[dg] + before + rank_w;
          ko[pos] = key;
          po[pos] = p;
        }
        __syncthreads();
        for (int d = tid(); d < 256; d += T) {
          int t = 0;
          for (int w = 0; w < W; ++w) {
            t += s.wcnt[w][d];
            s.wcnt[w][d] = 0;
          }
          s.base[d] += t;
        }
        __syncthreads();
      }
      src ^= 1;
    }
    return src;
  }
};

__device__ __forceinline__ int bits_for(unsigned long long top) {
  int b = 1;
  while (b < 64 && (top >> b) != 0) ++b;
  return b;
}

__device__ __forceinline__ int64_t lower_bound_u64(const unsigned long long *a, int64_t lo, int64_t hi,
                                                   unsigned long long x) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Neighbouring-community table of one vertex (or community): the LDS table
// when the number of entries to insert is at most SLOTS/2, else the graph's
// dense global table (value per community id, touched ids listed).  Slots
// taken are listed, so reading and clearing cost the number of distinct keys.
template <int T, int SLOTS>
struct Tab {
  using Sh = FSh<T, SLOTS>;
  bool dense;
  double *dv;    // dense values
  int32_t *df;   // dense taken flags
  int32_t *dl;   // dense list

  __device__ void add(Sh &s, int key, double x) const {
    if (dense) {
      unsafeAtomicAdd(&dv[key], x);
      if (atomicExch(&df[key], 1) == 0) dl[atomicAdd(&s.tcnt, 1)] = key;
      return;
    }
    uint32_t h = mix32((uint32_t)key) & (uint32_t)(SLOTS - 1);
    for (int probe = 0; probe < SLOTS; ++probe) {
      const int k = __atomic_load_n(&s.tkeys[h], __ATOMIC_RELAXED);
      if (k == key) { atomicAdd(&s.tvals[h], x); return; }
      if (k == kEmpty) {
        const int old = atomicCAS(&s.tkeys[h], kEmpty, key);
        if (old == kEmpty) {
          atomicAdd(&s.tvals[h], x);
          s.tlist[atomicAdd(&s.tcnt, 1)] = (int)h;
          return;
        }
        if (old == key) { atomicAdd(&s.tvals[h], x); return; }
      }
      h = (h + 1) & (uint32_t)(SLOTS - 1);
    }
  }
  // entry q < s.tcnt (after a barrier following the inserts)
  __device__ void get(const Sh &s, int q, int &key, double &x) const {
    if (dense) {
      key = dl[q];
      x = ldx(&dv[key]);
    } else {
      const int h = s.tlist[q];
      key = s.tkeys[h];
      x = s.tvals[h];
    }
  }
  // clears what was taken; ends with the table empty and a barrier
  __device__ void clear(Sh &s) const {
    const int n = s.tcnt;
    for (int q = (int)threadIdx.x; q < n; q += T) {
      if (dense) {
        const int key = dl[q];
        dv[key] = 0.0;
        df[key] = 0;
      } else {
        const int h = s.tlist[q];
        s.tkeys[h] = kEmpty;
        s.tvals[h] = 0.0;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s.tcnt = 0;
    __syncthreads();
  }
};

// Level graph of the pass loop.
struct FLevel {
  int64_t n, nnz;
  const int64_t *off;
  const int32_t *idx;
  const float *w;
};

template <int T, int SLOTS>
struct FleetRun {
  using Sh = FSh<T, SLOTS>;
  using B = Blk<T, SLOTS>;
  Sh &s;
  FleetGraph &g;
  const FleetJob &job;
  FleetResult *res;
  const FleetParams &prm;
  int br = 0;  // buffer of the sorted batch

  __device__ Tab<T, SLOTS> table(int64_t entries) const {
    Tab<T, SLOTS> t;
    t.dense = entries > SLOTS / 2;
    t.dv = g.dense;
    t.df = g.tflag;
    t.dl = g.tlist;
    return t;
  }

  // Candidate positions of the tile [b0, b0+T) with flag set, ascending, in
  // s.list; count returned (all threads).
  __device__ int compact(int64_t b0, bool flag) {
    long long tot;
    const long long ex = B::excl(flag ? 1 : 0, &tot, s);
    if (flag) s.list[ex] = (int)(b0 + B::tid());
    __syncthreads();
    return (int)tot;
  }

  // ---------------- Alg. "leidenMove" (serial sweep) -----------------------
  // One vertex: best community by Eq. 2, applied at once.  Returns true if
  // it moved.
  __device__ bool move_vertex(const FLevel &L, int i, double M2, bool track, double &gsum, long long &moves) {
    const int64_t e0 = L.off[i], e1 = L.off[i + 1];
    const int d = g.Cl[i];
    const double Ki = g.Kl[i];
    const Tab<T, SLOTS> t = table(e1 - e0);
    double own = 0.0;
    for (int64_t e = e0 + B::tid(); e < e1; e += T) {
      const int j = L.idx[e];
      if (j == i) continue;
      const int c = g.Cl[j];
      const double x = (double)L.w[e];
      t.add(s, c, x);
      if (c == d) own += x;
    }
    const double b = B::sum_d(own, s);  // barrier: inserts complete
    const int nk = s.tcnt;
    const double Sd = g.Sl[d];
    double bg = 0.0;
    int bc = kNoComm;
    for (int q = B::tid(); q < nk; q += T) {
      int c;
      double a;
      t.get(s, q, c, a);
      if (c == d) continue;
      const double sc = move_score(M2, a, b, Ki, g.Sl[c], Sd);
      if (sc > 0.0 && better(sc, c, bg, bc)) { bg = sc; bc = c; }
    }
    B::argmax(bg, bc, s);
    t.clear(s);
    if (bc == kNoComm) return false;
    if (B::tid() == 0) {
      g.Cl[i] = bc;
      g.Sl[d] -= Ki;
      g.Sl[bc] += Ki;
      gsum += bg;
      moves += 1;
      if (track) {
        g.dC[d] = 1;
        g.dC[bc] = 1;
      }
    }
    for (int64_t e = e0 + B::tid(); e < e1; e += T) {
      const int j = L.idx[e];
      if (j != i) g.U[j] = 1;
    }
    __syncthreads();
    return true;
  }

  // Iterations of the local-moving phase; returns l (iterations executed).
  __device__ int move(const FLevel &L, bool use_rng, double M2, double Tp, bool track, long long &moves_out) {
    int l = 0;
    long long moves = 0;
    for (int it = 0; it < prm.max_iter; ++it) {
      double gsum = 0.0;  // thread 0: the moves' gains in visiting order
      for (int64_t b0 = 0; b0 < L.n; b0 += T) {
        const int64_t i = b0 + B::tid();
        int cnt = compact(b0, i < L.n && g.U[i] && (!use_rng || g.rng[i]));
        int k = 0;
        while (k < cnt) {
          const int v = s.list[k];
          __syncthreads();
          if (B::tid() == 0) g.U[v] = 0;
          const bool moved = move_vertex(L, v, M2, track, gsum, moves);
          if (moved) {
            // later vertices of the tile may have been marked unprocessed
            cnt = compact(b0, i < L.n && i > v && g.U[i] && (!use_rng || g.rng[i]));
            k = 0;
          } else {
            ++k;
          }
        }
        __syncthreads();
      }
      l = it + 1;
      if (B::tid() == 0) s.rd[0] = gsum;
      __syncthreads();
      const double gs = s.rd[0];
      __syncthreads();
      if (gs <= Tp) break;
    }
    moves_out = moves;
    return l;
  }

  // ---------------- Alg. "leidenRefine" (serial sweep) ---------------------
  __device__ bool refine_vertex(const FLevel &L, int i, double M2) {
    const int64_t e0 = L.off[i], e1 = L.off[i + 1];
    const int c = g.Cl[i];
    const int cb = g.CB[i];
    const double Ki = g.Kl[i];
    const Tab<T, SLOTS> t = table(e1 - e0);
    double own = 0.0;
    for (int64_t e = e0 + B::tid(); e < e1; e += T) {
      const int j = L.idx[e];
      if (j == i || g.CB[j] != cb) continue;
      const int cj = g.Cl[j];
      const double x = (double)L.w[e];
      t.add(s, cj, x);
      if (cj == c) own += x;
    }
    const double b = B::sum_d(own, s);
    const int nk = s.tcnt;
    const double Sd = g.Sl[c];
    double bg = 0.0;
    int bc = kNoComm;
    for (int q = B::tid(); q < nk; q += T) {
      int cj;
      double a;
      t.get(s, q, cj, a);
      if (cj == c) continue;
      const double sc = move_score(M2, a, b, Ki, g.Sl[cj], Sd);
      if (sc > 0.0 && better(sc, cj, bg, bc)) { bg = sc; bc = cj; }
    }
    B::argmax(bg, bc, s);
    t.clear(s);
    if (bc == kNoComm) return false;
    if (g.Cl[bc] != bc) return false;
    if (B::tid() == 0) {
      g.Sl[c] = 0.0;
      g.Sl[bc] += Ki;
      g.Cl[i] = bc;
    }
    __syncthreads();
    return true;
  }

  __device__ void refine(const FLevel &L, double M2) {
    for (int64_t b0 = 0; b0 < L.n; b0 += T) {
      const int64_t i = b0 + B::tid();
      const bool in_bound = i < L.n && g.dC[g.CB[i]];
      int cnt = compact(b0, in_bound && g.Sl[g.Cl[i]] == g.Kl[i]);
      int k = 0;
      while (k < cnt) {
        const int v = s.list[k];
        __syncthreads();
        if (refine_vertex(L, v, M2)) {
          cnt = compact(b0, in_bound && i > v && g.Sl[g.Cl[i]] == g.Kl[i]);
          k = 0;
        } else {
          ++k;
        }
      }
      __syncthreads();
    }
  }

  // ---------------- Alg. "leidenSubsetRenumber", break, renumber -----------
  __device__ void subset_renumber(int64_t n) {
    int32_t *rep = g.tmpi;
    for (int64_t c = B::tid(); c < n; c += T) rep[c] = INT_MAX;
    __syncthreads();
    for (int64_t i = B::tid(); i < n; i += T) atomicMin(&rep[g.Cl[i]], (int)i);
    __syncthreads();
    for (int64_t c = B::tid(); c < n; c += T) {
      g.S2[c] = 0.0;
      g.dC2[c] = 0;
    }
    __syncthreads();
    for (int64_t c = B::tid(); c < n; c += T) {
      const int r = ldx(&rep[c]);
      if (r != INT_MAX) {
        g.S2[r] = g.Sl[c];
        g.dC2[r] = g.dC[c];
      }
    }
    __syncthreads();
    for (int64_t i = B::tid(); i < n; i += T) g.Cl[i] = ldx(&rep[g.Cl[i]]);
    __syncthreads();
    if (B::tid() == 0) {
      double *ts = g.Sl;
      g.Sl = g.S2;
      g.S2 = ts;
      uint8_t *tc = g.dC;
      g.dC = g.dC2;
      g.dC2 = tc;
    }
    __syncthreads();
  }

  __device__ void break_changed(int64_t n) {
    for (int64_t i = B::tid(); i < n; i += T) {
      if (g.dC[g.Cl[i]]) {
        g.Cl[i] = (int)i;
        g.Sl[i] = g.Kl[i];
      }
    }
    __syncthreads();
  }

  // Dense ascending relabel of lab[0..n) (labels < bound); returns the count.
  __device__ int64_t renumber(int32_t *lab, int64_t n, int64_t bound) {
    int32_t *map = g.tmpi;
    for (int64_t c = B::tid(); c <= bound; c += T) map[c] = 0;
    __syncthreads();
    for (int64_t i = B::tid(); i < n; i += T) map[lab[i]] = 1;
    __syncthreads();
    const long long k = B::scan(map, map, bound, s);
    for (int64_t i = B::tid(); i < n; i += T) lab[i] = map[lab[i]];
    __syncthreads();
    return k;
  }

  // ---------------- Alg. "leidenAggregate" ---------------------------------
  // Super-vertex CSR of L under dense labels Cl (< nc) into level buffer ob,
  // K' (row sums of the stored float weights, in row order) into Kl.
  // Entries are sorted by (C[u], C[v]) with a stable sort, so the sums of a
  // pair take its entries in member-then-CSR order.
  __device__ FLevel aggregate(const FLevel &L, int64_t nc, int ob) {
    unsigned long long *key[2] = {g.akey[0], g.akey[1]};
    int32_t *pay[2] = {g.apay[0], g.apay[1]};
    for (int64_t u = B::wid(); u < L.n; u += B::W) {
      const unsigned long long cu = (unsigned long long)g.Cl[u];
      for (int64_t e = L.off[u] + lane(); e < L.off[u + 1]; e += kWave) {
        key[0][e] = cu * (unsigned long long)nc + (unsigned long long)g.Cl[L.idx[e]];
        pay[0][e] = (int32_t)e;
      }
    }
    __syncthreads();
    const unsigned long long top = (unsigned long long)nc * (unsigned long long)nc - 1ull;
    const int r = B::sort(key, pay, L.nnz, nc > 1 ? bits_for(top) : 0, s);
    const unsigned long long *sk = key[r];
    const int32_t *sp = pay[r];
    // distinct keys: head flags, then output positions by a scan
    int64_t *pos = (int64_t *)key[r ^ 1];
    for (int64_t t = B::tid(); t < L.nnz; t += T) pos[t] = (t == 0 || sk[t] != sk[t - 1]) ? 1 : 0;
    __syncthreads();
    const int64_t nu = B::scan(pos, pos, L.nnz, s);
    int64_t *off = g.loff[ob];
    int32_t *idx = g.lidx[ob];
    float *w = g.lw[ob];
    int64_t *rc = g.mcnt;
    double *sum = g.asum;
    for (int64_t c = B::tid(); c <= nc; c += T) rc[c] = 0;
    for (int64_t o = B::tid(); o < nu; o += T) sum[o] = 0.0;
    __syncthreads();
    for (int64_t t = B::tid(); t < L.nnz; t += T) {
      const bool head = t == 0 || sk[t] != sk[t - 1];
      const int64_t o = ldx(&pos[t]) - (head ? 0 : 1);
      unsafeAtomicAdd(&sum[o], (double)L.w[sp[t]]);
      if (head) {
        idx[o] = (int32_t)(sk[t] % (unsigned long long)nc);
        atomicAdd((unsigned long long *)&rc[sk[t] / (unsigned long long)nc], 1ull);
      }
    }
    __syncthreads();
    for (int64_t o = B::tid(); o < nu; o += T) w[o] = (float)ldx(&sum[o]);
    __syncthreads();
    B::scan(rc, off, nc, s);
    for (int64_t c = B::tid(); c < nc; c += T) {
      double k = 0.0;
      for (int64_t e = off[c]; e < off[c + 1]; ++e) k += (double)w[e];
      g.Kl[c] = k;
    }
    __syncthreads();
    FLevel o{nc, nu, off, idx, w};
    return o;
  }

  // ---------------- the pass loop of Alg. "leiden" --------------------------
  // On entry Cl, Kl, Sl, dC, U, rng hold the level-0 state; result: dense
  // labels in g.C.
  __device__ void core(const FLevel &L0, double M2, bool track) {
    const int64_t n0 = L0.n;
    for (int64_t i = B::tid(); i < n0; i += T) g.Ctop[i] = (int)i;
    if (prm.refine_variant == 1) {
      for (int64_t i = B::tid(); i < n0; i += T) g.dC[i] = 1;
      track = false;
    }
    __syncthreads();
    FLevel L = L0;
    int buf = 0;
    double tau = prm.tau0;
    int pass;
    for (pass = 0; pass < prm.max_passes; ++pass) {
      const int64_t nl = L.n;
      const double Tp = tau * M2 * M2 / 2.0;
      long long mv = 0;
      const int li = move(L, pass == 0, M2, Tp, track && pass == 0, mv);
      if (B::tid() == 0 && pass < 16) {
        res->move_iters[pass] = li;
        res->level_vertices[pass] = nl;
      }
      if (pass == 0) {
        long long ch = 0;
        for (int64_t c = B::tid(); c < nl; c += T) ch += g.dC[c] ? 1 : 0;
        ch = B::sum_l(ch, s);
        if (B::tid() == 0) {
          res->moves_pass0 = mv;
          res->changed = ch;
        }
      }
      subset_renumber(nl);
      for (int64_t i = B::tid(); i < nl; i += T) g.CB[i] = g.Cl[i];
      __syncthreads();
      break_changed(nl);
      refine(L, M2);
      if (B::tid() == 0) res->passes = pass + 1;
      if ((pass > 0 || prm.refine_variant == 2) && li <= 1) break;
      const int64_t nc = renumber(g.Cl, nl, nl);
      if (B::tid() == 0 && pass < 16) res->communities[pass] = nc;
      if (prm.agg_tol < 1.0 && (double)nc / (double)nl > prm.agg_tol) break;
      for (int64_t i = B::tid(); i < n0; i += T) g.Ctop[i] = g.Cl[g.Ctop[i]];
      __syncthreads();
      L = aggregate(L, nc, buf);
      buf ^= 1;
      for (int64_t i = B::tid(); i < nc; i += T) {
        g.Sl[i] = g.Kl[i];
        g.U[i] = 1;
        g.Cl[i] = (int)i;
        g.dC[i] = 1;
      }
      __syncthreads();
      tau = tau / prm.tol_drop;
    }
    if (pass >= prm.max_passes && B::tid() == 0) res->passes = prm.max_passes;
    for (int64_t i = B::tid(); i < n0; i += T) g.Ctop[i] = g.Cl[g.Ctop[i]];
    __syncthreads();
    renumber(g.Ctop, n0, n0);
    for (int64_t i = B::tid(); i < n0; i += T) g.C[i] = g.Ctop[i];
    __syncthreads();
  }

  // ---------------- graph update (Sec. 3.5, 5.1.4) ------------------------
  // Validates the batch against the current CSR and writes G^t into the other
  // buffer.  Returns the error bits (0: applied; the graph then switches).
  __device__ int apply_batch() {
    const int64_t n = g.n;
    const int64_t nd = job.nd, ni = job.ni;
    const int64_t E = 2 * (nd + ni);
    const int cur = g.cur;
    const int64_t *off = g.off[cur];
    const int32_t *idx = g.idx[cur];
    const float *w = g.w[cur];
    unsigned long long *key[2] = {job.bkey[0], job.bkey[1]};
    int32_t *pay[2] = {job.bpay[0], job.bpay[1]};
    int err = 0;
    for (int64_t t = B::tid(); t < E; t += T) {
      const int64_t k = t >> 1;
      const bool del = k < nd;
      const int a = del ? job.du[k] : job.iu[k - nd];
      const int b = del ? job.dv[k] : job.iv[k - nd];
      const int u = (t & 1) ? b : a, v = (t & 1) ? a : b;
      float x = 0.0f;
      if (!del) {
        x = job.iw[k - nd];
        if (!(x > 0.0f) || !isfinite(x)) err |= 32;
      }
      if (u < 0 || u >= n || v < 0 || v >= n) {
        err |= 1;
        key[0][t] = kNoKey;
      } else {
        if (u == v) err |= 2;
        key[0][t] = (unsigned long long)u * (unsigned long long)n + (unsigned long long)v;
      }
      pay[0][t] = (int32_t)t;
      job.bw[t] = x;
    }
    err = B::or_i(err, s);
    if (err) return err;
    const unsigned long long top = (unsigned long long)n * (unsigned long long)n - 1ull;
    const int r = (E > 0) ? B::sort(key, pay, E, bits_for(top), s) : 0;
    br = r;
    const unsigned long long *sk = key[r];
    const int32_t *sp = pay[r];
    int32_t *pre = job.bpre;
    int32_t *seg0 = g.CB;    // first sorted position of each row's batch entries (-1: none)
    for (int64_t u = B::tid(); u < n; u += T) seg0[u] = -1;
    __syncthreads();
    for (int64_t t = B::tid(); t < E; t += T) {
      const unsigned long long kk = sk[t];
      const int u = (int)(kk / (unsigned long long)n), v = (int)(kk % (unsigned long long)n);
      const bool del = sp[t] < 2 * nd;
      if (t > 0 && sk[t - 1] == kk) err |= 4;
      if (t == 0 || sk[t - 1] / (unsigned long long)n != (unsigned long long)u) seg0[u] = (int)t;
      const int64_t p = lower_bound_i32(idx, off[u], off[u + 1], v);
      const bool found = p < off[u + 1] && idx[p] == v;
      if (del && !found) err |= 8;
      if (!del && found) err |= 16;
      if (del && found) job.bw[sp[t]] = w[p];
      pre[t] = del ? 1 : 0;
      atomicAdd(&g.rowd[u], del ? -1 : 1);
    }
    err = B::or_i(err, s);
    if (err) {
      for (int64_t u = B::tid(); u < n; u += T) g.rowd[u] = 0;
      __syncthreads();
      return err;
    }
    B::scan(pre, pre, E, s);
    // new offsets
    const int nb = cur ^ 1;
    int64_t *noff = g.off[nb];
    int32_t *nidx = g.idx[nb];
    float *nw = g.w[nb];
    for (int64_t u = B::tid(); u < n; u += T) {
      g.mcnt[u] = off[u + 1] - off[u] + ldx(&g.rowd[u]);
      g.rowd[u] = 0;
    }
    __syncthreads();
    const int64_t nnz_new = B::scan(g.mcnt, noff, n, s);
    // surviving old entries
    for (int64_t u = B::wid(); u < n; u += B::W) {
      const int64_t o0 = off[u], o1 = off[u + 1];
      const int s0 = seg0[u];
      if (s0 < 0) {
        for (int64_t e = o0 + lane(); e < o1; e += kWave) {
          nidx[noff[u] + (e - o0)] = idx[e];
          nw[noff[u] + (e - o0)] = w[e];
        }
        continue;
      }
      int64_t s1 = s0;
      const unsigned long long lo = (unsigned long long)u * (unsigned long long)n;
      s1 = lower_bound_u64(sk, s0, E, lo + (unsigned long long)n);
      for (int64_t e = o0 + lane(); e < o1; e += kWave) {
        const int v = idx[e];
        const int64_t p = lower_bound_u64(sk, s0, s1, lo + (unsigned long long)v);
        const int64_t dels = pre[p] - pre[s0];
        const int64_t inss = (p - s0) - dels;
        if (p < s1 && sk[p] == lo + (unsigned long long)v) continue;  // deleted (an insertion cannot match)
        const int64_t o = noff[u] + (e - o0) - dels + inss;
        nidx[o] = v;
        nw[o] = w[e];
      }
    }
    // inserted entries
    for (int64_t t = B::tid(); t < E; t += T) {
      if (sp[t] < 2 * nd) continue;
      const unsigned long long kk = sk[t];
      const int u = (int)(kk / (unsigned long long)n), v = (int)(kk % (unsigned long long)n);
      const int s0 = seg0[u];
      const int64_t olds = lower_bound_i32(idx, off[u], off[u + 1], v) - off[u];
      const int64_t dels = pre[t] - pre[s0];
      const int64_t inss = (t - s0) - dels;
      const int64_t o = noff[u] + olds - dels + inss;
      nidx[o] = v;
      nw[o] = job.bw[sp[t]];
    }
    __syncthreads();
    if (B::tid() == 0) {
      g.cur = nb;
      g.nnz = nnz_new;
    }
    __syncthreads();
    return 0;
  }

  // ---------------- marking, changedCommunities, updateWeights -------------
  // On the sorted batch (key / payload buffer r) and G^t; previous C, K,
  // Sigma, M2.  Leaves U = affected, rng = in range, dC = changed.
  __device__ void mark(int mode, int r) {
    const int64_t n = g.n;
    const int64_t nd = job.nd, ni = job.ni;
    const int64_t E = 2 * (nd + ni);
    const unsigned long long *sk = job.bkey[r];
    const int32_t *sp = job.bpay[r];
    const int64_t *off = g.off[g.cur];
    const int32_t *idx = g.idx[g.cur];
    for (int64_t i = B::tid(); i < n; i += T) {
      g.U[i] = (mode == 1) ? 1 : 0;
      g.dC[i] = 0;
      g.dE[i] = 0;
      g.dCm[i] = 0;
    }
    __syncthreads();
    for (int64_t t = B::tid(); t < E; t += T) {
      const unsigned long long kk = sk[t];
      const int u = (int)(kk / (unsigned long long)n), v = (int)(kk % (unsigned long long)n);
      const bool del = sp[t] < 2 * nd;
      const bool same = g.C[u] == g.C[v];
      if (same) g.dC[g.C[u]] = 1;  // changedCommunities
      if (mode == 3 && ((del && same) || (!del && !same))) g.U[u] = 1;
      if (mode == 2 && del && same) {
        g.U[u] = 1;
        g.dE[u] = 1;
        g.dCm[g.C[v]] = 1;
      }
    }
    if (mode == 2) {
      // per unique source of insertions: the community of the best score
      // over its cross-community insertions (previous K, Sigma, M2)
      for (int64_t t = B::tid(); t < E; t += T) {
        const unsigned long long kk = sk[t];
        const int u = (int)(kk / (unsigned long long)n);
        if (t > 0 && sk[t - 1] / (unsigned long long)n == (unsigned long long)u) continue;
        int64_t t1 = t;
        while (t1 < E && sk[t1] / (unsigned long long)n == (unsigned long long)u) ++t1;
        const int cu = g.C[u];
        int best = -1;
        double bestg = 0.0;
        for (int64_t a = t; a < t1; ++a) {
          if (sp[a] < 2 * nd) continue;
          const int ca = g.C[(int)(sk[a] % (unsigned long long)n)];
          if (ca == cu) continue;
          bool seen = false;
          for (int64_t q = t; q < a && !seen; ++q)
            if (sp[q] >= 2 * nd && g.C[(int)(sk[q] % (unsigned long long)n)] == ca) seen = true;
          if (seen) continue;
          double h = 0.0;
          for (int64_t q = a; q < t1; ++q)
            if (sp[q] >= 2 * nd && g.C[(int)(sk[q] % (unsigned long long)n)] == ca)
              h += (double)job.bw[sp[q]];
          const double sc = (g.M2 * h) - (g.K[u] * g.Sig[ca]);
          if (best < 0 || sc > bestg || (sc == bestg && ca < best)) { best = ca; bestg = sc; }
        }
        if (best >= 0) {
          g.U[u] = 1;
          g.dE[u] = 1;
          g.dCm[best] = 1;
        }
      }
      __syncthreads();
      for (int64_t u = B::wid(); u < n; u += B::W) {
        if (!g.dE[u]) continue;
        for (int64_t e = off[u] + lane(); e < off[u + 1]; e += kWave) g.U[idx[e]] = 1;
      }
      __syncthreads();
      for (int64_t i = B::tid(); i < n; i += T)
        if (g.dCm[g.C[i]]) g.U[i] = 1;
    }
    __syncthreads();
    for (int64_t i = B::tid(); i < n; i += T) g.rng[i] = (mode == 2) ? g.U[i] : 1;
    // updateWeights: K and Sigma of the previous membership, and 2m
    double dm = 0.0;
    for (int64_t t = B::tid(); t < E; t += T) {
      const int u = (int)(sk[t] / (unsigned long long)n);
      const bool del = sp[t] < 2 * nd;
      const double x = (double)job.bw[sp[t]];
      unsafeAtomicAdd(&g.K[u], del ? -x : x);
      unsafeAtomicAdd(&g.Sig[g.C[u]], del ? -x : x);
      dm += del ? -x : x;
    }
    dm = B::sum_d(dm, s);
    __syncthreads();
    if (B::tid() == 0) g.M2 = g.M2 + dm;
    __syncthreads();
    long long aff = 0;
    for (int64_t i = B::tid(); i < n; i += T) aff += g.U[i] ? 1 : 0;
    aff = B::sum_l(aff, s);
    if (B::tid() == 0) res->affected = aff;
    __syncthreads();
  }

  // Eq. 1 of the current graph and g.C (dense labels); also Sigma^t.
  __device__ double modularity() {
    const int64_t n = g.n;
    const int64_t *off = g.off[g.cur];
    const int32_t *idx = g.idx[g.cur];
    const float *w = g.w[g.cur];
    double *sig = g.dense;   // holds 0 between uses
    for (int64_t c = B::tid(); c < n; c += T) g.Sig[c] = 0.0;
    __syncthreads();
    for (int64_t i = B::tid(); i < n; i += T) unsafeAtomicAdd(&g.Sig[g.C[i]], ldx(&g.K[i]));
    for (int64_t u = B::wid(); u < n; u += B::W) {
      const int cu = g.C[u];
      double in = 0.0;
      for (int64_t e = off[u] + lane(); e < off[u + 1]; e += kWave)
        if (g.C[idx[e]] == cu) in += (double)w[e];
      in = group_sum<kWave>(in);
      if (lane() == 0 && in != 0.0) unsafeAtomicAdd(&sig[cu], in);
    }
    __syncthreads();
    const double M2 = g.M2;
    double q = 0.0;
    for (int64_t c = B::tid(); c < n; c += T) {
      const double sc = ldx(&sig[c]);
      const double a = ldx(&g.Sig[c]) / M2;
      if (M2 > 0.0) q += sc / M2 - a * a;
      sig[c] = 0.0;
    }
    q = B::sum_d(q, s);
    return M2 > 0.0 ? q : 0.0;
  }

  __device__ void run() {
    const int mode = job.mode;
    const int64_t n = g.n;
    if (B::tid() == 0) {
      res->status = 0;
      res->err = 0;
      res->passes = 0;
      res->q = 0.0;
      res->affected = res->changed = res->moves_pass0 = 0;
      for (int k = 0; k < 16; ++k) {
        res->move_iters[k] = 0;
        res->level_vertices[k] = 0;
        res->communities[k] = 0;
      }
    }
    if (mode != 0 && !g.has_state) {
      if (B::tid() == 0) res->status = 3;
      return;
    }
    double M2;
    bool track;
    if (mode == 0) {
      const int64_t *off = g.off[g.cur];
      const float *w = g.w[g.cur];
      for (int64_t i = B::tid(); i < n; i += T) {
        double k = 0.0;
        for (int64_t e = off[i]; e < off[i + 1]; ++e) k += (double)w[e];
        g.K[i] = k;
        g.Kl[i] = k;
        g.Sl[i] = k;
        g.Cl[i] = (int)i;
        g.dC[i] = 1;
        g.U[i] = 1;
        g.rng[i] = 1;
      }
      double m2 = 0.0;
      for (int64_t i = B::tid(); i < n; i += T) m2 += g.K[i];
      m2 = B::sum_d(m2, s);
      if (B::tid() == 0) g.M2 = m2;
      __syncthreads();
      M2 = m2;
      track = false;
      if (B::tid() == 0) res->affected = n;
    } else {
      const int err = apply_batch();
      if (err) {
        if (B::tid() == 0) {
          res->status = 1;
          res->err = err;
        }
        return;
      }
      mark(mode, br);
      for (int64_t i = B::tid(); i < n; i += T) {
        g.Cl[i] = g.C[i];
        g.Kl[i] = ldx(&g.K[i]);
        g.Sl[i] = ldx(&g.Sig[i]);
      }
      __syncthreads();
      M2 = g.M2;
      track = true;
    }
    FLevel L0{n, g.nnz, g.off[g.cur], g.idx[g.cur], g.w[g.cur]};
    if (n > 0) core(L0, M2, track);
    const double q = modularity();
    if (job.out)
      for (int64_t i = B::tid(); i < n; i += T) job.out[i] = g.C[i];
    if (B::tid() == 0) {
      res->q = q;
      g.has_state = 1;
    }
    __syncthreads();
  }
};

template <int T, int SLOTS>
__global__ __launch_bounds__(T) void k_fleet(FleetLaunch a) {
  __shared__ FSh<T, SLOTS> s;
  for (int k = threadIdx.x; k < SLOTS; k += T) {
    s.tkeys[k] = kEmpty;
    s.tvals[k] = 0.0;
  }
  if (threadIdx.x == 0) s.tcnt = 0;
  __syncthreads();
  const int njobs = *a.njobs;
  for (;;) {
    if (threadIdx.x == 0) s.cnt = (int)atomicAdd(a.next, 1ull);
    __syncthreads();
    const int j = s.cnt;
    __syncthreads();
    if (j >= njobs) break;
    if (threadIdx.x == 0) {
      s.job = a.jobs[j];
      s.g = a.graphs[s.job.graph];
    }
    __syncthreads();
    // the graph record and the job stay in LDS: fields every thread reads,
    // written by thread 0 between barriers
    FleetRun<T, SLOTS> run{s, s.g, s.job, &a.results[j], a.prm};
    run.run();
    __syncthreads();
    if (threadIdx.x == 0) {
      FleetGraph *dst = &a.graphs[s.job.graph];
      dst->nnz = s.g.nnz;
      dst->cur = s.g.cur;
      dst->M2 = s.g.M2;
      dst->has_state = s.g.has_state;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t fleet_launch(const FleetLaunch &L, int variant, int blocks, hipStream_t s) {
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_fleet<64, 512>), blocks, 64, 0, s, L); break;
    case 1: hipLaunchKernelGGL((k_fleet<128, 512>), blocks, 128, 0, s, L); break;
    case 2: hipLaunchKernelGGL((k_fleet<256, 512>), blocks, 256, 0, s, L); break;
    case 3: hipLaunchKernelGGL((k_fleet<64, 2048>), blocks, 64, 0, s, L); break;
    case 4: hipLaunchKernelGGL((k_fleet<128, 2048>), blocks, 128, 0, s, L); break;
    default: hipLaunchKernelGGL((k_fleet<256, 2048>), blocks, 256, 0, s, L); break;
  }
  return hipGetLastError();
}

}  // namespace lk
