/*
 * Serial CPU oracle for dynamic Leiden community detection (Static, ND, DS, DF).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may build, load
 * or call it; the product path never does.  It shares no code, header, table
 * or helper with the GPU library.
 *
 * Every routine follows a passage of Sahu, "A Starting Point for Dynamic
 * Community Detection with Leiden Algorithm" (arXiv 2405.11658); the passage
 * is named in the comment above it.  Where the paper is silent or ambiguous the
 * chosen reading is stated next to the code (the same readings are listed in
 * the design notes of the repository).
 *
 * Conventions (paper, Sec. 5.1.2 "Configuration"):
 *   vertex ids int32, CSR offsets int64, stored edge weights float32,
 *   every weight total (K, Sigma, table values, scores, modularity) float64,
 *   8-bit flag vectors.
 * An undirected graph stores both directions; a self-loop (i,i,w) is stored
 * once and counts w towards K_i.  M2 = 2m = sum of all stored weights.
 *
 * Build with -ffp-contract=off: decision scores must not be FMA-contracted.
 *
 * Parity pins: see tests/test_oracle_pins.py (brute force, closed forms,
 * invariants).  Every exported function below is pinned there.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

#define OR_MODE_STATIC 0
#define OR_MODE_ND 1
#define OR_MODE_DS 2
#define OR_MODE_DF 3

#define OR_MAXP 64

typedef struct {
  double tau0;            /* initial iteration tolerance, 0.01 (Sec. 4.6)        */
  double tol_drop;        /* tolerance drop per pass, 10 (Sec. 4.6)              */
  double agg_tol;         /* aggregation tolerance; 1.0 = never skip (Sec. 4.6)  */
  int32_t max_iter;       /* local-moving iterations per pass, 20 (Sec. 4.6)     */
  int32_t max_passes;     /* passes; not stated in the paper, 10                 */
  int32_t sync_mode;      /* 0: serial asynchronous, 1: synchronous (sliced)     */
  int32_t refine_variant; /* 0 subset refine, 1 full refine, 2 no continued passes (Sec. 4.1-4.3) */
  int32_t nslices;        /* synchronous mode: slices per sweep (>= 1) */
} or_params;

typedef struct {
  int32_t passes;
  int32_t move_iters[OR_MAXP];
  int32_t refine_rounds[OR_MAXP];
  int64_t level_vertices[OR_MAXP];
  int64_t level_entries[OR_MAXP];
  int64_t communities[OR_MAXP];
  int64_t refined_vertices[OR_MAXP]; /* vertices whose bound is flagged changed at refinement */
  int64_t affected;      /* |{i : deltaV[i]}| at the start */
  int64_t changed;       /* |{c : deltaC'[c]}| after the first local-moving phase */
  int64_t moves_pass0;   /* vertex moves in the first local-moving phase */
} or_stats;

/* ------------------------------------------------------------------------ */
/* Dense "collision-free" table keyed by community id (Sec. 4.6: per-thread  */
/* hashtables indexed by id).  val[] has one slot per possible key; keys[]   */
/* lists the touched slots so a clear costs only what was inserted.           */
/* ------------------------------------------------------------------------ */
typedef struct {
  double *val;
  uint8_t *has;
  int32_t *keys;
  int64_t nkeys;
} dtab;

static int dtab_init(dtab *t, int64_t n) {
  int64_t m = n > 0 ? n : 1;
  t->val = (double *)calloc((size_t)m, sizeof(double));
  t->has = (uint8_t *)calloc((size_t)m, 1);
  t->keys = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  t->nkeys = 0;
  return (t->val && t->has && t->keys) ? OR_OK : OR_ENOMEM;
}
static void dtab_free(dtab *t) { free(t->val); free(t->has); free(t->keys); }
static void dtab_clear(dtab *t) {
  for (int64_t k = 0; k < t->nkeys; k++) {
    t->val[t->keys[k]] = 0.0;
    t->has[t->keys[k]] = 0;
  }
  t->nkeys = 0;
}
static void dtab_add(dtab *t, int32_t key, double w) {
  if (!t->has[key]) { t->has[key] = 1; t->keys[t->nkeys++] = key; }
  t->val[key] += w;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* Delta-modularity score, Eq. 2 multiplied by 2m^2:                          */
/*   g = M2*(K_{i->c} - K_{i->d}) - K_i*(K_i + Sigma_c - Sigma_d)             */
/* with Sigma_d including K_i.  Evaluated with this exact parenthesisation.   */
/* ------------------------------------------------------------------------ */
static double score(double M2, double a, double b, double Ki, double Sc, double Sd) {
  return (M2 * (a - b)) - (Ki * ((Ki + Sc) - Sd));
}

/* Best community among table keys other than d.  Only strictly positive   */
/* gains qualify; equal gains go to the smaller community id.  When         */
/* guard_self >= 0, singleton targets (sizes[c] == 1) with id > guard_self   */
/* are excluded (synchronous refinement only).                              */
static int32_t best_community(const dtab *H, int32_t d, double M2, double Ki,
                              const double *Sig, const int32_t *sizes,
                              int32_t guard_self, double *g_out) {
  double b = H->has[d] ? H->val[d] : 0.0;
  int32_t best = -1;
  double bestg = 0.0;
  for (int64_t k = 0; k < H->nkeys; k++) {
    int32_t c = H->keys[k];
    if (c == d) continue;
    if (guard_self >= 0 && sizes[c] == 1 && c > guard_self) continue;
    double g = score(M2, H->val[c], b, Ki, Sig[c], Sig[d]);
    if (!(g > 0.0)) continue;
    if (best < 0 || g > bestg || (g == bestg && c < best)) { best = c; bestg = g; }
  }
  *g_out = bestg;
  return best;
}

/* Fixed-order sum used by the synchronous mode: ascending 256-element tiles */
/* summed sequentially, then the tile sums summed sequentially.              */
static double tiled_sum(const double *x, int64_t n) {
  double total = 0.0;
  for (int64_t t0 = 0; t0 < n; t0 += 256) {
    int64_t t1 = t0 + 256 < n ? t0 + 256 : n;
    double s = 0.0;
    for (int64_t i = t0; i < t1; i++) s += x[i];
    total += s;
  }
  return total;
}

/* A level graph (G' in Alg. "leiden"): CSR, int64 offsets. */
typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *off;
  int32_t *idx;
  float *w;
  int owned;
} lgraph;

static void lgraph_free(lgraph *g) {
  if (g->owned) { free(g->off); free(g->idx); free(g->w); }
  memset(g, 0, sizeof(*g));
}

/* ------------------------------------------------------------------------ */
/* Local-moving phase, Alg. "leidenMove" with "scanCommunities" (self=false). */
/* Serial asynchronous reading: one sweep per iteration over vertex ids in    */
/* ascending order; a vertex is skipped unless unprocessed; it is marked      */
/* processed before the range test; a mover marks its neighbours (other than  */
/* itself) unprocessed, which a later vertex of the same sweep may see.       */
/* Convergence: the summed gain of an iteration, in units of 2m^2, compared   */
/* with Tp = tau * M2^2 / 2 (i.e. Delta-Q <= tau).  Returns the number of     */
/* iterations performed (1 when the first iteration converges).              */
/* ------------------------------------------------------------------------ */
static int32_t move_async(const lgraph *G, int32_t *C, const double *K, double *Sig,
                          uint8_t *dC, uint8_t *U, const uint8_t *rng, int track,
                          double M2, double Tp, int32_t max_iter, dtab *H, int64_t *nmoves,
                          double *gtot) {
  int32_t l = 0;
  for (int32_t it = 0; it < max_iter; it++) {
    double gsum = 0.0;
    for (int64_t i = 0; i < G->n; i++) {
      if (!U[i]) continue;
      U[i] = 0;
      if (!rng[i]) continue;
      int32_t d = C[i];
      dtab_clear(H);
      for (int64_t e = G->off[i]; e < G->off[i + 1]; e++) {
        int32_t j = G->idx[e];
        if (j == (int32_t)i) continue;
        dtab_add(H, C[j], (double)G->w[e]);
      }
      double g;
      int32_t c = best_community(H, d, M2, K[i], Sig, NULL, -1, &g);
      if (c < 0) continue;
      Sig[d] -= K[i];
      Sig[c] += K[i];
      C[i] = c;
      gsum += g;
      *gtot += g;
      (*nmoves)++;
      for (int64_t e = G->off[i]; e < G->off[i + 1]; e++)
        if (G->idx[e] != (int32_t)i) U[G->idx[e]] = 1;
      if (track) { dC[d] = 1; dC[c] = 1; }
    }
    l = it + 1;
    if (gsum <= Tp) break;
  }
  return l;
}

/* Slice of a vertex in the synchronous mode: MurmurHash3's 32-bit finaliser */
/* (fmix32, Appleby) of the id, modulo the number of slices.                 */
static int32_t slice_of(int64_t i, int32_t S) {
  uint32_t h = (uint32_t)i;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return (int32_t)(h % (uint32_t)S);
}

/* Synchronous local-moving (deterministic mode; not in the paper, whose     */
/* serial asynchronous order a GPU cannot reproduce).  An iteration sweeps   */
/* the S slices in order.  In a slice, every unprocessed in-range vertex of   */
/* the slice is marked processed and proposes its best move from the current */
/* state; a proposal d -> c is blocked when a neighbour of the same slice     */
/* proposes the exact reverse move c -> d with priority (larger gain; equal   */
/* gains: smaller id).  Accepted moves are applied at once and mark their    */
/* neighbours unprocessed (a later slice sees them in the same iteration);   */
/* blocked proposers stay unprocessed.  The iteration's gain is the sum of   */
/* the accepted gains in the fixed tile order above.                          */
static int32_t move_sync(const lgraph *G, int32_t *C, const double *K, double *Sig,
                         uint8_t *dC, uint8_t *U, const uint8_t *rng, int track,
                         double M2, double Tp, int32_t max_iter, int32_t S, dtab *H,
                         int64_t *nmoves, double *gtot) {
  int64_t n = G->n;
  int64_t m = n ? n : 1;
  int32_t *prop = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  int32_t *from = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  int32_t *sl = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  double *gp = (double *)malloc((size_t)m * sizeof(double));
  double *gi = (double *)malloc((size_t)m * sizeof(double));
  uint8_t *acc = (uint8_t *)malloc((size_t)m);
  int32_t l = 0;
  for (int64_t i = 0; i < n; i++) sl[i] = slice_of(i, S);
  for (int32_t it = 0; it < max_iter; it++) {
    for (int64_t i = 0; i < n; i++) gi[i] = 0.0;
    for (int32_t s = 0; s < S; s++) {
      /* proposals of the slice, from the current state */
      for (int64_t i = 0; i < n; i++) {
        prop[i] = -1;
        if (sl[i] != s || !U[i]) continue;
        U[i] = 0;
        if (!rng[i]) continue;
        int32_t d = C[i];
        dtab_clear(H);
        for (int64_t e = G->off[i]; e < G->off[i + 1]; e++) {
          int32_t j = G->idx[e];
          if (j == (int32_t)i) continue;
          dtab_add(H, C[j], (double)G->w[e]);
        }
        double g;
        int32_t c = best_community(H, d, M2, K[i], Sig, NULL, -1, &g);
        if (c < 0) continue;
        prop[i] = c;
        from[i] = d;
        gp[i] = g;
      }
      /* swap resolution among proposing neighbours of the slice */
      for (int64_t i = 0; i < n; i++) {
        acc[i] = 0;
        if (prop[i] < 0) continue;
        int win = 1;
        for (int64_t e = G->off[i]; e < G->off[i + 1] && win; e++) {
          int32_t j = G->idx[e];
          if (j == (int32_t)i || prop[j] < 0) continue;
          if (prop[j] != from[i] || from[j] != prop[i]) continue;
          if (gp[j] > gp[i] || (gp[j] == gp[i] && j < (int32_t)i)) win = 0;
        }
        acc[i] = (uint8_t)win;
      }
      for (int64_t i = 0; i < n; i++) {
        if (prop[i] < 0) continue;
        if (!acc[i]) { U[i] = 1; continue; }
        int32_t c = prop[i], d = from[i];
        C[i] = c;
        Sig[d] -= K[i];
        Sig[c] += K[i];
        gi[i] = gp[i];
        (*nmoves)++;
        for (int64_t e = G->off[i]; e < G->off[i + 1]; e++)
          if (G->idx[e] != (int32_t)i) U[G->idx[e]] = 1;
        if (track) { dC[d] = 1; dC[c] = 1; }
      }
    }
    double gsum = tiled_sum(gi, n);
    *gtot += gsum;
    l = it + 1;
    if (gsum <= Tp) break;
  }
  free(prop); free(from); free(sl); free(gp); free(gi); free(acc);
  return l;
}

/* ------------------------------------------------------------------------ */
/* Alg. "leidenSubsetRenumber": relabel each community by one of its member  */
/* vertices and re-key Sigma' and deltaC' accordingly.  The paper takes any  */
/* member; this reading takes the smallest member id so the result is        */
/* deterministic.                                                            */
/* ------------------------------------------------------------------------ */
static void subset_renumber(int64_t n, int32_t *C, double *Sig, uint8_t *dC,
                            int32_t *rep, double *Sig2, uint8_t *dC2) {
  for (int64_t c = 0; c < n; c++) rep[c] = -1;
  for (int64_t i = 0; i < n; i++)
    if (rep[C[i]] < 0) rep[C[i]] = (int32_t)i; /* ascending i: first is smallest */
  for (int64_t c = 0; c < n; c++) { Sig2[c] = 0.0; dC2[c] = 0; }
  for (int64_t c = 0; c < n; c++) {
    if (rep[c] < 0) continue;
    Sig2[rep[c]] = Sig[c];
    dC2[rep[c]] = dC[c];
  }
  for (int64_t i = 0; i < n; i++) C[i] = rep[C[i]];
  memcpy(Sig, Sig2, (size_t)n * sizeof(double));
  memcpy(dC, dC2, (size_t)n);
}

/* Function "breakChangedCommunities" of Alg. "leiden": isolate every vertex */
/* of a changed community.                                                    */
static void break_changed(int64_t n, int32_t *C, const double *K, double *Sig, const uint8_t *dC) {
  for (int64_t i = 0; i < n; i++) {
    if (!dC[C[i]]) continue;
    C[i] = (int32_t)i;
    Sig[i] = K[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Alg. "leidenRefine" with "scanBounded" (self=false): one sweep of         */
/* constrained merges of isolated vertices inside their community bound.     */
/* Reading: the changed test uses the flag of the vertex's bound, deltaC'[CB */
/* [i]] (after the break every vertex is its own label, so testing its own   */
/* label would skip all non-representatives).  Serially the compare-and-swap */
/* on Sigma'[c] always succeeds once the isolation test has passed.          */
/* ------------------------------------------------------------------------ */
static int32_t refine_async(const lgraph *G, const int32_t *CB, int32_t *C, const double *K,
                            double *Sig, const uint8_t *dC, double M2, dtab *H) {
  for (int64_t i = 0; i < G->n; i++) {
    if (!dC[CB[i]]) continue;
    int32_t c = C[i];
    if (Sig[c] != K[i]) continue;
    dtab_clear(H);
    for (int64_t e = G->off[i]; e < G->off[i + 1]; e++) {
      int32_t j = G->idx[e];
      if (j == (int32_t)i) continue;
      if (CB[j] != CB[i]) continue;
      dtab_add(H, C[j], (double)G->w[e]);
    }
    double g;
    int32_t cs = best_community(H, c, M2, K[i], Sig, NULL, -1, &g);
    if (cs < 0) continue;
    if (C[cs] != cs) continue;
    Sig[c] = 0.0;
    Sig[cs] += K[i];
    C[i] = cs;
  }
  return 1;
}

/* Synchronous refinement (deterministic mode; not in the paper).  One sweep */
/* over the S slices in order, like the paper's single sweep.  In a slice,    */
/* every isolated vertex of a changed bound proposes its best target inside   */
/* the bound from the current state; a proposal is accepted when the target's */
/* representative is not proposing in the slice, or when the two propose to  */
/* each other and the proposer has priority (larger gain; equal gains:        */
/* smaller id).  Accepted merges are applied at once.                         */
static int32_t refine_sync(const lgraph *G, const int32_t *CB, int32_t *C, const double *K,
                           double *Sig, const uint8_t *dC, double M2, int32_t S, dtab *H) {
  int64_t n = G->n;
  int64_t m = n ? n : 1;
  int32_t *sz = (int32_t *)calloc((size_t)m, sizeof(int32_t));
  int32_t *prop = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  double *gp = (double *)malloc((size_t)m * sizeof(double));
  uint8_t *acc = (uint8_t *)malloc((size_t)m);
  for (int64_t i = 0; i < n; i++) sz[C[i]]++;
  for (int32_t s = 0; s < S; s++) {
    for (int64_t i = 0; i < n; i++) {
      prop[i] = -1;
      if (slice_of(i, S) != s) continue;
      if (!dC[CB[i]]) continue;
      if (C[i] != (int32_t)i || sz[i] != 1) continue;
      dtab_clear(H);
      for (int64_t e = G->off[i]; e < G->off[i + 1]; e++) {
        int32_t j = G->idx[e];
        if (j == (int32_t)i) continue;
        if (CB[j] != CB[i]) continue;
        dtab_add(H, C[j], (double)G->w[e]);
      }
      double g;
      prop[i] = best_community(H, (int32_t)i, M2, K[i], Sig, NULL, -1, &g);
      gp[i] = g;
    }
    for (int64_t i = 0; i < n; i++) {
      int32_t c = prop[i];
      acc[i] = 0;
      if (c < 0) continue;
      if (prop[c] < 0) acc[i] = 1;
      else if (prop[c] == (int32_t)i && (gp[i] > gp[c] || (gp[i] == gp[c] && (int32_t)i < c))) acc[i] = 1;
    }
    for (int64_t i = 0; i < n; i++) {
      if (!acc[i]) continue;
      int32_t c = prop[i];
      C[i] = c;
      Sig[i] -= K[i];
      Sig[c] += K[i];
      sz[i]--;
      sz[c]++;
    }
  }
  free(sz); free(prop); free(gp); free(acc);
  return 1;
}

/* "Renumber communities" of Alg. "leiden": dense labels in ascending order  */
/* of the old label.  Returns the number of communities.                     */
static int64_t renumber_dense(int64_t n, int32_t *C, int32_t *map) {
  for (int64_t c = 0; c < n; c++) map[c] = 0;
  for (int64_t i = 0; i < n; i++) map[C[i]] = 1;
  int64_t k = 0;
  for (int64_t c = 0; c < n; c++) {
    if (map[c]) map[c] = (int32_t)(k++);
    else map[c] = -1;
  }
  for (int64_t i = 0; i < n; i++) C[i] = map[C[i]];
  return k;
}

/* ------------------------------------------------------------------------ */
/* Alg. "leidenAggregate": super-vertex graph.  Row c lists, for every       */
/* community d adjacent to a member of c (self entries included,             */
/* "scanCommunities" with self=true), the FP64 sum of the weights, rounded   */
/* to float32.  Canonical form: rows compacted and ascending by d.           */
/* C must hold dense labels in [0, ncomm).                                    */
/* ------------------------------------------------------------------------ */
static int aggregate(const lgraph *G, const int32_t *C, int64_t ncomm, lgraph *out) {
  int64_t n = G->n;
  int64_t *coff = (int64_t *)calloc((size_t)(ncomm + 1), sizeof(int64_t));
  int32_t *mem = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  int64_t *fill = (int64_t *)malloc((size_t)(ncomm + 1) * sizeof(int64_t));
  out->n = ncomm;
  out->off = (int64_t *)calloc((size_t)(ncomm + 1), sizeof(int64_t));
  out->idx = (int32_t *)malloc((size_t)(G->nnz ? G->nnz : 1) * sizeof(int32_t));
  out->w = (float *)malloc((size_t)(G->nnz ? G->nnz : 1) * sizeof(float));
  out->owned = 1;
  dtab H;
  if (!coff || !mem || !fill || !out->off || !out->idx || !out->w || dtab_init(&H, ncomm) != OR_OK)
    return OR_ENOMEM;
  /* community-vertex CSR: count, exclusive scan, place (ascending ids) */
  for (int64_t i = 0; i < n; i++) coff[C[i] + 1]++;
  for (int64_t c = 0; c < ncomm; c++) coff[c + 1] += coff[c];
  for (int64_t c = 0; c <= ncomm; c++) fill[c] = coff[c];
  for (int64_t i = 0; i < n; i++) mem[fill[C[i]]++] = (int32_t)i;
  int64_t pos = 0;
  for (int64_t c = 0; c < ncomm; c++) {
    dtab_clear(&H);
    for (int64_t k = coff[c]; k < coff[c + 1]; k++) {
      int32_t i = mem[k];
      for (int64_t e = G->off[i]; e < G->off[i + 1]; e++)
        dtab_add(&H, C[G->idx[e]], (double)G->w[e]);
    }
    qsort(H.keys, (size_t)H.nkeys, sizeof(int32_t), cmp_i32);
    for (int64_t k = 0; k < H.nkeys; k++) {
      out->idx[pos] = H.keys[k];
      out->w[pos] = (float)H.val[H.keys[k]];
      pos++;
    }
    out->off[c + 1] = pos;
  }
  out->nnz = pos;
  dtab_free(&H);
  free(coff); free(mem); free(fill);
  return OR_OK;
}

static void row_sums(const lgraph *G, double *K) {
  for (int64_t i = 0; i < G->n; i++) {
    double s = 0.0;
    for (int64_t e = G->off[i]; e < G->off[i + 1]; e++) s += (double)G->w[e];
    K[i] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* Alg. "leiden" (dynamic-supporting Leiden): the pass loop.                  */
/* Inputs: the level-0 graph, the previous membership C_prev (labels in       */
/* [0,n)), K and Sigma for that membership, M2, the affected flags dV         */
/* (isAffected), the range flags (inAffectedRange, first pass only), the      */
/* changed-community flags dC0 and whether migrations are tracked.            */
/* Output: dense community labels in ascending order of the final label.     */
/* ------------------------------------------------------------------------ */
int or_core(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
            const int32_t *C_prev, const double *K, const double *Sig, double M2,
            const uint8_t *dV, const uint8_t *in_range, const uint8_t *dC0, int32_t track,
            const or_params *p, int32_t *C_out, or_stats *st) {
  or_stats st_local;
  if (!st) st = &st_local;
  memset(st, 0, sizeof(*st));
  if (n == 0) return OR_OK;
  lgraph G = {n, off[n], (int64_t *)off, (int32_t *)idx, (float *)w, 0};
  int32_t *Ctop = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *C = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *CB = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *tmpi = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  double *Kl = (double *)malloc((size_t)n * sizeof(double));
  double *Sl = (double *)malloc((size_t)n * sizeof(double));
  double *tmpd = (double *)malloc((size_t)n * sizeof(double));
  uint8_t *dC = (uint8_t *)malloc((size_t)n);
  uint8_t *U = (uint8_t *)malloc((size_t)n);
  uint8_t *ones = (uint8_t *)malloc((size_t)n);
  uint8_t *tmpb = (uint8_t *)malloc((size_t)n);
  dtab H;
  if (!Ctop || !C || !CB || !tmpi || !Kl || !Sl || !tmpd || !dC || !U || !ones || !tmpb ||
      dtab_init(&H, n) != OR_OK)
    return OR_ENOMEM;
  for (int64_t i = 0; i < n; i++) Ctop[i] = (int32_t)i;
  memcpy(C, C_prev, (size_t)n * sizeof(int32_t));
  memcpy(Kl, K, (size_t)n * sizeof(double));
  memcpy(Sl, Sig, (size_t)n * sizeof(double));
  memcpy(dC, dC0, (size_t)n);
  memcpy(U, dV, (size_t)n);
  memset(ones, 1, (size_t)n);
  for (int64_t i = 0; i < n; i++) st->affected += dV[i] ? 1 : 0;
  if (p->refine_variant == 1) { memset(dC, 1, (size_t)n); track = 0; }
  double tau = p->tau0;
  const int32_t S = p->nslices > 0 ? p->nslices : 1;
  int32_t pass;
  for (pass = 0; pass < p->max_passes; pass++) {
    int64_t nl = G.n;
    const uint8_t *rng = (pass == 0) ? in_range : ones;
    double Tp = tau * M2 * M2 / 2.0;
    int64_t nm = 0;
    double gt = 0.0;
    int32_t li;
    if (p->sync_mode)
      li = move_sync(&G, C, Kl, Sl, dC, U, rng, track && pass == 0, M2, Tp, p->max_iter, S, &H, &nm, &gt);
    else
      li = move_async(&G, C, Kl, Sl, dC, U, rng, track && pass == 0, M2, Tp, p->max_iter, &H, &nm, &gt);
    if (pass == 0) {
      st->moves_pass0 = nm;
      for (int64_t c = 0; c < nl; c++) st->changed += dC[c] ? 1 : 0;
    }
    st->move_iters[pass] = li;
    st->level_vertices[pass] = nl;
    st->level_entries[pass] = G.nnz;
    subset_renumber(nl, C, Sl, dC, tmpi, tmpd, tmpb);
    memcpy(CB, C, (size_t)nl * sizeof(int32_t));
    for (int64_t i = 0; i < nl; i++) st->refined_vertices[pass] += dC[CB[i]] ? 1 : 0;
    break_changed(nl, C, Kl, Sl, dC);
    if (p->sync_mode)
      st->refine_rounds[pass] = refine_sync(&G, CB, C, Kl, Sl, dC, M2, S, &H);
    else
      st->refine_rounds[pass] = refine_async(&G, CB, C, Kl, Sl, dC, M2, &H);
    st->passes = pass + 1;
    if ((pass > 0 || p->refine_variant == 2) && li <= 1) {
      /* count communities for the statistics only */
      memset(tmpb, 0, (size_t)nl);
      int64_t k = 0;
      for (int64_t i = 0; i < nl; i++) if (!tmpb[C[i]]) { tmpb[C[i]] = 1; k++; }
      st->communities[pass] = k;
      break;
    }
    int64_t ncomm = renumber_dense(nl, C, tmpi);
    st->communities[pass] = ncomm;
    if (p->agg_tol < 1.0 && (double)ncomm / (double)nl > p->agg_tol) {
      /* aggregation would merge too little: stop; the final lookup below
         then maps through the renumbered labels */
      break;
    }
    for (int64_t i = 0; i < n; i++) Ctop[i] = C[Ctop[i]];
    lgraph G2;
    memset(&G2, 0, sizeof(G2));
    if (aggregate(&G, C, ncomm, &G2) != OR_OK) return OR_ENOMEM;
    lgraph_free(&G);
    G = G2;
    row_sums(&G, Kl);
    memcpy(Sl, Kl, (size_t)G.n * sizeof(double));
    memset(U, 1, (size_t)G.n);
    for (int64_t i = 0; i < G.n; i++) C[i] = (int32_t)i;
    memset(dC, 1, (size_t)G.n);
    tau = tau / p->tol_drop;
  }
  for (int64_t i = 0; i < n; i++) Ctop[i] = C[Ctop[i]];
  /* dense relabel in ascending order of the final label */
  renumber_dense(n, Ctop, tmpi);
  memcpy(C_out, Ctop, (size_t)n * sizeof(int32_t));
  lgraph_free(&G);
  dtab_free(&H);
  free(Ctop); free(C); free(CB); free(tmpi); free(Kl); free(Sl); free(tmpd);
  free(dC); free(U); free(ones); free(tmpb);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 (modularity).  sigma_c: sum of stored entries (i,j) with both ends  */
/* in c (an internal undirected edge counts twice, a self-loop once); S_c:   */
/* sum of K_i over members.  Summed over ascending c in FP64; 0 when m = 0.  */
/* ------------------------------------------------------------------------ */
int or_modularity(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
                  const int32_t *C, double *q_out) {
  double *sig = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *tot = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  if (!sig || !tot) return OR_ENOMEM;
  double M2 = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (C[i] < 0 || C[i] >= n) { free(sig); free(tot); return OR_EINVAL; }
    for (int64_t e = off[i]; e < off[i + 1]; e++) {
      double we = (double)w[e];
      M2 += we;
      tot[C[i]] += we;
      if (C[idx[e]] == C[i]) sig[C[i]] += we;
    }
  }
  double q = 0.0;
  if (M2 > 0.0) {
    for (int64_t c = 0; c < n; c++) {
      double a = tot[c] / M2;
      q += sig[c] / M2 - a * a;
    }
  }
  *q_out = q;
  free(sig); free(tot);
  return OR_OK;
}

int or_aggregate(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
                 const int32_t *C, int64_t ncomm, int64_t *out_off, int32_t *out_idx,
                 float *out_w, int64_t *nnz_out) {
  for (int64_t i = 0; i < n; i++)
    if (C[i] < 0 || C[i] >= ncomm) return OR_EINVAL;
  lgraph G = {n, off[n], (int64_t *)off, (int32_t *)idx, (float *)w, 0};
  lgraph O;
  memset(&O, 0, sizeof(O));
  int rc = aggregate(&G, C, ncomm, &O);
  if (rc != OR_OK) return rc;
  memcpy(out_off, O.off, (size_t)(ncomm + 1) * sizeof(int64_t));
  memcpy(out_idx, O.idx, (size_t)O.nnz * sizeof(int32_t));
  memcpy(out_w, O.w, (size_t)O.nnz * sizeof(float));
  *nnz_out = O.nnz;
  lgraph_free(&O);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Batch update (Sec. 3.5 and 5.1.4): edge deletions and insertions, each     */
/* undirected edge listed once; both directions are applied.  Validity:       */
/* ids in range, no self-loop, no duplicate, a deletion must exist in         */
/* G^{t-1}, an insertion must not, inserted weights finite and > 0.  The      */
/* weight of a deleted edge is taken from G^{t-1}.  Rows of the input must    */
/* be sorted by neighbour id; rows of the output are sorted.                 */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t u, v; float w; int32_t kind; } dentry; /* kind 0 del, 1 ins */

static int cmp_dentry(const void *a, const void *b) {
  const dentry *x = (const dentry *)a, *y = (const dentry *)b;
  if (x->u != y->u) return (x->u > y->u) - (x->u < y->u);
  return (x->v > y->v) - (x->v < y->v);
}

static int64_t find_in_row(const int64_t *off, const int32_t *idx, int32_t u, int32_t v) {
  int64_t lo = off[u], hi = off[u + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (idx[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return (lo < off[u + 1] && idx[lo] == v) ? lo : -1;
}

int or_apply_batch(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
                   int64_t nd, const int32_t *du, const int32_t *dv,
                   int64_t ni, const int32_t *iu, const int32_t *iv, const float *iw,
                   int64_t *out_off, int32_t *out_idx, float *out_w, float *del_w) {
  int64_t m = 2 * (nd + ni);
  dentry *E = (dentry *)malloc((size_t)(m ? m : 1) * sizeof(dentry));
  if (!E) return OR_ENOMEM;
  for (int64_t k = 0; k < nd; k++) {
    if (du[k] < 0 || du[k] >= n || dv[k] < 0 || dv[k] >= n || du[k] == dv[k]) { free(E); return OR_EINVAL; }
    int64_t e = find_in_row(off, idx, du[k], dv[k]);
    if (e < 0) { free(E); return OR_EINVAL; }
    del_w[k] = w[e];
    E[2 * k] = (dentry){du[k], dv[k], w[e], 0};
    E[2 * k + 1] = (dentry){dv[k], du[k], w[e], 0};
  }
  for (int64_t k = 0; k < ni; k++) {
    if (iu[k] < 0 || iu[k] >= n || iv[k] < 0 || iv[k] >= n || iu[k] == iv[k]) { free(E); return OR_EINVAL; }
    if (!(iw[k] > 0.0f) || !isfinite(iw[k])) { free(E); return OR_EINVAL; }
    if (find_in_row(off, idx, iu[k], iv[k]) >= 0) { free(E); return OR_EINVAL; }
    E[2 * (nd + k)] = (dentry){iu[k], iv[k], iw[k], 1};
    E[2 * (nd + k) + 1] = (dentry){iv[k], iu[k], iw[k], 1};
  }
  qsort(E, (size_t)m, sizeof(dentry), cmp_dentry);
  for (int64_t k = 1; k < m; k++)
    if (E[k].u == E[k - 1].u && E[k].v == E[k - 1].v) { free(E); return OR_EINVAL; }
  /* merge row by row */
  int64_t pos = 0, b = 0;
  out_off[0] = 0;
  for (int64_t u = 0; u < n; u++) {
    int64_t e = off[u], e1 = off[u + 1];
    while (e < e1 || (b < m && E[b].u == u)) {
      int has_b = (b < m && E[b].u == u);
      if (e < e1 && (!has_b || idx[e] < E[b].v)) {
        out_idx[pos] = idx[e]; out_w[pos] = w[e]; pos++; e++;
      } else if (e < e1 && has_b && idx[e] == E[b].v) {
        /* a deletion of this existing entry */
        e++; b++;
      } else {
        /* an insertion (validated absent from the row) */
        out_idx[pos] = E[b].v; out_w[pos] = E[b].w; pos++; b++;
      }
    }
    out_off[u + 1] = pos;
  }
  free(E);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Marking of affected vertices and changed communities.                      */
/*  DF: Alg. "dynamicFrontier" - a deletion inside a community or an          */
/*      insertion across communities marks its source (both directions, so    */
/*      both endpoints); the range is everything.                             */
/*  DS: Alg. "deltaScreening" - deletions inside a community mark the source, */
/*      its neighbours and the community; per unique insertion source, the    */
/*      inserted cross-community weights are summed per community and the     */
/*      community with the best Eq. 2 score (c-independent terms dropped,     */
/*      previous K, Sigma, M2) is marked with the source and its neighbours;  */
/*      then neighbours of marked sources and members of marked communities   */
/*      are marked; the range is the marked set.                              */
/*  ND: Alg. "naiveDynamic" - everything affected, everything in range.       */
/*  changedCommunities of Alg. "leiden": a community is changed when a batch  */
/*      edge lies inside it (flag keyed by the community id).                 */
/* G^t is the updated graph; C, K, Sigma, M2 are the previous values.         */
/* ------------------------------------------------------------------------ */
int or_mark(int32_t mode, int64_t n, const int64_t *off, const int32_t *idx,
            int64_t nd, const int32_t *du, const int32_t *dv,
            int64_t ni, const int32_t *iu, const int32_t *iv, const float *iw,
            const int32_t *C, const double *K, const double *Sig, double M2,
            uint8_t *dV, uint8_t *in_range, uint8_t *dC) {
  memset(dV, 0, (size_t)n);
  memset(dC, 0, (size_t)n);
  /* changedCommunities, both directions of deletions and insertions */
  for (int64_t k = 0; k < nd; k++)
    if (C[du[k]] == C[dv[k]]) dC[C[du[k]]] = 1;
  for (int64_t k = 0; k < ni; k++)
    if (C[iu[k]] == C[iv[k]]) dC[C[iu[k]]] = 1;
  if (mode == OR_MODE_ND) {
    memset(dV, 1, (size_t)n);
    memset(in_range, 1, (size_t)n);
    return OR_OK;
  }
  if (mode == OR_MODE_DF) {
    for (int64_t k = 0; k < nd; k++)
      if (C[du[k]] == C[dv[k]]) { dV[du[k]] = 1; dV[dv[k]] = 1; }
    for (int64_t k = 0; k < ni; k++)
      if (C[iu[k]] != C[iv[k]]) { dV[iu[k]] = 1; dV[iv[k]] = 1; }
    memset(in_range, 1, (size_t)n);
    return OR_OK;
  }
  if (mode != OR_MODE_DS) return OR_EINVAL;
  uint8_t *dE = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *dCm = (uint8_t *)calloc((size_t)n, 1);
  /* directed insertions grouped by source */
  int64_t m = 2 * ni;
  dentry *E = (dentry *)malloc((size_t)(m ? m : 1) * sizeof(dentry));
  dtab H;
  if (!dE || !dCm || !E || dtab_init(&H, n) != OR_OK) return OR_ENOMEM;
  for (int64_t k = 0; k < nd; k++) {
    int32_t a = du[k], b = dv[k];
    if (C[a] == C[b]) {
      dV[a] = 1; dE[a] = 1; dCm[C[b]] = 1;
      dV[b] = 1; dE[b] = 1; dCm[C[a]] = 1;
    }
  }
  for (int64_t k = 0; k < ni; k++) {
    E[2 * k] = (dentry){iu[k], iv[k], iw[k], 1};
    E[2 * k + 1] = (dentry){iv[k], iu[k], iw[k], 1};
  }
  qsort(E, (size_t)m, sizeof(dentry), cmp_dentry);
  for (int64_t k = 0; k < m;) {
    int32_t i = E[k].u;
    int64_t k1 = k;
    dtab_clear(&H);
    while (k1 < m && E[k1].u == i) {
      if (C[i] != C[E[k1].v]) dtab_add(&H, C[E[k1].v], (double)E[k1].w);
      k1++;
    }
    if (H.nkeys > 0) {
      int32_t best = -1;
      double bestg = 0.0;
      for (int64_t t = 0; t < H.nkeys; t++) {
        int32_t c = H.keys[t];
        double g = (M2 * H.val[c]) - (K[i] * Sig[c]);
        if (best < 0 || g > bestg || (g == bestg && c < best)) { best = c; bestg = g; }
      }
      dV[i] = 1; dE[i] = 1; dCm[best] = 1;
    }
    k = k1;
  }
  for (int64_t i = 0; i < n; i++) {
    if (dE[i])
      for (int64_t e = off[i]; e < off[i + 1]; e++) dV[idx[e]] = 1;
  }
  for (int64_t i = 0; i < n; i++)
    if (dCm[C[i]]) dV[i] = 1;
  memcpy(in_range, dV, (size_t)n);
  dtab_free(&H);
  free(dE); free(dCm); free(E);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. "updateWeights": K and Sigma of the previous membership adjusted by  */
/* every directed batch entry; M2 tracked the same way (Sec. 5.1.5).          */
/* ------------------------------------------------------------------------ */
void or_update_weights(int64_t nd, const int32_t *du, const int32_t *dv, const float *dw,
                       int64_t ni, const int32_t *iu, const int32_t *iv, const float *iw,
                       const int32_t *C, double *K, double *Sig, double *M2) {
  double m2 = *M2;
  for (int64_t k = 0; k < nd; k++) {
    double x = (double)dw[k];
    K[du[k]] -= x; Sig[C[du[k]]] -= x;
    K[dv[k]] -= x; Sig[C[dv[k]]] -= x;
    m2 -= 2.0 * x;
  }
  for (int64_t k = 0; k < ni; k++) {
    double x = (double)iw[k];
    K[iu[k]] += x; Sig[C[iu[k]]] += x;
    K[iv[k]] += x; Sig[C[iv[k]]] += x;
    m2 += 2.0 * x;
  }
  *M2 = m2;
}

/* Static Leiden: singleton start, everything affected and changed, no      */
/* tracking (Alg. "leiden" with changedCommunities returning all).           */
int or_static(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
              const or_params *p, int32_t *C_out, double *K_out, double *Sig_out,
              double *M2_out, or_stats *st) {
  if (n == 0) { *M2_out = 0.0; return OR_OK; }
  int32_t *C0 = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  uint8_t *ones = (uint8_t *)malloc((size_t)n);
  if (!C0 || !ones) return OR_ENOMEM;
  lgraph G = {n, off[n], (int64_t *)off, (int32_t *)idx, (float *)w, 0};
  row_sums(&G, K_out);
  double m2 = 0.0;
  for (int64_t i = 0; i < n; i++) { C0[i] = (int32_t)i; m2 += K_out[i]; }
  memset(ones, 1, (size_t)n);
  int rc = or_core(n, off, idx, w, C0, K_out, K_out, m2, ones, ones, ones, 0, p, C_out, st);
  if (rc == OR_OK) {
    for (int64_t c = 0; c < n; c++) Sig_out[c] = 0.0;
    for (int64_t i = 0; i < n; i++) Sig_out[C_out[i]] += K_out[i];
  }
  *M2_out = m2;
  free(C0); free(ones);
  return rc;
}

/* Dynamic update on an already-updated graph G^t: marking, changed         */
/* communities, updateWeights, the pass loop, then Sigma^t recomputed for    */
/* the new membership (the paper returns the updateWeights value; the next   */
/* update needs the totals of C^t).                                          */
int or_update(int32_t mode, int64_t n, const int64_t *off, const int32_t *idx, const float *w,
              int64_t nd, const int32_t *du, const int32_t *dv, const float *dw,
              int64_t ni, const int32_t *iu, const int32_t *iv, const float *iw,
              const int32_t *C_prev, double *K, double *Sig, double *M2,
              const or_params *p, int32_t *C_out, uint8_t *dV_out, uint8_t *dC_out, or_stats *st) {
  if (mode != OR_MODE_ND && mode != OR_MODE_DS && mode != OR_MODE_DF) return OR_EINVAL;
  if (n == 0) return OR_OK;
  uint8_t *rng = (uint8_t *)malloc((size_t)n);
  if (!rng) return OR_ENOMEM;
  int rc = or_mark(mode, n, off, idx, nd, du, dv, ni, iu, iv, iw, C_prev, K, Sig, *M2, dV_out, rng, dC_out);
  if (rc != OR_OK) { free(rng); return rc; }
  or_update_weights(nd, du, dv, dw, ni, iu, iv, iw, C_prev, K, Sig, M2);
  rc = or_core(n, off, idx, w, C_prev, K, Sig, *M2, dV_out, rng, dC_out, 1, p, C_out, st);
  if (rc == OR_OK) {
    for (int64_t c = 0; c < n; c++) Sig[c] = 0.0;
    for (int64_t i = 0; i < n; i++) Sig[C_out[i]] += K[i];
  }
  free(rng);
  return rc;
}

/* Single local-moving decision for vertex i (the body of Alg. "leidenMove"  */
/* for one vertex): table of neighbour-community weights without i's own     */
/* self-loop, best community by Eq. 2.  Exposed so the score can be pinned    */
/* against exact modularity differences.  Returns the target or -1.          */
int32_t or_best_move(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
                     const int32_t *C, const double *K, const double *Sig, double M2,
                     int32_t i, double *g_out) {
  dtab H;
  if (dtab_init(&H, n) != OR_OK) return -2;
  for (int64_t e = off[i]; e < off[i + 1]; e++) {
    if (idx[e] == i) continue;
    dtab_add(&H, C[idx[e]], (double)w[e]);
  }
  int32_t c = best_community(&H, C[i], M2, K[i], Sig, NULL, -1, g_out);
  dtab_free(&H);
  return c;
}

/* One local-moving phase (Alg. "leidenMove") on a given graph and state,     */
/* exposed so its bookkeeping can be pinned directly.  Returns the number of */
/* iterations; *gain_out receives the total gain of the moves in units of     */
/* 2m^2 (the sum of the per-move scores).                                     */
int32_t or_move_phase(int64_t n, const int64_t *off, const int32_t *idx, const float *w,
                      int32_t *C, const double *K, double *Sig, uint8_t *dC, uint8_t *U,
                      const uint8_t *rng, int32_t track, double M2, double tau, int32_t max_iter,
                      int32_t sync_mode, int64_t *nmoves, double *gain_out) {
  lgraph G = {n, off[n], (int64_t *)off, (int32_t *)idx, (float *)w, 0};
  dtab H;
  if (dtab_init(&H, n) != OR_OK) return -1;
  double Tp = tau * M2 * M2 / 2.0;
  *gain_out = 0.0;
  int32_t l = sync_mode ? move_sync(&G, C, K, Sig, dC, U, rng, track, M2, Tp, max_iter, sync_mode, &H, nmoves, gain_out)
                        : move_async(&G, C, K, Sig, dC, U, rng, track, M2, Tp, max_iter, &H, nmoves, gain_out);
  dtab_free(&H);
  return l;
}

/* Alg. "leidenSubsetRenumber" exposed for a direct pin. */
void or_subset_renumber(int64_t n, int32_t *C, double *Sig, uint8_t *dC) {
  int32_t *rep = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  double *S2 = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
  uint8_t *d2 = (uint8_t *)malloc((size_t)(n ? n : 1));
  subset_renumber(n, C, Sig, dC, rep, S2, d2);
  free(rep); free(S2); free(d2);
}
