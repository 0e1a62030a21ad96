// Host-side launchers of the library's HIP kernels (one translation unit per
// phase).  Every launcher enqueues on `s` and returns without synchronising;
// the driver checks hipGetLastError after each phase.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace lk {

constexpr int kNB = 6;        // degree buckets: <=4, <=8, <=32, <=256, <=2048, >2048

// Slice of a vertex in a sweep: MurmurHash3's 32-bit finaliser of the id,
// modulo the number of slices.
__host__ __device__ inline int slice_of(int64_t i, int S) {
  uint32_t h = (uint32_t)i;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return (int)(h % (uint32_t)S);
}
constexpr int kChunk = 1024;  // CSR positions per chunk in chunked edge kernels

inline int bucket_of_host(int64_t deg) {
  return deg <= 4 ? 0 : deg <= 8 ? 1 : deg <= 32 ? 2 : deg <= 256 ? 3 : deg <= 2048 ? 4 : 5;
}
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int flat_grid(int64_t n, int block = 256, int cap = 4096) {
  int64_t g = ceil_div(n > 0 ? n : 1, block);
  return (int)(g < cap ? g : cap);
}

// ---- k_util.hip ------------------------------------------------------------
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void fill_f64(double *p, double v, int64_t n, hipStream_t s);
void fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);
// out[b] = row owning position b*kChunk (b < nchunks); out[nchunks] = nrows-1.
void chunk_start_rows(const int64_t *off, int64_t nrows, int64_t nnz, int32_t *out, hipStream_t s);
// K[r] = sum of w over row r (FP64); K must be zeroed.
void row_sums(const int64_t *off, const float *w, int64_t nrows, int64_t nnz, const int32_t *crow,
              double *K, hipStream_t s);
// out[C[i]] += v[i] (out zeroed by the caller).
void scatter_add(const double *v, const int32_t *C, int64_t n, double *out, hipStream_t s);
// C[i] = map[C[i]]
void gather_map(int32_t *C, const int32_t *map, int64_t n, hipStream_t s);
// C[i] = map[C[i]] where C[i] < bound; larger labels are left as they are
void gather_map_bounded(int32_t *C, const int32_t *map, int64_t n, int64_t bound, hipStream_t s);
// flags of the labels in use (used) and of those with a member with edges (act)
void mark_used_active(const int32_t *C, const int64_t *off, int64_t n, int32_t *used, int32_t *act, hipStream_t s);
// used[c] = used[c] && !act[c] (in place), for c < n
void flags_inactive(int32_t *used, const int32_t *act, int64_t n, hipStream_t s);
// map[c] = act[c] ? pa[c] : na + pi[c], for c < n
void active_first_map(const int32_t *act, const int32_t *pa, const int32_t *pi, int64_t na, int64_t n, int32_t *map,
                      hipStream_t s);
// flags[C[i]] = 1
void mark_used(const int32_t *C, int64_t n, int32_t *flags, hipStream_t s);
// C[i] < bound for all i?  sets *err |= flag otherwise.
void check_labels(const int32_t *C, int64_t n, int64_t bound, int32_t *err, hipStream_t s);
// Rows strictly ascending (sorted, no duplicate entry), ids in range, weights
// finite and > 0?  Sets *err |= 1 otherwise.  crow: chunk_start_rows of off.
void check_rows_chunked(const int64_t *off, const int32_t *idx, const float *w, int64_t n, int64_t nnz,
                        const int32_t *crow, int32_t *err, hipStream_t s);
void check_offsets(const int64_t *off, int64_t n, int64_t nnz, int32_t *err, hipStream_t s);

// ---- k_prim.hip: scans and radix sort (temp == nullptr returns the temp size) ----
size_t scan_excl_i32(void *temp, size_t tbytes, const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
size_t scan_excl_i64(void *temp, size_t tbytes, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
size_t scan_excl_i32_to_i64(void *temp, size_t tbytes, const int32_t *in, int64_t *out, int64_t n,
                            hipStream_t s);
void reset_iter(int32_t *counts, int n, double *d0, unsigned long long *u0, unsigned long long *u1,
                hipStream_t s);
size_t sort_pairs_u64_i32(void *temp, size_t tbytes, const unsigned long long *kin,
                          unsigned long long *kout, const int32_t *vin, int32_t *vout, int64_t n,
                          hipStream_t s);
size_t sort_pairs_u64_f64(void *temp, size_t tbytes, const unsigned long long *kin,
                          unsigned long long *kout, const double *vin, double *vout, int64_t n,
                          hipStream_t s);
size_t seg_sort_i32_f32(void *temp, size_t tbytes, const int32_t *kin, int32_t *kout,
                        const float *vin, float *vout, int64_t nnz, int64_t nseg,
                        const int64_t *off, hipStream_t s);

constexpr int kPT = 256;                  // threads of a primitive workgroup
constexpr int kPR = 16;                   // rounds of kPT items per tile
constexpr int64_t kPTile = kPT * kPR;     // items per tile

// Segments of a radix sort: tiles of kPTile items that never cross a segment.
// With tseg == nullptr there is one segment, items [0, n).
struct RsSeg {
  int64_t ntiles;
  int64_t n;
  const int32_t *tseg;    // [ntiles] segment of each tile
  const int64_t *tfirst;  // [nseg + 1] first tile of each segment
  const int64_t *sbeg;    // [nseg] first item of each segment
  const int64_t *send;    // [nseg] end of each segment
};
struct TileSpan {
  int64_t f0, nt;  // first tile and tile count of the tile's segment
  int64_t lo, hi;  // the tile's items
  int64_t sb;      // first item of the segment
};
__device__ __forceinline__ TileSpan tile_span(const RsSeg &g, int64_t t) {
  TileSpan r;
  if (!g.tseg) {
    r.f0 = 0;
    r.nt = g.ntiles;
    r.sb = 0;
    r.lo = t * kPTile;
    r.hi = r.lo + kPTile < g.n ? r.lo + kPTile : g.n;
    return r;
  }
  const int s = g.tseg[t];
  r.f0 = g.tfirst[s];
  r.nt = g.tfirst[s + 1] - r.f0;
  r.sb = g.sbeg[s];
  r.lo = r.sb + (t - r.f0) * kPTile;
  r.hi = r.lo + kPTile < g.send[s] ? r.lo + kPTile : g.send[s];
  return r;
}
RsSeg rs_plain(int64_t n);
int rs_passes(int bits);
size_t rs_tmp_bytes(int64_t ntiles);
int key_bits(unsigned long long x);  // bits needed for x (0 for 0)
// Stable sort of every segment by the low `bits` key bits (rs_passes(bits)
// passes); (k1, v1) are second buffers covering the same items.  Returns 0 if
// the result is in (k0, v0), 1 if in (k1, v1) (odd pass count).  tmp:
// rs_tmp_bytes(g.ntiles) bytes.
template <class K, class V>
int rsort(K *k0, V *v0, K *k1, V *v1, const RsSeg &g, int bits, void *tmp, hipStream_t s);

// ---- k_move.hip -------------------------------------------------------------
// Hub plan of a level: the vertices of the largest degree bucket grouped by
// slice, each split into edge chunks (one gather workgroup each) and owning
// a global open-addressing table split into scoring segments.
constexpr int64_t kHubDeg = 2048;  // degree above which a vertex is a hub
constexpr int kHubEC = 512;        // edges per gather workgroup
constexpr int kHubSeg = 4096;      // table slots per scoring workgroup
constexpr int64_t kHubMinCap = 256; // smallest hub table (a power of two)
struct HubPlan {
  int32_t *hubv;   // [nhub] hub ids, slice-major
  int64_t *hch;    // [nhub+1] first edge chunk of each hub
  int64_t *htab;   // [nhub] first table slot, counted from the start of the hub's slice
  int64_t *hcap;   // [nhub] table slots (a power of two, at least 2 * degree)
  int64_t *hsg;    // [nhub+1] first table segment
  int32_t *chub;   // hub index of each chunk
  int32_t *shub;   // hub index of each segment
  int *keys;       // tables of one slice (shared by the slices), kEmpty when free;
                   // scoring leaves them free again
  double *vals;
  double *own;     // [nhub] weight to the hub's own community (zero between uses)
  double *pg;      // per-segment best gain
  int32_t *pc;     // per-segment best community
  int32_t *flag;   // [nhub] 1 when the hub's move is blocked (reset by the final reduction)
};

struct MoveArgs {
  // level graph
  int64_t n;
  const int64_t *off;
  const int32_t *idx;
  const float *w;
  // state
  int32_t *C;
  const double *K;
  double *Sig;
  uint8_t *dC;
  uint8_t *U;
  const uint8_t *rng;
  double M2;
  int track;
  // work
  int32_t *prop;
  int32_t *from;
  double *gp;
  double *gi;            // per-vertex accepted gain (synchronous sums), nullable
  int32_t *lists;        // frontier, bucketed by (slice, degree bucket)
  const int32_t *region; // device: region starts [S*kNB+1], index s*kNB+b
  int32_t *counts;       // device: frontier counts [S*kNB]
  int nsl;               // slices per sweep
  int s;                 // current slice
  const int32_t *vbyslice;  // vertices grouped by slice
  int64_t vbeg, vend;    // range of the current slice in vbyslice
  double *gain;          // device scalar (atomic sums), nullable when gi is used
  unsigned long long *moves;  // device scalar
  // multi-workgroup hub path
  HubPlan hp;
  uint8_t *act;          // hub is in the frontier of its slice
  int hub_front;         // the hub gather writes act itself (asynchronous mode)
  int64_t hbeg, hend;    // hubs of the current slice
  int64_t qbeg, qend;    // their edge chunks
  int64_t gbeg, gend;    // their table segments
  unsigned long long *hub_scanned;  // nullable: edges scanned by the hub gather
  unsigned long long *sweep_work;   // nullable: [vertices evaluated, edges scanned] by the async sweep
  // asynchronous sweep
  unsigned long long *anext;  // device counter: next list position (zeroed per sweep)
  const int32_t *alist;       // vertices with edges, ascending
  int64_t alen;
  int *akeys;                 // per-wavefront global tables, 2*kHubDeg slots each
  double *avals;
  int64_t hubdeg;             // degree above which a vertex takes the hub path (<= kHubDeg)
  int32_t cached;             // asynchronous sweep: cache-served reads of C and Sigma (large levels)
  int32_t defer;              // asynchronous sweep: batch the Sigma updates of popular communities
};
// Per level: counts[s*kNB+b] of vertices with edges, slice sizes, and the
// vertex-by-slice grouping (slice_fill zeroed, slice_off = starts of slices).
// Vertices of degree > hubdeg (<= kHubDeg) go to the last (hub) bucket.
void slice_hist(const int64_t *off, int64_t n, int S, int64_t hubdeg, int32_t *counts, int32_t *slice_cnt,
                hipStream_t s);
void slice_scatter(int64_t n, int S, const int32_t *slice_off, int32_t *slice_fill, int32_t *vbyslice,
                   hipStream_t s);
// Hub plan construction (per level): hubs of each slice placed at
// slice_off[s] + fill; per-hub chunk / slot / segment counts (to be scanned
// into hch, htab, hsg); expansion into chub / shub; bounds[k] = arr[at[k]].
void hub_find(const int64_t *off, int64_t n, int S, int64_t hubdeg, const int32_t *hub_soff, int32_t *hub_fill,
              int32_t *hubv, hipStream_t s);
void hub_sizes(const int64_t *off, const int32_t *hubv, int64_t nhub, int64_t *nch, int64_t *ncap, int64_t *nseg,
               hipStream_t s);
void hub_expand(const HubPlan &h, int64_t nhub, hipStream_t s);
void hub_rel(int64_t *htab, int64_t nhub, const int32_t *hub_soff, int S, const int64_t *slice_base, hipStream_t s);
void gather_bounds(const int64_t *arr, const int32_t *at, int count, int64_t *out, hipStream_t s);
// region_h: host copy of the region starts of this level.
void move_frontier(const MoveArgs &a, hipStream_t s);
void move_propose(const MoveArgs &a, const int64_t *region_h, hipStream_t s);
void move_propose_bucket(const MoveArgs &a, const int64_t *region_h, int b, hipStream_t s);
void move_apply_bucket(const MoveArgs &a, const int64_t *region_h, int b, hipStream_t s);
// the two halves of bucket kNB-1 (hubs): chunk gather, then segment scoring + final argmax
void move_hub_gather(const MoveArgs &a, hipStream_t s);
void move_hub_score(const MoveArgs &a, hipStream_t s);
void move_apply(const MoveArgs &a, const int64_t *region_h, hipStream_t s);
// out = sum of gi in ascending 256-tiles then sequentially (fixed order).
void tiled_sum(const double *gi, int64_t n, double *tiles, double *out, hipStream_t s);

// ---- k_refine.hip -------------------------------------------------------------
void subset_renumber(int64_t n, int32_t *C, int32_t *rep, const double *Sig, double *Sig2,
                     const uint8_t *dC, uint8_t *dC2, hipStream_t s);
struct RefineArgs {
  int64_t n;
  const int64_t *off;
  const int32_t *idx;
  const float *w;
  int32_t *C;
  int32_t *CB;
  unsigned long long *CP;   // asynchronous sweep: CB << 32 | C per vertex, kept with C
  int32_t cached;           // asynchronous sweep: cache-served reads (large levels)
  int32_t defer;            // asynchronous sweep: batch the joins of popular communities
  unsigned long long *sweep_work;  // nullable: [candidates evaluated, edges scanned] by the async sweep
  const double *K;
  double *Sig;
  const uint8_t *dC;
  int32_t *S;
  double M2;
  int32_t *prop;
  double *gp;
  int32_t *lists;
  const int32_t *region;    // [S*kNB+1]
  int32_t *counts;          // [S*kNB]
  int nsl;
  int s;
  unsigned long long *refined;  // device scalar: vertices in changed bounds
  // asynchronous sweep
  unsigned long long *anext;
  const int32_t *alist;
  int64_t alen;
  int *akeys;
  double *avals;
  // multi-workgroup path for hub candidates (as in MoveArgs)
  HubPlan hp;
  uint8_t *act;
  int64_t hbeg, hend, qbeg, qend, gbeg, gend;
  int64_t hubdeg;
};
void refine_break(const RefineArgs &a, hipStream_t s);
void refine_propose_bucket(const RefineArgs &a, const int64_t *region_h, int b, hipStream_t s);
void refine_propose(const RefineArgs &a, const int64_t *region_h, hipStream_t s);
void refine_accept(const RefineArgs &a, const int64_t *region_h, hipStream_t s);

// ---- k_async.hip ---------------------------------------------------------------
constexpr int kAsyncChunk = 64;  // vertex ids taken per grab of the asynchronous sweeps
// `waves` wavefronts sweep the list; vertices of degree <= a.hubdeg only.
// Tables: LDS, else 2*kHubDeg slots per wavefront in akeys/avals; `wide`
// selects larger LDS tables (for levels of high average degree).
void move_async(const MoveArgs &a, int waves, bool wide, hipStream_t s);
// list of vertices with edges in ascending order: flags then scan then scatter
void edge_flags(const int64_t *off, int64_t n, int32_t *flags, hipStream_t s);
void edge_list(const int64_t *off, int64_t n, const int32_t *pos, int32_t *list, hipStream_t s);
void refine_async(const RefineArgs &a, int waves, bool wide, hipStream_t s);
void pack_cb(const int32_t *C, const int32_t *CB, int64_t n, unsigned long long *CP, hipStream_t s);
// hub frontier of slice a.s (a.hbeg..a.hend of the hub plan) for the hub-only sliced phase

// ---- k_aggregate.hip -----------------------------------------------------------
struct AggArgs {
  int64_t n, nnz, ncomm;
  const int64_t *off;
  const int32_t *idx;
  const float *w;
  const int32_t *C;
};
constexpr int kAggSmall = 1024;  // segments up to this many entries are sorted by one wavefront
void agg_vkeys(int64_t n, const int32_t *C, uint32_t *keys, int32_t *vals, hipStream_t s);
void agg_vdeg(int64_t n, const int64_t *off, const int32_t *vs, int64_t *deg, int32_t *pos, hipStream_t s);
void agg_cdeg(int64_t n, const uint32_t *Cs, const int64_t *eoff, int64_t *hpos, int64_t *cdeg, hipStream_t s);
void agg_group(const AggArgs &a, const int32_t *crow, const int32_t *pos, const int64_t *eoff, uint32_t *gkey,
               float *gval, hipStream_t s);
// u64 / l64 / v64 (nullable): the rows' weights also as the FP64 run sums
// before rounding, at the same positions.
void agg_small(const int64_t *seg, int64_t ncomm, const uint32_t *gkey, const float *gval, uint32_t *ukey,
               float *uval, double *u64, int32_t *rowlen, double *K, hipStream_t s);
void agg_large_flags(const int64_t *seg, int64_t ncomm, int32_t *flag, hipStream_t s);
void agg_large_list(const int64_t *seg, int64_t ncomm, int32_t *flag, const int32_t *lidx, int32_t *lc, int64_t *lsb,
                    int64_t *lse, int64_t *ltn, hipStream_t s);
void agg_tile_seg(const int64_t *tfirst, int64_t nl, int64_t ntl, int32_t *tseg, hipStream_t s);
void agg_large_runs(int pass, const uint32_t *gkey, const float *gval, const RsSeg &g, int64_t *hc, double *tin,
                    uint32_t *ukey, float *uval, double *l64, double *tks, hipStream_t s);
void agg_large_rows(int64_t nl, const int32_t *lc, const int64_t *tfirst, const int64_t *hc, const double *tks,
                    int32_t *rowlen, double *K, hipStream_t s);
// rows of the small segments from (ukey, uval), of the large ones from (lkey, lval)
void agg_compact(const int64_t *seg, int64_t ncomm, const int32_t *lc, const int64_t *lsb, const int32_t *tseg,
                 const int64_t *tfirst, int64_t ntl, const int32_t *rowlen, const int64_t *out_off, const uint32_t *ukey, const float *uval,
                 const uint32_t *lkey, const float *lval, const double *v64, int32_t *out_idx, float *out_w,
                 double *out_w64, hipStream_t s);

// ---- k_modularity.hip --------------------------------------------------------
// acc[0] += sigma total, S[c] += K-contributions (S zeroed, ncomm = n)
void modularity_edges(const int64_t *off, const int32_t *idx, const float *w, const int32_t *crow,
                      int64_t n, int64_t nnz, const int32_t *C, double *acc, double *S,
                      hipStream_t s);
// acc[0] += weight of the entries inside a community (Sigma and 2m known elsewhere)
void modularity_intra(const int64_t *off, const int32_t *idx, const float *w, const int32_t *crow, int64_t nnz,
                      const int32_t *C, double *acc, hipStream_t s);
void modularity_intra64(const int64_t *off, const int32_t *idx, const double *w, const int32_t *crow, int64_t nnz,
                        const int32_t *C, double *acc, hipStream_t s);
// out[to[v]] = val[v] for v < n (every writer of one target writes the same value)
void scatter_labels(const int32_t *to, const int32_t *val, int64_t n, int32_t *out, hipStream_t s);
// acc[1] += sum_c S_c, acc[2] += sum_c (S_c)^2 scaled: computed as sum (S_c/M2)^2 after M2 known
void modularity_comm(const double *S, int64_t n, double *acc, hipStream_t s);
void modularity_comm_sq(const double *S, int64_t n, double M2, double *acc, hipStream_t s);

// ---- k_batch.hip ---------------------------------------------------------------
struct BatchArgs {
  int64_t n, nnz;
  const int64_t *off;
  const int32_t *idx;
  const float *w;
  int64_t nd, ni;
  const int32_t *du, *dv, *iu, *iv;
  const float *iw;
  int64_t E;                      // 2*(nd+ni)
  unsigned long long *keys;       // E
  int32_t *vals;                  // E
  unsigned long long *skeys;      // E
  int32_t *svals;                 // E
  float *ew;                      // E, weight of directed entry (by entry id)
  int32_t *err;                   // device scalar
  int64_t *bstart;                // n (segment start in sorted order, -1 none)
  int32_t *bcnt;                  // n
  int32_t *dcnt;                  // n deletions per row
  int32_t *icnt;                  // n insertions per row
  int32_t *isdel;                 // E+1
  int32_t *delpre;                // E+1
  int64_t *newdeg;                // n+1
  int64_t *newoff;                // n+1
  const int32_t *crow;            // chunk starts of the old graph
  int32_t *nidx;
  float *nw;
};
void batch_build(const BatchArgs &a, hipStream_t s);
void batch_dups_rows(const BatchArgs &a, hipStream_t s);  // dup check + per-row counts/segments
void batch_newdeg(const BatchArgs &a, hipStream_t s);
void batch_apply_old(const BatchArgs &a, hipStream_t s);  // surviving old entries, merge positions
void batch_apply_ins(const BatchArgs &a, hipStream_t s);  // inserted entries

struct MarkArgs {
  int64_t n;
  const int64_t *off;   // G^t
  const int32_t *idx;
  int64_t E;
  int64_t nd2;          // 2*nd: entry ids below are deletions
  const unsigned long long *skeys;
  const int32_t *svals;
  const float *ew;
  const int32_t *C;     // C^{t-1}
  const double *K;      // K^{t-1}
  const double *Sig;    // Sigma^{t-1}
  double M2;
  uint8_t *dV, *rng, *dC, *dE, *dCm;
  // DS work
  unsigned long long *k2, *k2s;
  double *v2, *v2s;
  int32_t *list;
  int32_t *count;
};
void mark_df(const MarkArgs &a, hipStream_t s);   // DF marks + changedCommunities
void mark_changed(const MarkArgs &a, hipStream_t s);
void mark_ds_del(const MarkArgs &a, hipStream_t s);
void mark_ds_keys(const MarkArgs &a, hipStream_t s);       // k2/v2 for cross insertions
void mark_ds_best(const MarkArgs &a, hipStream_t s);       // on sorted k2s/v2s
void mark_ds_expand(const MarkArgs &a, hipStream_t s);     // list of dE, neighbours, communities
void update_weights(const MarkArgs &a, double *K, double *Sig, double *m2delta, hipStream_t s);

}  // namespace lk

namespace lk {
// out[0] += number of nonzero bytes in p[0..n)
void count_nonzero_u8(const uint8_t *p, int64_t n, unsigned long long *out, hipStream_t s);
// dst = src (bytes), n elements
void copy_u8(const uint8_t *src, uint8_t *dst, int64_t n, hipStream_t s);
}  // namespace lk
