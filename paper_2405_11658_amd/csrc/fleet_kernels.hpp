// Fused many-graph engine: one persistent launch updates many small graphs.
//
// A workgroup takes a job (one graph and its batch) from a queue in device
// memory and runs the whole update of that graph alone: batch validation and
// graph update (Sec. 3.5, 5.1.4), the ND / DS / DF marking and
// changedCommunities (Alg. "naiveDynamic", "deltaScreening",
// "dynamicFrontier", "leiden"), updateWeights, the pass loop of Alg. "leiden"
// (local moving, subset renumbering, breaking of changed communities,
// refinement, renumbering, aggregation), the final lookup and relabel, Sigma
// of the result and its modularity (Eq. 1).  Jobs never wait on each other,
// so the only synchronisation is the workgroup barrier.
//
// Local moving and refinement follow the serial asynchronous reading of
// Alg. "leidenMove" and "leidenRefine": the vertices of a level are visited
// one at a time in ascending id order, each reading the state the previous
// ones left; the workgroup's threads share the work of one vertex (its edges
// and its table of neighbouring communities).  The result of a job therefore
// does not depend on timing, on the number of wavefronts per workgroup or on
// the table size (the tuning parameters), only on the graph and the batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lk {

// Per graph, resident between launches.  Two CSR buffers (the graph and its
// update), the community state, and a workspace sized for n vertices and
// `cap` entries (the capacity of every CSR buffer of the graph).
struct FleetGraph {
  int64_t n;
  int64_t nnz;           // entries of the current CSR (updated by the kernel)
  int64_t cap;           // entry capacity of each CSR / level-graph buffer
  int32_t cur;           // which CSR buffer holds the graph (0 / 1; updated by the kernel)
  int32_t has_state;     // C, K, Sigma, M2 are valid (set by static / set_state)
  double M2;             // 2m of the current graph (updated by the kernel)
  int64_t *off[2];       // n+1
  int32_t *idx[2];       // cap
  float *w[2];           // cap
  int32_t *C;            // n: membership (dense labels)
  double *K;             // n
  double *Sig;           // n
  // workspace
  int32_t *Cl, *CB, *Ctop, *tmpi;   // n (+1 for tmpi)
  double *Kl, *Sl, *S2, *dense;     // n each; dense holds 0 between uses
  int32_t *tflag;                   // n, 0 between uses
  int32_t *tlist;                   // n: touched ids of the dense table
  uint8_t *dC, *dC2, *U, *rng, *dE, *dCm;  // n each
  int64_t *loff[2];                 // level graphs: n+1 offsets
  int32_t *lidx[2];                 // cap
  float *lw[2];                     // cap
  int32_t *rowd;                    // n: per-row entry count change of the batch (0 between uses)
  int64_t *mcnt;                    // n+1: aggregation / batch row counts
  unsigned long long *akey[2];      // cap: aggregation sort keys
  int32_t *apay[2];                 // cap: aggregation sort payloads
  double *asum;                     // cap: aggregation sums
};

// One job of a launch.
struct FleetJob {
  int32_t graph;         // index into the graph table
  int32_t mode;          // 0 = static, 1 = ND, 2 = DS, 3 = DF
  int64_t nd, ni;        // undirected deletions / insertions of the batch
  const int32_t *du, *dv, *iu, *iv;
  const float *iw;
  // per-job scratch (sized for E = 2(nd+ni) directed entries, at least 1)
  unsigned long long *bkey[2];   // E
  int32_t *bpay[2];              // E
  float *bw;                     // E (weight by directed entry id)
  int32_t *bpre;                 // E+1: deletions before each sorted entry
  int32_t *out;          // n, dense labels of the result (nullable)
};

struct FleetResult {
  int32_t status;        // 0 ok, 1 invalid batch, 3 no state
  int32_t err;           // batch error bits (as leiden_update's message)
  int32_t passes;
  int32_t pad;
  double q;
  int64_t affected, changed, moves_pass0;
  int32_t move_iters[16];
  int64_t level_vertices[16];
  int64_t communities[16];
};

struct FleetParams {
  double tau0, tol_drop, agg_tol;
  int32_t max_iter, max_passes;
  int32_t refine_variant;
  int32_t pad;
};

struct FleetLaunch {
  FleetGraph *graphs;
  const FleetJob *jobs;
  FleetResult *results;
  const int32_t *njobs;            // device scalar: jobs of this launch
  unsigned long long *next;        // device scalar: next job (reset by the host before each launch)
  FleetParams prm;
};

// Kernel variants: workgroup of 64 * waves threads, LDS table of `slots`
// entries (vertices and communities of degree up to slots / 2 use it, higher
// ones the graph's dense global table).
constexpr int kFleetVariants = 6;
struct FleetVariant {
  int waves;
  int slots;
};
constexpr FleetVariant kFleetVariant[kFleetVariants] = {{1, 512}, {2, 512}, {4, 512},
                                                        {1, 2048}, {2, 2048}, {4, 2048}};
// Enqueue the persistent launch with `blocks` workgroups of variant v.
hipError_t fleet_launch(const FleetLaunch &L, int variant, int blocks, hipStream_t s);

}  // namespace lk
