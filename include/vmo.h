/*
 * vmo.h -- C ABI of the MI355X (gfx950) implementation of the geometric
 * ("visual") matrix ordering of Fagginger Auer and Bisseling, "A Geometric
 * Approach to Matrix Ordering" (arXiv 1105.4490).
 *
 * Pointer conventions.  Every array argument is a DEVICE pointer unless its
 * comment says (host).  The caller owns every input and output buffer.  The
 * library owns only its workspace, a per-context caching pool of device
 * memory.  Calls on one context must not overlap (one context per host
 * thread).
 *
 * Streams and completion.  Every call runs its kernels on `stream` (a
 * hipStream_t; NULL = the null stream).  Calls marked [async] return once
 * their work is queued: their device outputs are ready when the stream
 * reaches that point (a later kernel or copy on the same stream sees them;
 * the host waits with vmo_sync or hipStreamSynchronize), and the caller keeps
 * the inputs alive and unchanged until then.  Some [async] calls still read a
 * few sizes back on the way (each says which and why); those waits end before
 * the call's last kernels.  All other calls return after their work is done
 * (they have host outputs).  A call on a stream other than the previous
 * [async] call's first waits for that call's work (the pool's blocks are then
 * free to reuse).
 *
 * Errors.  No call throws.  A call returns VMO_OK (0) or a negative status;
 * vmo_last_error() then holds a message.  Inputs are validated on the host
 * for scalars and on the device for array contents (pins in range and
 * ascending within a net, weights and coordinates finite).  Checks whose
 * result the call needs before its next step are read back at once and
 * reported by the call itself as VMO_E_INVALID, without writing partial
 * results the caller could mistake for output.  Checks that [async] calls
 * make on the device without waiting (those marked "checked on the device")
 * skip the call's writes when they fail and set the context's error word;
 * vmo_sync then returns VMO_E_INVALID with a message naming the check.
 *
 * Ids are 0-based (the paper counts from 1).  Permutations are in gather form:
 * perm[new] = old.
 */
#ifndef VMO_H
#define VMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vmo_status;
enum {
  VMO_OK = 0,
  VMO_E_INVALID = -1,     /* bad argument or array content                  */
  VMO_E_NOMEM = -2,       /* device allocation failed                       */
  VMO_E_DEVICE = -3,      /* a HIP runtime call failed                      */
  VMO_E_UNSUPPORTED = -4, /* a size beyond what this build handles          */
  VMO_E_BUSY = -5         /* serving queue full                             */
};

typedef struct vmo_ctx_s* vmo_ctx;
typedef void* vmo_stream; /* hipStream_t */

/* Context on HIP device `device`.  Allocates nothing until first use.
   pool_bytes bounds the device memory the workspace pool keeps cached between
   calls: after a call that waits for its work (and in vmo_sync), idle blocks
   beyond pool_bytes are returned to the device, largest first; 0 = no bound
   (every block stays cached, so the steady state allocates nothing). */
vmo_status vmo_create(vmo_ctx* out /* (host) */, int device, size_t pool_bytes);
/* Waits for the context's pending work, then frees it and its pool. */
vmo_status vmo_destroy(vmo_ctx ctx);
/* Waits until `stream` has finished the work queued on it (and the previous
   [async] call's work, if that ran on another stream), then reports what the
   device-side checks of [async] calls since the last vmo_sync found:
   VMO_E_INVALID with a message naming the failed checks (the word is then
   cleared), VMO_E_DEVICE if a bounded device-side wait ran out, else VMO_OK. */
vmo_status vmo_sync(vmo_ctx ctx, vmo_stream stream);
/* Message of the last failed call on this context (host string, owned by the
   context, valid until the next call). */
const char* vmo_last_error(vmo_ctx ctx);
/* Bytes currently held by the context's workspace pool. */
size_t vmo_pool_bytes(vmo_ctx ctx);

/* ---------------------------------------------------------------------------
 * Hypergraph (Definition of a hypergraph, Sec. 1.1).  V = {0..k-1}; the nets
 * E form a collection (duplicates and empty nets allowed) stored as CSR:
 * net e holds pins[net_ptr[e] .. net_ptr[e+1]), strictly ascending, each in
 * [0, k).  w: vertex weights [k] (NULL = all 1); c: net costs [l] (NULL = all
 * 1).  Weights and costs are >= 0; the layout needs them > 0.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t k, l;
  const int64_t* net_ptr; /* [l+1], net_ptr[0] = 0 */
  const int32_t* pins;    /* [net_ptr[l]]          */
  const float* w;         /* [k] or NULL           */
  const float* c;         /* [l] or NULL           */
} vmo_hypergraph;

/* Matrix-to-hypergraph models (Table 1).  Input: the pattern of an m x n
   sparse matrix as CSR (rowptr int64 [m+1], col int32, columns strictly
   ascending within a row; values are not used).
     VMO_ROW_NET:    vertices = the n columns, net i = columns of row i.
     VMO_COLUMN_NET: vertices = the m rows, net j = rows with a_ij != 0.
     VMO_SYMMETRIC:  (m == n) vertices = 0..n-1, nets = the distinct pairs
                     {i, j}, i < j, with a_ij != 0 or a_ji != 0, in
                     lexicographic order; diagonal entries are dropped.
     VMO_BIPARTITE:  vertices = the m rows (0..m-1), then the n columns
                     (m..m+n-1); one edge {i, m + j} per nonzero a_ij, in
                     CSR order (a graph: usable in VMO_GRAPH mode).
   Outputs: net_ptr [cap_nets+1], pins [cap_pins]; capacities must be at
   least: row-net l = m, pins = nnz; column-net l = n, pins = nnz; symmetric
   l <= nnz, pins <= 2 nnz; bipartite l = nnz, pins = 2 nnz.  *k, *l, *npins
   (host) receive the sizes. */
enum { VMO_ROW_NET = 0, VMO_COLUMN_NET = 1, VMO_SYMMETRIC = 2, VMO_BIPARTITE = 3 };
vmo_status vmo_model(vmo_ctx ctx, int model, int32_t m, int32_t n, const int64_t* rowptr,
                     const int32_t* col, int64_t* net_ptr, int32_t* pins, int32_t cap_nets,
                     int64_t cap_pins, int32_t* k, int32_t* l, int64_t* npins, vmo_stream stream);

/* [async] Dual hypergraph (Definition of the dual, Sec. 1.1): net v of the
   dual lists, ascending, the nets of h that contain v.  Outputs dptr [k+1],
   dpins [net_ptr[l]].  (Weights and costs swap roles; they are not copied.)
   Reads back: the pin check and net_ptr[l] (the sort's size). */
vmo_status vmo_dual(vmo_ctx ctx, const vmo_hypergraph* h, int64_t* dptr, int32_t* dpins,
                    vmo_stream stream);

/* [async] Connected components (Algorithm 1, Sec. 2.3): label[v] = the
   smallest vertex id in v's component, where nets connect their pins.  Reads
   back: the pin check, and one changed-flag per hooking round (the loop ends
   when a round changes nothing). */
vmo_status vmo_components(vmo_ctx ctx, const vmo_hypergraph* h, int32_t* label, vmo_stream stream);

/* Cut metrics of a partition (Sec. 4.1: a row/column is cut when it meets
   more than one diagonal block; the cut-net metric of the footnote there;
   Table 4 takes the maximum over splits).  lambda(e) = number of distinct
   values of part[] over the pins of net e.  Part ids are >= 0 and below
   2^30.  part_weight[p] (optional, [nparts]) = sum of w over part p < nparts,
   added in FP64 one vertex at a time in ascending vertex id.  Integral costs
   give exact sums; other costs are summed in FP64 in a fixed order (the same
   on every run). */
typedef struct {
  double lambda_minus_one; /* sum_e c(e) max(lambda(e) - 1, 0) */
  double cut_net;          /* sum of c(e) over nets with lambda(e) > 1 */
  int64_t nets_cut;        /* number of nets with lambda(e) > 1 */
  double max_split;        /* max over the splits h of split_cut[h] (below)  */
  int32_t max_split_node;  /* heap id of the first split reaching it (0: none) */
  int32_t separators;      /* 1 if part ids >= nparts occur (graph mode)     */
} vmo_cut_result;
/* split_cut[h] reads part[] as the leaves of a recursive bisection into
   P = nparts parts (Sec. 4.2; Table 4 reports the maximum over splits): node h
   (heap numbering, root 1) holds a contiguous part range, the root [0, P), its
   first child the first ceil(K/2) of its K parts, the second child the rest.
   Without separator ids, split_cut[h] = the sum of c(e), one by one in
   ascending net id, over the nets cut at h (pins in more than one part, h the
   deepest node holding all of them).  With separator ids (graph mode: vertex
   v in the separator S_h has part P + h), split_cut[h] = |S_h|. */
vmo_status vmo_cut(vmo_ctx ctx, const vmo_hypergraph* h, const int32_t* part, int32_t nparts,
                   double* part_weight, vmo_cut_result* out /* (host) */, vmo_stream stream);

/* vmo_cut for callers that cannot allocate memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the same
   kernels and the same results as vmo_cut, with every workspace block taken
   from a static 64 MiB device arena that the library holds on each GPU it
   runs on until the process ends.  It calls no hipMalloc, hipFree or other
   allocating routine.  Limits: at most 2^20 vertices and 2^20 nets
   (VMO_E_UNSUPPORTED beyond, before any work), and the arena must hold the
   call's blocks (about 28 bytes per net, 16 bytes per vertex when w is given
   and part_weight is asked for, and 32 bytes per pin of nets with more than 64
   pins; VMO_E_UNSUPPORTED when it does not).  Every call on a GPU uses that
   GPU's one arena, which keeps the last call's contents: calls that overlap
   on one GPU (other threads, other contexts, other streams) race and must not
   be made.  The call synchronises `stream` before returning. */
vmo_status vmo_cut_noalloc(vmo_ctx ctx, const vmo_hypergraph* h, const int32_t* part, int32_t nparts,
                           double* part_weight, vmo_cut_result* out /* (host) */, vmo_stream stream);

/* ---------------------------------------------------------------------------
 * One 2-means split (Algorithm 4 with m = 2; sides by the plane of
 * Algorithm 7).  x: k points in R^4 as FP32 SoA [4][k] (x[d*k + i]).  The
 * points are mapped once to a 2^20 grid over their bounding box; k-means++
 * seeding (exact D^2 draw from SplitMix64 keyed by seed) and at most t_max
 * Lloyd updates follow, with exact integer sums and an FP64 plane test
 * (s <= 0 -> part 1).  Outputs: side[k] (0 = part 1, 1 = part 2),
 * centres [2][4] FP32 (the centres of the final assignment), *iters (host)
 * = Lloyd updates performed, *split (host) = 1 if split, 0 if the points
 * cannot be split (all coincide, or a side came out empty; side = 0). */
vmo_status vmo_bisect(vmo_ctx ctx, const float* x, int32_t k, uint64_t seed, int32_t t_max,
                      uint8_t* side, float* centres, int32_t* iters, int32_t* split,
                      vmo_stream stream);

/* ---------------------------------------------------------------------------
 * Layout (Sec. 2): coordinates x: V -> R^4 minimising eq. (6) by the
 * multilevel steepest descent of Algorithms 2 and 3, each connected component
 * alone, components then packed side by side.
 * ------------------------------------------------------------------------- */
typedef struct {
  uint64_t seed;          /* keys every random draw                       */
  int32_t coarsest_iters; /* descent steps at the coarsest level (100)    */
  int32_t level_iters;    /* descent steps at every other level (30)      */
  int32_t min_coarse;     /* stop coarsening at <= this many vertices (64)*/
  int32_t max_levels;     /* at most this many coarsenings (40)           */
  int32_t leaf_cap;       /* tree leaves hold <= this many points (8)     */
  int32_t match_max_net;  /* nets larger than this do not propose (64)   */
  float theta;            /* opening angle of the tree walk (0.5; 0 = exact) */
  float step0_frac;       /* first step = this x box volume^(1/4) (0.1)   */
  float decay;            /* step length factor per step (0.9)            */
  float jitter;           /* prolongation displacement scale (1e-3)       */
  float stall;            /* stop coarsening if k shrinks by less (0.95)  */
  float pack_gap;         /* gap between packed components (0.1)          */
} vmo_layout_params;
/* Fills p with the defaults above and the given seed. */
void vmo_layout_defaults(vmo_layout_params* p /* (host) */, uint64_t seed);

/* Upper bound of the device memory the workspace of vmo_layout takes for a
   hypergraph of k vertices, l nets and npins pins (the serving loop admits
   layouts by it). */
size_t vmo_layout_bytes(int32_t k, int32_t l, int64_t npins);

/* [async] Full layout.  x [4][k] FP32 SoA output.  Reads back: the input
   checks, the component count and each component's size, each coarse level's
   sizes (its buffers are sized from them), one matching flag per eight
   matching rounds, and the component boxes (packing offsets).  The descent
   reads nothing back: each level's step length is formed on the device from
   its bounding box. */
vmo_status vmo_layout(vmo_ctx ctx, const vmo_hypergraph* h, const vmo_layout_params* p /* (host) */,
                      float* x, vmo_stream stream);

/* One coarsening step (Sec. 2.3: greedy heavy-net matching, single-neighbour
   vertices join their neighbour, identical nets merge with summed cost).
   level and comp key the random tie-break.  Outputs: pi[k] (coarse id of each
   vertex), coarse hypergraph into cptr [l+1], cpins [net_ptr[l]], cw [k],
   cc [l] (capacities of the fine sizes suffice); *kc, *lc (host). */
vmo_status vmo_coarsen(vmo_ctx ctx, const vmo_hypergraph* h, uint64_t seed, uint64_t comp,
                       int32_t level, int32_t match_max_net, int32_t* pi, int64_t* cptr,
                       int32_t* cpins, float* cw, float* cc, int32_t* kc, int32_t* lc,
                       vmo_stream stream);

/* The 2^d-tree of Algorithm 3 over points x [4][k] with weights w [k]
   (NULL = 1): pre-order nodes; a node at depth L covers a cell of side
   2^(16-L) of a 2^16 grid on the bounding cube; leaves hold <= leaf_cap
   points (or share one grid cell).  Outputs (capacity max_nodes, at most
   17 k + 1 nodes exist): ints [n][8] = first, count, depth, leaf, next, 0,0,0;
   cell2 [n][4] = cell centre x 2 in grid units; flt [n][5] = W, X0..X3
   (charge and its weighted centre); order [k] = point ids in tree order.
   *n_nodes (host). */
/* (vmo_tree reads back the node count, a host output; it does not wait for
   the copy of the node arrays: [async] for ints, cell2, flt and order.  The
   tree is built as the layout builds it: in one workgroup up to 4,096
   points, else by the multi-kernel build; both give the same tree.) */
vmo_status vmo_tree(vmo_ctx ctx, const float* x, const float* w, int32_t k, int32_t leaf_cap,
                    int32_t* ints, int32_t* cell2, float* flt, int32_t* order, int32_t max_nodes,
                    int32_t* n_nodes, vmo_stream stream);

/* [async] Gradient eq. (7) of the energy at x: attraction through the net
   centres, repulsion by the tree walk of Algorithm 3.  y [4][k], z [4][l]
   (net centres, may be NULL); *interactions (host, may be NULL) = charge
   interactions evaluated by the walk (reading it back waits for the walk). */
vmo_status vmo_gradient(vmo_ctx ctx, const vmo_hypergraph* h, const float* x, float theta,
                        int32_t leaf_cap, float* y, float* z, int64_t* interactions,
                        vmo_stream stream);

/* [async] `iters` descent steps of Algorithm 3 on x in place, steps it0 ..
   it0+iters-1 of a level.  *alpha (host) carries the step length: set from
   the bounding box at step 0 (read back then), multiplied by p->decay after
   every step. */
vmo_status vmo_layout_steps(vmo_ctx ctx, const vmo_hypergraph* h, const vmo_layout_params* p,
                            float* x, int32_t it0, int32_t iters, double* alpha, vmo_stream stream);

/* ---------------------------------------------------------------------------
 * Recursive ordering (Algorithm 7 applied recursively, Sec. 4.2; recursive
 * BBD of Sec. 4.1; recursive SBD of Sec. 5).  A node of the split tree with K
 * parts splits its vertices by 2-means into side 1 (ceil(K/2) parts, heap id
 * 2h) and side 2 (floor(K/2) parts, heap id 2h+1); it is a leaf if K = 1,
 * it has < 2 vertices, or its points cannot split.
 *   VMO_NET mode: any hypergraph; a net belongs to the deepest node holding
 *     all its pins (it is cut at that node when the node is internal).
 *   VMO_GRAPH mode: every net is an edge {v, w}, v < w; after each split the
 *     separator loop of Algorithm 7 (edges in net order; the end nearer the
 *     plane joins S, ties to v) builds S_h, which leaves both children.
 * SBD emits nodes in-order (left, node, right); BBD post-order.  Vertices in a
 * block ascend by id; nets within a node's block ascend; empty nets last.
 * ------------------------------------------------------------------------- */
enum { VMO_NET = 0, VMO_GRAPH = 1 };
enum { VMO_SBD = 0, VMO_BBD = 1 };
typedef struct {
  int32_t* vperm;     /* [k] new -> old                                       */
  int32_t* nperm;     /* [l] new -> old (VMO_NET; NULL to skip)               */
  int32_t* part;      /* [k] leaf part in [0,P); separator vertices P + heap id */
  int32_t* node_heap; /* [4P] heap id of the node at each emission rank, -1 pad */
  int32_t* node_vptr; /* [4P+1] vertex block boundaries by rank, k pad        */
  int32_t* node_nptr; /* [4P+2] net block boundaries by rank, then the empty-net
                          bucket, l pad (VMO_NET; NULL to skip)                */
  double* split_cut;  /* [4P] by rank: nets cut at the node (sum of costs) in
                          VMO_NET, |S_h| in VMO_GRAPH; 0 for leaves           */
  int32_t* n_nodes;   /* [1] number of tree nodes                             */
} vmo_order_out;

/* [async] x: coordinates [4][k]; NULL = compute them first with
   vmo_layout(lp).  P >= 1 parts; t_max Lloyd updates per split (32 is the
   usual value).  Reads back: the input checks, one convergence flag per eight
   Lloyd iterations, and each recursion level's segment count (the next
   level's launches and buffers are sized from it). */
vmo_status vmo_order(vmo_ctx ctx, const vmo_hypergraph* h, int mode, int order, const float* x,
                     const vmo_layout_params* lp /* (host) */, int32_t P, uint64_t seed,
                     int32_t t_max, const vmo_order_out* out /* (host) */, vmo_stream stream);
vmo_status vmo_order_sbd(vmo_ctx ctx, const vmo_hypergraph* h, int mode, const float* x,
                         const vmo_layout_params* lp, int32_t P, uint64_t seed, int32_t t_max,
                         const vmo_order_out* out, vmo_stream stream);
vmo_status vmo_order_bbd(vmo_ctx ctx, const vmo_hypergraph* h, int mode, const float* x,
                         const vmo_layout_params* lp, int32_t P, uint64_t seed, int32_t t_max,
                         const vmo_order_out* out, vmo_stream stream);

/* Recursive ordering of the border (Sec. 4.2: the freedom left in the cut
 * rows and columns of a recursive BBD, used to bring them into recursive BBD
 * form as in the rightmost partitioning of the figure on matrix
 * partitionings).  h: the graph of a VMO_GRAPH ordering (every net an edge
 * {v, w}, v < w); in: that ordering's vperm, part, node_heap, node_vptr and
 * n_nodes (device arrays as vmo_order writes them; nperm, node_nptr and
 * split_cut are not read); P: its part count.  Every vertex w of the
 * separator of a node h (depth d = floor(log2 h)) gets b two-bit words, the
 * first the most significant: word i has bit 1 (value 1) if an edge joins w to
 * a vertex in the first part (heap 2g) of the split of a node g at depth
 * d + i below h, and bit 2 (value 2) for the second part (2g + 1); vertices in
 * separators or leaves at depth <= d + i set nothing.  vperm_out[k] (device;
 * may be in->vperm) receives vperm with every separator block sorted stably by
 * the words; leaf blocks, part ids and the node tables are unchanged.  b in
 * [0, 15] (0: a copy).  VMO_E_INVALID if h is not a graph or the ordering
 * arrays are inconsistent (heap ids outside [1, 4P), block boundaries not
 * non-decreasing from 0 to k, part ids neither in [0, P) nor P + heap id,
 * vperm not a permutation). */
/* [async]; reads back the input checks and the node count. */
vmo_status vmo_order_border(vmo_ctx ctx, const vmo_hypergraph* h, const vmo_order_out* in /* (host) */, int32_t P,
                            int32_t b, int32_t* vperm_out, vmo_stream stream);

/* Schur-complement recursion (Sec. 4.2: the separator vertices V3 of a BBD
 * ordering, with the edges among them, E'3, ordered again by the same method).
 * h, in, P: as for vmo_order_border (h the graph of the ordering, in its
 * device arrays).  x: the coordinates the ordering used, [4][k] FP32 SoA
 * (device).  Every separator block of in with at least two vertices (its
 * first vertex has part >= P) is reordered by the VMO_GRAPH, VMO_BBD ordering
 * of its induced graph: local vertex i = the block's i-th vertex, with its
 * coordinates from x; edges = the nets of h with both ends in the block, in
 * net order, each as {min, max} of its local ends; P3 parts, t_max Lloyd
 * updates, the same seed, and the heap id of the block's node as the job index
 * of the random draws; mu (device [k], or NULL): a strengthened diagonal as
 * for vmo_order_matched, restricted to each block (partners outside the block
 * are dropped), so matched pairs stay together inside the Schur complement.  vperm_out[k] (device; may be in->vperm) receives vperm
 * with position lo + i of each such block holding the outer vertex at
 * lo + v3[i], v3 the block ordering's vperm; other blocks, part ids and the
 * node tables are unchanged.  One level: the blocks' own separators are not
 * reordered again.  P3 in [1, 2^24] (1: a copy).  All blocks are ordered in
 * one batched pass.  VMO_E_INVALID as for vmo_order_border, or if x is NULL
 * or not finite. */
/* [async]; reads back the input checks, the separator blocks' sizes and the
   batched ordering's level sizes. */
vmo_status vmo_order_schur(vmo_ctx ctx, const vmo_hypergraph* h, const float* x, const int32_t* mu,
                           const vmo_order_out* in /* (host) */, int32_t P, int32_t P3, uint64_t seed,
                           int32_t t_max, int32_t* vperm_out, vmo_stream stream);

/* ---------------------------------------------------------------------------
 * Strengthened diagonal (Sec. 4.2: a perfect matching M of the bipartite
 * graph, kept intact by Algorithm 7; Sec. 5: obtained by a heavy edge matching
 * augmented to a perfect matching by Hopcroft-Karp).
 *
 * vmo_match: matching of the bipartite graph of an m x n pattern (CSR as for
 * vmo_model; a: [nnz] values or NULL, only |a| is used, must be finite).
 * Heavy edge matching: nonzero e has the priority bits(|a_e|) << 32 |
 * fmix32(e + seed) (1.0 for every e when a is NULL; fmix32 = the 32-bit
 * finalizer of MurmurHash3, a bijection, so priorities are unique); the result
 * is the greedy matching that visits nonzeros by decreasing priority and takes
 * those whose row and column are free.  augment != 0: then augmented to a
 * maximum matching (a perfect one when the pattern has full structural rank)
 * by phases of breadth-first alternating-path forests from the free rows
 * (deterministic; which maximum matching is returned is not specified beyond
 * that).  Outputs (device): mrow[m] = matched column or -1, mcol[n] = matched
 * row or -1, mu[m+n] (or NULL) = partner in the bipartite model's vertex ids
 * (rows 0..m-1, columns m..m+n-1) or -1; *size (host) = matched pairs. */
vmo_status vmo_match(vmo_ctx ctx, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col,
                     const float* a, uint32_t seed, int augment, int32_t* mrow, int32_t* mcol, int32_t* mu,
                     int64_t* size /* (host) */, vmo_stream stream);

/* Graph-mode ordering with a strengthened diagonal (Algorithm 7 with its
 * matched-pair rule): as vmo_order with mode = VMO_GRAPH, but whenever a vertex
 * v enters a separator, mu[v] enters with it, so every pair {v, mu[v]} ends in
 * one block (with the bipartite model and a perfect matching: square diagonal
 * blocks).  mu: device [k], mu[v] = partner or -1; must be an involution
 * without fixed points whose pairs are edges of h (else VMO_E_INVALID).  An
 * all -1 mu gives vmo_order's result. */
/* [async]; reads back as vmo_order, and the check of mu. */
vmo_status vmo_order_matched(vmo_ctx ctx, const vmo_hypergraph* h, int order, const float* x,
                             const vmo_layout_params* lp /* (host) */, const int32_t* mu, int32_t P,
                             uint64_t seed, int32_t t_max, const vmo_order_out* out /* (host) */,
                             vmo_stream stream);

/* Row and column permutations of a square m x m matrix from an ordering of its
 * bipartite model (vperm over 2m vertices) with a perfect strengthened
 * diagonal mu (Sec. 4.2: the rows and columns of each block are the block's
 * vertices): rperm[t] = the t-th row in vperm order, cperm[t] = mu[rperm[t]]
 * - m, so the matching lies on the diagonal.  VMO_E_INVALID if vperm is not a
 * permutation of 0..2m-1 or a row has no partner column. */
/* [async], no readback: the permutation and partner checks are made on the
   device (checked on the device: a failure leaves rperm and cperm unwritten
   and vmo_sync returns VMO_E_INVALID). */
vmo_status vmo_matched_perms(vmo_ctx ctx, int32_t m, const int32_t* vperm, const int32_t* mu, int32_t* rperm,
                             int32_t* cperm, vmo_stream stream);

/* Kernighan-Lin refinement of bisections of a graph (Sec. 3: partitionings
 * made by Algorithm 4 improve under a few Kernighan-Lin iterations; Kernighan
 * and Lin 1970).  h: a graph (every net an edge {v, w}, v < w); every edge
 * weighs 1, parallel edges add up.  label (device [k], in/out): 2 g + s puts
 * v on side s (0 or 1) of bisection g, -1 leaves it out.  Each bisection is
 * refined on its own with only its inner edges counting: a pass sets D(v) =
 * (edges to the other side) - (edges to its own side), then min(|A|, |B|)
 * times locks the unlocked pair (a in A, b in B) of largest gain D(a) + D(b)
 * - 2 m(a, b) (m = edges joining them; ties to the smallest a, then the
 * smallest b) and updates D as if they had swapped; the first j pairs, j the
 * smallest index of largest prefix gain G(j), change sides if G(j) > 0, else
 * the bisection is done.  At most `passes` passes.  Side sizes are kept.
 * gain (device [G] or NULL): cut reduction of every bisection;
 * *ngroups (host, or NULL): G = 1 + the largest g.  One workgroup per
 * bisection; a pass costs O(|bisection|^2) work.  VMO_E_INVALID for labels
 * below -1, a hypergraph that is not a graph, degrees above 1024 or k >= 2^25. */
/* [async]; reads back the label check, the bisection count and the local
   adjacency's sizes. */
vmo_status vmo_refine_kl(vmo_ctx ctx, const vmo_hypergraph* h, int32_t* label, int32_t passes, int64_t* gain,
                         int32_t* ngroups /* (host) */, vmo_stream stream);

/* Finegrain coordinates (Sec. 4.2: each nonzero mapped to the average of the
 * points of its row and its column in a layout of the bipartite graph).
 * x: [4][m+n] (rows, then columns); xnz: [4][nnz], xnz[d][e] = (x[d][i] +
 * x[d][m+j]) * 0.5 in FP32 for nonzero e = (i, j) in CSR order. */
/* [async], no readback: rowptr (from 0, non-decreasing) and the columns (in
   [0, n), ascending within a row) are checked on the device (a failure leaves
   xnz unwritten and vmo_sync returns VMO_E_INVALID). */
vmo_status vmo_finegrain(vmo_ctx ctx, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col,
                         const float* x, float* xnz, vmo_stream stream);

/* Many orderings in one pass: every level of every job is processed by the
   same launches over one segment list (jobs[i].job_index keys its random
   draws as the job number).  Results equal those of vmo_order per job with
   the same job_index. */
typedef struct {
  vmo_hypergraph h;
  int32_t mode, order;
  const float* x;       /* [4][k]; must not be NULL here                    */
  int32_t P;
  uint64_t seed;
  uint64_t job_index;
  vmo_order_out out;
} vmo_job;
/* [async]; reads back as vmo_order. */
vmo_status vmo_order_batch(vmo_ctx ctx, int32_t njobs, const vmo_job* jobs /* (host) */,
                           int32_t t_max, vmo_stream stream);

/* Same ordering with one launch sequence per segment per level (the plain
   per-subproblem form, for comparison with vmo_order_batch). */
vmo_status vmo_order_batch_plain(vmo_ctx ctx, int32_t njobs, const vmo_job* jobs, int32_t t_max,
                                 vmo_stream stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of ordering jobs on one GPU.  A server owns a
 * worker thread, its own HIP stream and fixed device arenas sized from
 * budget_bytes (vertices, tree nodes, edges, nets, pins).  Jobs are admitted
 * in arrival order when a slot and contiguous arena ranges are free, which
 * bounds the device memory the server holds; their state then stays resident
 * on the device.  Every tick runs one recursion level for the segments of all
 * resident jobs in the same launches; a job submitted while others run joins
 * at the next tick, and a finished job is written to its output buffers and
 * leaves, freeing its ranges.  A job's result does not depend on the other
 * jobs in the mix (its random draws are keyed by seed and job_index).
 * budget_bytes bounds all the device memory the server holds: 40 % sizes the
 * arenas, 60 % the layouts of jobs with x == NULL, which are laid out
 * (vmo_layout with *lp) after admission by layout threads that run beside the
 * ticks.  Such a job is admitted only when its layout's footprint
 * (vmo_layout_bytes) fits in half of the layout share beside the layouts in
 * flight; the layout threads' cached workspace is trimmed to the other half
 * after each layout.  A job whose layout could never fit is refused
 * (VMO_E_UNSUPPORTED).
 * The caller keeps every buffer of a job valid and unchanged until the job is
 * done.  Submit, poll and wait may be called from any host thread.
 * ------------------------------------------------------------------------- */
typedef struct vmo_server_s* vmo_server;
typedef struct {
  int device;
  size_t budget_bytes;    /* device memory of the arenas                     */
  int32_t max_jobs;       /* resident jobs at most                           */
  int32_t t_max;          /* Lloyd updates per split                         */
  int32_t layout_threads; /* host threads, each with its own stream, laying
                             out jobs that come without coordinates (0..64;
                             0: the serving thread lays them out itself)     */
} vmo_serve_params;
typedef struct {
  int64_t submitted, completed, ticks, resident, pending;
  double busy_ms;      /* worker time spent in admission, ticks and emission */
  int64_t capacity_vertices, capacity_pins, capacity_edges;
  int64_t max_tick_jobs;      /* most jobs whose segments one tick ran together */
  int64_t tick_jobs;          /* sum over ticks of the jobs each ran          */
  int64_t layout_budget_bytes;/* budget share of the layouts (see above)      */
  int64_t layout_bytes_peak;  /* largest estimated footprint of the layouts in flight */
} vmo_serve_stats;
void vmo_serve_defaults(vmo_serve_params* p /* (host) */);
vmo_status vmo_serve_create(vmo_server* out /* (host) */, const vmo_serve_params* p /* (host) */);
/* Non-blocking.  VMO_E_UNSUPPORTED if the job can never fit the arenas. */
vmo_status vmo_serve_submit(vmo_server s, const vmo_job* job /* (host) */, const vmo_layout_params* lp /* (host) */,
                            uint64_t* ticket /* (host) */);
/* *done = 1 once the job's outputs are written; then *job_status and
   *latency_ms (submission to completion, host clock) are set. */
vmo_status vmo_serve_poll(vmo_server s, uint64_t ticket, int32_t* done, vmo_status* job_status,
                          double* latency_ms);
vmo_status vmo_serve_wait(vmo_server s, uint64_t ticket, vmo_status* job_status, double* latency_ms);
/* Drops the record of a finished ticket. */
vmo_status vmo_serve_forget(vmo_server s, uint64_t ticket);
vmo_status vmo_serve_get_stats(vmo_server s, vmo_serve_stats* out /* (host) */);
/* Message of a failed job (host string owned by the server). */
const char* vmo_serve_error(vmo_server s, uint64_t ticket);
/* Stops after the running tick; jobs not finished by then are marked done
   with VMO_E_BUSY.  No other thread may use the server once this is called. */
vmo_status vmo_serve_destroy(vmo_server s);

/* ---------------------------------------------------------------------------
 * Live kernel timing for measurement tools.  While enabled, the library
 * brackets launches of its main kernels with HIP events recorded on the
 * launch stream and accumulates, per kernel name, the summed durations, the
 * count of timed launches and their algorithmic work.  vmo_profile(ctx, n):
 * n = 0 disables; n >= 1 times every n-th launch of each kernel name (n = 1:
 * every launch; a larger n keeps the events' own cost, tens of microseconds
 * of stream time per timed launch, off most launches); n <= -1 times every
 * |n|-th launch without the work the kernels count on the device (the walk
 * then runs its uncounted form and reports work 0).  Kernels:
 *   "walk"   tree walk of the layout; work = charge interactions evaluated
 *            (counted by the kernel);
 *   "assign" Lloyd assignment pass; work = bytes of the positions it scans
 *            (16 B of grid coordinates + 1 B side each).
 * Counting adds one atomic per wavefront to the walk.  Disabling clears the
 * totals.  vmo_profile_read of a name never launched returns zeros.
 * ------------------------------------------------------------------------- */
typedef struct {
  double total_ms;
  int64_t launches;
  double work;
} vmo_profile_entry;
vmo_status vmo_profile(vmo_ctx ctx, int every /* 0: off; n >= 1: every n-th launch; -n: uncounted */);
vmo_status vmo_profile_read(vmo_ctx ctx, const char* kernel, vmo_profile_entry* out /* (host) */);
vmo_status vmo_profile_reset(vmo_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* VMO_H */
