/*
 * CPU ORACLE for the geometric matrix ordering method of Fagginger Auer and
 * Bisseling, "A Geometric Approach to Matrix Ordering" (arXiv 1105.4490).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product (the HIP
 * library behind include/vmo.h) shares no code, header, table or helper with
 * it.  Everything here is written sequentially, in the order the paper
 * states its steps, with the free choices the paper leaves open fixed as
 * listed below.  Compile with -O2 -ffp-contract=off -fopenmp (no contraction:
 * every float and double operation is a single IEEE rounding; the few fused
 * multiply-adds are explicit fmaf calls).  OpenMP runs only loops whose
 * iterations are independent (one vertex or one sampled point each, its terms
 * summed in its own fixed order), so the thread count never changes a result.
 *
 * Contents (paper passage in brackets):
 *   o_rng             counter-based SplitMix64 (Steele, Lea, Flood 2014).
 *   o_dual            dual hypergraph [Definition of the dual, Sec. 1.1].
 *   o_components      connected components, label = minimum vertex id
 *                     [Algorithm 1, Sec. 2.3; Theorem on disconnected graphs].
 *   o_cut             (lambda-1), cut-net metric, part weights
 *                     [Sec. 4.1 cut rows/columns; footnote on the cut-net
 *                      metric; Table 4 max cut per split].
 *   o_split_cuts      per-split cut of a recursive bisection's partition
 *                     [Table 4 maximum cut per split; Sec. 4.1].
 *   o_quantize        20-bit grid for exact 2-means sums (not in the paper;
 *                     an exactness device, see the reading of Alg. 4 below).
 *   o_bisect          one 2-means split [Algorithm 4 with m = 2, Algorithm 7
 *                     first part: sides and splitting plane].
 *   o_order           recursive SBD/BBD ordering, net mode and graph mode
 *                     [Algorithm 7; Sec. 4.1 recursive BBD; Sec. 4.2
 *                      permutations; Sec. 5 SBD form].
 *   o_border          recursive ordering of the border: separator blocks
 *                     sorted by b two-bit words [Sec. 4.2, cut rows and
 *                     columns into recursive BBD form].
 *   o_schur           Schur-complement recursion: every separator block
 *                     reordered by Algorithm 7 applied to its own graph
 *                     [Sec. 4.2, recursion on G3 = (V3, E'3)].
 *   o_match_heavy     heavy edge matching of the bipartite representation
 *                     (priority |a_ij|, ties by a scrambled index)
 *                     [Sec. 5, strengthened diagonal for the LU runs].
 *   o_match_augment   Hopcroft-Karp augmentation to a maximum matching
 *                     [Sec. 5; Hopcroft and Karp 1973].
 *   o_order_mu        o_order in graph mode with a strengthened diagonal mu:
 *                     a separator vertex takes its partner along
 *                     [Algorithm 7, the matched pair lines; Sec. 4.2].
 *   o_matched_perms   row and column permutations with the matching on the
 *                     diagonal [Sec. 4.2, permutations from V1, V2, V3].
 *   o_finegrain       nonzero coordinates = mean of row and column points
 *                     [Sec. 4.2, layout of the finegrain representation].
 *   o_refine_kl       Kernighan-Lin passes on bisections of a graph
 *                     [Sec. 3, partitionings of Algorithm 4 improved by
 *                     Kernighan-Lin; Kernighan and Lin 1970].
 *   o_coarsen         one coarsening step [Sec. 2.3, coarsening by greedy
 *                     heavy-net matching, single-neighbour rule, net merge].
 *   o_tree            2^d-tree with cluster charges [Sec. 2.1 tree
 *                     approximation; Algorithm 3 tree and sibling links].
 *   o_gradient        gradient eq. (7), STRICT mode: FP32, the walk summed in
 *                     the frozen two-level order of parts that the GPU
 *                     reproduces bit for bit [Algorithm 3; eq. (7)].
 *   o_gradient_plain  the same definition evaluated plainly: FP64, one
 *                     running sum per point over the depth-first walk, no
 *                     parts, no fused operations; with the magnitudes that
 *                     bound an FP32 evaluation's rounding [eq. (7)].
 *   o_layout_iter     one steepest-descent step, strict [Algorithm 3].
 *   o_layout_iter_plain  one step with the plain gradient, FP64 update.
 *   o_layout          multilevel layout of every component, packed
 *                     [Algorithm 2; Theorem on connectedness].
 *
 * Readings of points the paper leaves open (the GPU path implements the same
 * readings from its own code):
 *   - Ids are 0-based.  Nets form a multiset: duplicates and empty nets are
 *     kept, so the dual of the dual is the hypergraph itself.
 *   - d = 4, alpha = beta = 1, gamma = 2, delta = d - 2 = 2 (Sec. 2.1, Sec. 5).
 *   - Coordinates are FP32 (the paper packs one point in a 4-float register).
 *   - 2-means runs on coordinates quantized once per job to a 2^20 grid; sums
 *     are exact int64, the plane test is FP64 evaluated left to right, and a
 *     point with s(v) <= 0 goes to part 1 (Algorithm 7 uses <=).
 *   - k-means++ seeding draws from SplitMix64 keyed by (seed, job, node); the
 *     D^2 draw is exact 128/192-bit integer arithmetic.
 *   - Lloyd iterations stop when no assignment changes, or after t_max
 *     centre updates ("a fixed number of iterations" in Algorithm 4).
 *   - A node with K parts gives ceil(K/2) to side 1 and floor(K/2) to side 2;
 *     it is a leaf if K = 1, it has < 2 vertices, all its points coincide, or
 *     a side comes out empty ("until it can no longer continue", Sec. 5).
 *   - Net mode: a net belongs to the deepest node whose vertex set holds all
 *     its pins.  SBD lists nodes in-order, BBD post-order; ascending id within
 *     a block; empty nets last.  Graph mode: the separator loop of Algorithm 7
 *     visits edges in net order, and the separator S_h sits at node h.
 *   - Layout: far-field test on integer cell geometry, theta = 1/2; tree
 *     moments summed bottom-up in FP64; every vertex steps a length set by
 *     the bounding-box volume along its own gradient direction, the length
 *     shrinking by 0.9 per step; coarsening and random choices keyed by
 *     SplitMix64.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* SplitMix64: state advances by the golden gamma, output is the mix function */
static uint64_t o_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
#define O_GAMMA 0x9E3779B97F4A7C15ULL

/* Counter-based draw: chained SplitMix64 outputs keyed by three words. */
uint64_t o_rng(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t h = o_mix64(seed + O_GAMMA * (a + 1));
  h = o_mix64(h + O_GAMMA * (b + 1));
  return o_mix64(h + O_GAMMA * (c + 1));
}

/* Host threads of the independent per-vertex loops (OpenMP). */
void o_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int o_max_threads(void) { return omp_get_max_threads(); }

/* n-th output (n >= 1) of the plain SplitMix64 stream started at `seed`. */
uint64_t o_splitmix64(uint64_t seed, uint64_t n) { return o_mix64(seed + O_GAMMA * n); }

#define TAG_INIT 1u
#define TAG_PROLONG 2u
#define TAG_MATCH 3u
#define TAG_KMEANS 16u

/* ------------------------------------------------------------------------- */
/* Dual hypergraph: net v of G* lists, in ascending order, the nets holding v */
int o_dual(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, int64_t* dptr, int32_t* dpins) {
  memset(dptr, 0, sizeof(int64_t) * (size_t)(k + 1));
  for (int64_t p = 0; p < ptr[l]; ++p) {
    if (pins[p] < 0 || pins[p] >= k) return -1;
    dptr[pins[p] + 1]++;
  }
  for (int32_t v = 0; v < k; ++v) dptr[v + 1] += dptr[v];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
  for (int32_t v = 0; v < k; ++v) fill[v] = dptr[v];
  for (int32_t e = 0; e < l; ++e)
    for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) dpins[fill[pins[p]]++] = e;
  free(fill);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Connected components by breadth-first search from each vertex in ascending
   order: the first vertex that reaches a component is its minimum id. */
int o_components(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, int32_t* label) {
  int64_t* dptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k + 1));
  int32_t* dp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ptr[l] > 0 ? ptr[l] : 1));
  if (o_dual(k, l, ptr, pins, dptr, dp)) { free(dptr); free(dp); return -1; }
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  char* net_seen = (char*)calloc((size_t)(l > 0 ? l : 1), 1);
  for (int32_t v = 0; v < k; ++v) label[v] = -1;
  for (int32_t s = 0; s < k; ++s) {
    if (label[s] >= 0) continue;
    int32_t qh = 0, qt = 0;
    queue[qt++] = s;
    label[s] = s;
    while (qh < qt) {
      int32_t v = queue[qh++];
      for (int64_t a = dptr[v]; a < dptr[v + 1]; ++a) {
        int32_t e = dp[a];
        if (net_seen[e]) continue;
        net_seen[e] = 1;
        for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) {
          int32_t u = pins[p];
          if (label[u] < 0) { label[u] = s; queue[qt++] = u; }
        }
      }
    }
  }
  free(dptr); free(dp); free(queue); free(net_seen);
  return 0;
}

/* ------------------------------------------------------------------------- */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Cut metrics of a partition.  lambda(e) = number of distinct part ids among
   the pins of e.  out[0] = sum c(e) max(lambda-1, 0); out[1] = sum of c(e)
   over nets with lambda > 1; out[2] = number of such nets.  part_weight[p] =
   sum of w(v) over part(v) = p for p < nparts (ids >= nparts are not
   weighed).  Sums in FP64 in ascending net / vertex order. */
int o_cut(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* c,
          const int32_t* part, const float* w, int32_t nparts, double* out, double* part_weight) {
  int64_t maxlen = 0;
  for (int32_t e = 0; e < l; ++e) if (ptr[e + 1] - ptr[e] > maxlen) maxlen = ptr[e + 1] - ptr[e];
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxlen > 0 ? maxlen : 1));
  double lm1 = 0.0, cn = 0.0, ncut = 0.0;
  for (int32_t e = 0; e < l; ++e) {
    int64_t len = ptr[e + 1] - ptr[e];
    if (len == 0) continue;
    for (int64_t p = 0; p < len; ++p) {
      int32_t v = pins[ptr[e] + p];
      if (v < 0 || v >= k) { free(buf); return -1; }
      buf[p] = part[v];
    }
    qsort(buf, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t lam = 1;
    for (int64_t p = 1; p < len; ++p) if (buf[p] != buf[p - 1]) lam++;
    double ce = c ? (double)c[e] : 1.0;
    lm1 += ce * (double)(lam - 1);
    if (lam > 1) { cn += ce; ncut += 1.0; }
  }
  out[0] = lm1; out[1] = cn; out[2] = ncut;
  if (part_weight) {
    for (int32_t p = 0; p < nparts; ++p) part_weight[p] = 0.0;
    for (int32_t v = 0; v < k; ++v)
      if (part[v] >= 0 && part[v] < nparts) part_weight[part[v]] += w ? (double)w[v] : 1.0;
  }
  free(buf);
  return 0;
}

/* Per-split cut of a partition made by recursive bisection into P parts
   [Table 4: the maximum over splits of the rows/columns cut there; Sec. 4.1
   cut nets of the recursive BBD].  Node h (heap numbering, root 1) of the
   bisection holds the part range [p0, p0 + K): the root [0, P), child 2h the
   first ceil(K/2) parts, child 2h + 1 the rest.  A net whose pins lie in more
   than one part, all below P, is cut at the deepest node holding all of them;
   split[h] = sum of c(e) over the nets cut at h, in ascending net order.  If
   some part id is P or more (separator vertices of graph mode carry P + h),
   split[h] = the number of vertices with part id P + h instead.  split has 4P
   entries (heap ids below 4P); returns 1 in graph mode, 0 in net mode. */
static int32_t node_of_range(int32_t P, int32_t lo, int32_t hi) {
  int32_t h = 1, p0 = 0, K = P;
  while (K > 1) {
    int32_t K1 = (K + 1) / 2;
    if (hi < p0 + K1) { h = 2 * h; K = K1; }
    else if (lo >= p0 + K1) { h = 2 * h + 1; p0 += K1; K -= K1; }
    else break;
  }
  return h;
}

int o_split_cuts(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* c,
                 const int32_t* part, int32_t P, double* split) {
  for (int32_t h = 0; h < 4 * P; ++h) split[h] = 0.0;
  int graph = 0;
  for (int32_t v = 0; v < k; ++v) if (part[v] >= P) graph = 1;
  if (graph) {
    for (int32_t v = 0; v < k; ++v) {
      int32_t h = part[v] - P;
      if (h >= 1 && h < 4 * P) split[h] += 1.0;
    }
    return 1;
  }
  for (int32_t e = 0; e < l; ++e) {
    if (ptr[e + 1] - ptr[e] < 2) continue;
    int32_t lo = part[pins[ptr[e]]], hi = lo;
    for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) {
      int32_t q = part[pins[p]];
      if (q < lo) lo = q;
      if (q > hi) hi = q;
    }
    if (lo == hi || lo < 0 || hi >= P) continue;
    split[node_of_range(P, lo, hi)] += c ? (double)c[e] : 1.0;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Quantization: once per job, map the bounding box of the FP32 points to a
   2^20 grid.  lo = exact FP32 minimum per dimension; ext = largest side in
   FP64; scale = (2^20 - 1) / ext; q = floor((x - lo) * scale). */
#define QMAX 1048575u
int o_quantize(int32_t k, const float* x, uint32_t* q, float* lo_out, double* scale_out) {
  float lo[4], hi[4];
  for (int d = 0; d < 4; ++d) {
    lo[d] = x[(size_t)d * k];
    hi[d] = x[(size_t)d * k];
    for (int32_t i = 0; i < k; ++i) {
      float v = x[(size_t)d * k + i];
      if (!isfinite(v)) return -1;
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  }
  double ext = 0.0;
  for (int d = 0; d < 4; ++d) {
    double e = (double)hi[d] - (double)lo[d];
    if (e > ext) ext = e;
  }
  double s = ext > 0.0 ? (double)QMAX / ext : 0.0;
  for (int d = 0; d < 4; ++d) {
    for (int32_t i = 0; i < k; ++i) {
      uint32_t v = 0;
      if (s > 0.0) {
        double t = ((double)x[(size_t)d * k + i] - (double)lo[d]) * s;
        double f = floor(t);
        v = f >= (double)QMAX ? QMAX : (uint32_t)f;
      }
      q[(size_t)d * k + i] = v;
    }
    lo_out[d] = lo[d];
  }
  *scale_out = s;
  return 0;
}

/* Splitting plane of Algorithm 7: r = z2 - z1, delta = (z1 + z2)/2 . r.
   Every product and sum is rounded separately, left to right. */
static void plane_from(const double* c1, const double* c2, double* r, double* delta) {
  double m[4];
  for (int d = 0; d < 4; ++d) {
    r[d] = c2[d] - c1[d];
    double s = c1[d] + c2[d];
    m[d] = s * 0.5;
  }
  double a0 = m[0] * r[0];
  double a1 = m[1] * r[1];
  double a2 = m[2] * r[2];
  double a3 = m[3] * r[3];
  double t = a0 + a1;
  t = t + a2;
  t = t + a3;
  *delta = t;
}

/* s(v) = x(v).r - delta, same rounding discipline.  s <= 0 means part 1. */
static double splane(const uint32_t* q, size_t stride, int32_t v, const double* r, double delta) {
  double a0 = (double)q[v] * r[0];
  double a1 = (double)q[stride + v] * r[1];
  double a2 = (double)q[2 * stride + v] * r[2];
  double a3 = (double)q[3 * stride + v] * r[3];
  double t = a0 + a1;
  t = t + a2;
  t = t + a3;
  return t - delta;
}

/* One 2-means split of the vertices ids[0..n) (ascending ids) of node h of
   job `job`: k-means++ seeding with m = 2, then Lloyd iterations, Algorithm 4;
   sides by the plane of Algorithm 7.  Returns 0 when split (side[i] in {1,2}),
   1 when the node cannot split (all points coincide, or a side came out
   empty).  cen = centres used in the final assignment (grid units),
   plane = (r0..r3, delta), iters = centre updates done. */
static int o_split(const uint32_t* q, size_t stride, const int32_t* ids, int32_t n, uint64_t seed,
                   uint64_t job, int32_t h, int32_t t_max, uint8_t* side, double cen[2][4],
                   double plane[5], int32_t* iters) {
  uint64_t key = TAG_KMEANS | (job << 8);
  *iters = 0;
  /* z1: uniform member of the node */
  uint64_t r0 = o_rng(seed, key, (uint64_t)h, 0);
  int32_t i1 = (int32_t)(((u128)r0 * (u128)(uint64_t)n) >> 64);
  /* D^2 weights, exact */
  int64_t* dd = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  u128 T = 0;
  int32_t v1 = ids[i1];
  for (int32_t i = 0; i < n; ++i) {
    int32_t v = ids[i];
    int64_t s = 0;
    for (int d = 0; d < 4; ++d) {
      int64_t df = (int64_t)q[d * stride + v] - (int64_t)q[d * stride + v1];
      s += df * df;
    }
    dd[i] = s;
    T += (u128)(uint64_t)s;
  }
  if (T == 0) { free(dd); return 1; }
  /* t = floor(r1 * T / 2^64) with T < 2^75: 192-bit product, high part */
  uint64_t r1 = o_rng(seed, key, (uint64_t)h, 1);
  uint64_t Tlo = (uint64_t)T, Thi = (uint64_t)(T >> 64);
  u128 plo = (u128)r1 * (u128)Tlo;
  u128 t = (plo >> 64) + (u128)r1 * (u128)Thi;
  u128 acc = 0;
  int32_t i2 = -1;
  for (int32_t i = 0; i < n; ++i) {
    acc += (u128)(uint64_t)dd[i];
    if (acc > t) { i2 = i; break; }
  }
  free(dd);
  int32_t v2 = ids[i2];
  double c1[4], c2[4], r[4], delta;
  for (int d = 0; d < 4; ++d) { c1[d] = (double)q[d * stride + v1]; c2[d] = (double)q[d * stride + v2]; }
  plane_from(c1, c2, r, &delta);
  int64_t cnt[2] = {0, 0};
  for (int32_t i = 0; i < n; ++i) {
    double s = splane(q, stride, ids[i], r, delta);
    side[i] = s <= 0.0 ? 1 : 2;
    cnt[side[i] - 1]++;
  }
  if (cnt[0] == 0 || cnt[1] == 0) return 1;
  for (int32_t it = 1; it <= t_max; ++it) {
    int64_t S[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int64_t N[2] = {0, 0};
    for (int32_t i = 0; i < n; ++i) {
      int a = side[i] - 1;
      N[a]++;
      for (int d = 0; d < 4; ++d) S[a][d] += (int64_t)q[d * stride + ids[i]];
    }
    double m1[4], m2[4], rr[4], dl;
    for (int d = 0; d < 4; ++d) {
      m1[d] = (double)S[0][d] / (double)N[0];
      m2[d] = (double)S[1][d] / (double)N[1];
    }
    plane_from(m1, m2, rr, &dl);
    int64_t nc[2] = {0, 0};
    int changed = 0;
    for (int32_t i = 0; i < n; ++i) {
      double s = splane(q, stride, ids[i], rr, dl);
      uint8_t sd = s <= 0.0 ? 1 : 2;
      if (sd != side[i]) changed = 1;
      side[i] = sd;
      nc[sd - 1]++;
    }
    memcpy(c1, m1, sizeof c1);
    memcpy(c2, m2, sizeof c2);
    memcpy(r, rr, sizeof r);
    delta = dl;
    *iters = it;
    if (nc[0] == 0 || nc[1] == 0) return 1;
    if (!changed) break;
  }
  for (int d = 0; d < 4; ++d) { cen[0][d] = c1[d]; cen[1][d] = c2[d]; plane[d] = r[d]; }
  plane[4] = delta;
  return 0;
}

/* One split of a whole point set (vmo_bisect): quantize, then o_split on all
   k points with job 0, node 1.  side[v] = 0 for part 1, 1 for part 2.
   centres [2][4] reported in coordinates: lo + c / scale, rounded to FP32.
   Returns 0 split, 1 unsplittable (side all 0), <0 error. */
int o_bisect(int32_t k, const float* x, uint64_t seed, int32_t t_max, uint8_t* side_out,
             float* centres, int32_t* iters, double* plane_out) {
  if (k < 1) return -1;
  uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * 4 * (size_t)k);
  float lo[4];
  double s;
  if (o_quantize(k, x, q, lo, &s)) { free(q); return -1; }
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t i = 0; i < k; ++i) ids[i] = i;
  uint8_t* sd = (uint8_t*)malloc((size_t)k);
  double cen[2][4], plane[5];
  int rc = 1;
  *iters = 0;
  if (k >= 2) rc = o_split(q, (size_t)k, ids, k, seed, 0, 1, t_max, sd, cen, plane, iters);
  if (rc == 0) {
    for (int32_t i = 0; i < k; ++i) side_out[i] = (uint8_t)(sd[i] - 1);
    for (int a = 0; a < 2; ++a)
      for (int d = 0; d < 4; ++d) centres[a * 4 + d] = (float)((double)lo[d] + cen[a][d] / s);
    if (plane_out) for (int d = 0; d < 5; ++d) plane_out[d] = plane[d];
  } else {
    for (int32_t i = 0; i < k; ++i) side_out[i] = 0;
    for (int a = 0; a < 2; ++a) for (int d = 0; d < 4; ++d) centres[a * 4 + d] = 0.0f;
  }
  free(q); free(ids); free(sd);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Recursive ordering. */
typedef struct {
  int exists, leaf, K, p0;
  int32_t* verts; int32_t nv;   /* leaf: its vertices; internal: unused      */
  int32_t* sep; int32_t ns;     /* graph mode separator S_h (ascending)       */
  int32_t* nets; int32_t nn;    /* net mode: nets alive at this node          */
} ONode;

static void emit_walk(ONode* nd, int32_t nmax, int32_t h, int post, int32_t* order, int32_t* cnt) {
  if (h >= nmax || !nd[h].exists) return;
  if (nd[h].leaf) { order[(*cnt)++] = h; return; }
  emit_walk(nd, nmax, 2 * h, post, order, cnt);
  if (!post) order[(*cnt)++] = h;
  emit_walk(nd, nmax, 2 * h + 1, post, order, cnt);
  if (post) order[(*cnt)++] = h;
}

/* mode 0 = net mode (cut nets placed at the node that splits them),
   mode 1 = graph mode (Algorithm 7 vertex separator; nets must be edges
   {v, w} with v < w).  ord 0 = SBD (in-order), 1 = BBD (post-order).
   Outputs (caller allocated): vperm[k], nperm[l] (net mode; may be NULL),
   part[k], node_heap[4P], node_vptr[4P+1], node_nptr[4P+2] (net mode; may be
   NULL), split_cut[4P] (by emission rank), n_nodes[1].  Returns 0 or <0. */
/* A strengthened diagonal mu (graph mode only; NULL = none): mu[v] = the
   vertex matched to v, or -1.  It must be an involution without fixed points
   whose pairs {v, mu(v)} are edges of the graph. */
static int check_mu(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const int32_t* mu) {
  if (k < 1) return -1;
  for (int32_t v = 0; v < k; ++v) {
    const int32_t w = mu[v];
    if (w < -1 || w >= k || w == v) return -1;
    if (w >= 0 && mu[w] != v) return -1;
  }
  char* ok = (char*)calloc((size_t)k, 1);
  for (int32_t e = 0; e < l; ++e) {
    const int32_t a = pins[ptr[e]], b = pins[ptr[e] + 1];
    if (mu[a] == b) ok[a] = ok[b] = 1;
  }
  int rc = 0;
  for (int32_t v = 0; v < k; ++v)
    if (mu[v] >= 0 && !ok[v]) rc = -1;
  free(ok);
  return rc;
}

int o_order_mu(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* c,
               int mode, int ord, const float* x, const int32_t* mu, int32_t P, uint64_t seed, uint64_t job,
               int32_t t_max, int32_t* vperm, int32_t* nperm, int32_t* part, int32_t* node_heap,
               int32_t* node_vptr, int32_t* node_nptr, double* split_cut, int32_t* n_nodes_out) {
  if (k < 1 || P < 1 || l < 0) return -1;
  if (mode == 1)
    for (int32_t e = 0; e < l; ++e)
      if (ptr[e + 1] - ptr[e] != 2 || pins[ptr[e]] >= pins[ptr[e] + 1]) return -1;
  if (mu && (mode != 1 || check_mu(k, l, ptr, pins, mu))) return -1;
  int32_t nmax = 4 * P;
  uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * 4 * (size_t)k);
  float lo[4];
  double sc;
  if (o_quantize(k, x, q, lo, &sc)) { free(q); return -1; }
  ONode* nd = (ONode*)calloc((size_t)nmax, sizeof(ONode));
  int32_t* netnode = (int32_t*)malloc(sizeof(int32_t) * (size_t)(l > 0 ? l : 1));
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  uint8_t* sd_of = (uint8_t*)malloc((size_t)k);
  double* s_of = (double*)malloc(sizeof(double) * (size_t)k);
  char* in_sep = (char*)calloc((size_t)k, 1);
  for (int32_t v = 0; v < k; ++v) mark[v] = 0;
  for (int32_t e = 0; e < l; ++e) netnode[e] = -1; /* -1 = empty net */
  nd[1].exists = 1; nd[1].K = P; nd[1].p0 = 0;
  nd[1].verts = (int32_t*)malloc(sizeof(int32_t) * (size_t)k); nd[1].nv = k;
  for (int32_t v = 0; v < k; ++v) nd[1].verts[v] = v;
  if (mode == 0) {
    nd[1].nets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(l > 0 ? l : 1));
    for (int32_t e = 0; e < l; ++e) if (ptr[e + 1] > ptr[e]) nd[1].nets[nd[1].nn++] = e;
  }
  for (int32_t h = 1; h < nmax; ++h) {
    ONode* N = &nd[h];
    if (!N->exists) continue;
    int32_t n = N->nv;
    uint8_t* side = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    double cen[2][4], plane[5];
    int32_t its;
    int rc = 1;
    if (N->K > 1 && n >= 2) rc = o_split(q, (size_t)k, N->verts, n, seed, job, h, t_max, side, cen, plane, &its);
    if (rc != 0) {
      N->leaf = 1;
      for (int32_t i = 0; i < N->nn; ++i) netnode[N->nets[i]] = h;
      free(side);
      continue;
    }
    for (int32_t i = 0; i < n; ++i) {
      int32_t v = N->verts[i];
      mark[v] = h; sd_of[v] = side[i];
      s_of[v] = splane(q, (size_t)k, v, plane, plane[4]);
    }
    if (mode == 1) {
      /* Algorithm 7 separator: edges in order; a cut edge whose ends are both
         still in parts 1/2 sends the end nearer the plane into S (ties: v),
         together with its partner under mu (Algorithm 7, the matched pair
         lines), so that every matched pair stays in one of V1, V2, V3. */
      N->sep = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
      for (int32_t e = 0; e < l; ++e) {
        int32_t a = pins[ptr[e]], b = pins[ptr[e] + 1];
        if (mark[a] != h || mark[b] != h) continue;
        if (in_sep[a] || in_sep[b]) continue;
        if (sd_of[a] == sd_of[b]) continue;
        const int32_t t = fabs(s_of[a]) <= fabs(s_of[b]) ? a : b;
        in_sep[t] = 1;
        if (mu && mu[t] >= 0) in_sep[mu[t]] = 1;
      }
      for (int32_t i = 0; i < n; ++i) if (in_sep[N->verts[i]]) N->sep[N->ns++] = N->verts[i];
    }
    int32_t Kl = (N->K + 1) / 2, Kr = N->K / 2;
    ONode* L = &nd[2 * h];
    ONode* R = &nd[2 * h + 1];
    L->exists = R->exists = 1;
    L->K = Kl; L->p0 = N->p0; R->K = Kr; R->p0 = N->p0 + Kl;
    L->verts = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    R->verts = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
      int32_t v = N->verts[i];
      if (in_sep[v]) continue;
      if (side[i] == 1) L->verts[L->nv++] = v; else R->verts[R->nv++] = v;
    }
    if (mode == 0) {
      L->nets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N->nn > 0 ? N->nn : 1));
      R->nets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N->nn > 0 ? N->nn : 1));
      for (int32_t i = 0; i < N->nn; ++i) {
        int32_t e = N->nets[i];
        int has1 = 0, has2 = 0;
        for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) {
          if (sd_of[pins[p]] == 1) has1 = 1; else has2 = 1;
        }
        if (has1 && has2) netnode[e] = h;
        else if (has1) L->nets[L->nn++] = e;
        else R->nets[R->nn++] = e;
      }
    }
    free(side);
  }
  /* emission */
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)nmax);
  int32_t nnodes = 0;
  emit_walk(nd, nmax, 1, ord == 1, order, &nnodes);
  int32_t vp = 0;
  for (int32_t r = 0; r < nnodes; ++r) {
    int32_t h = order[r];
    node_heap[r] = h;
    node_vptr[r] = vp;
    if (nd[h].leaf) {
      for (int32_t i = 0; i < nd[h].nv; ++i) { vperm[vp++] = nd[h].verts[i]; part[nd[h].verts[i]] = nd[h].p0; }
    } else {
      for (int32_t i = 0; i < nd[h].ns; ++i) { vperm[vp++] = nd[h].sep[i]; part[nd[h].sep[i]] = P + h; }
    }
    split_cut[r] = 0.0;
    if (mode == 1 && !nd[h].leaf) split_cut[r] = (double)nd[h].ns;
  }
  for (int32_t r = nnodes; r < nmax; ++r) { node_heap[r] = -1; node_vptr[r] = k; split_cut[r] = 0.0; }
  node_vptr[nmax] = k;
  if (mode == 0) {
    int32_t np = 0;
    for (int32_t r = 0; r < nnodes; ++r) {
      int32_t h = order[r];
      if (node_nptr) node_nptr[r] = np;
      for (int32_t e = 0; e < l; ++e)
        if (netnode[e] == h) {
          if (nperm) nperm[np] = e;
          np++;
          if (!nd[h].leaf) split_cut[r] += c ? (double)c[e] : 1.0;
        }
    }
    if (node_nptr) node_nptr[nnodes] = np;
    for (int32_t e = 0; e < l; ++e) if (netnode[e] < 0) { if (nperm) nperm[np] = e; np++; }
    if (node_nptr) for (int32_t r = nnodes + 1; r <= nmax + 1; ++r) node_nptr[r] = l;
  }
  *n_nodes_out = nnodes;
  for (int32_t h = 0; h < nmax; ++h) { free(nd[h].verts); free(nd[h].sep); free(nd[h].nets); }
  free(nd); free(order); free(q); free(netnode); free(mark); free(sd_of); free(s_of); free(in_sep);
  return 0;
}

int o_order(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* c,
            int mode, int ord, const float* x, int32_t P, uint64_t seed, uint64_t job, int32_t t_max,
            int32_t* vperm, int32_t* nperm, int32_t* part, int32_t* node_heap, int32_t* node_vptr,
            int32_t* node_nptr, double* split_cut, int32_t* n_nodes_out) {
  return o_order_mu(k, l, ptr, pins, c, mode, ord, x, NULL, P, seed, job, t_max, vperm, nperm, part, node_heap,
                    node_vptr, node_nptr, split_cut, n_nodes_out);
}

/* ------------------------------------------------------------------------- */
/* Recursive ordering of the border [Sec. 4.2, the paragraphs on the freedom
   left in the cut rows and columns; the rightmost partitioning of the figure
   on matrix partitionings for recursive BBD].  Input: a graph-mode ordering
   (vperm, part, node_heap, node_vptr, n_nodes as o_order writes them; nets
   are edges {v, w}).  Every vertex w of the separator V3 of a node h (heap id,
   depth d = floor(log2 h)) gets b two-bit words, first word most significant,
   all 00 at the start.  Word i (i = 1..b) records the split of the nodes at
   depth d + i below h: when such a node Vj splits into Vj1, Vj2 and its own
   separator, every edge {v, w} with v in Vj1 sets the first bit (value 1) of
   w's word i and every edge with v in Vj2 its second bit (value 2); a v in a
   separator or a leaf at depth <= d + i sets nothing.  The vertices of each
   separator block are then sorted by their words, stably (equal words keep
   their order).  Leaf blocks and the part ids do not change.  b = 0 copies
   vperm.  Returns 0 or <0. */
static int32_t heap_depth(int32_t h) {
  int32_t d = 0;
  while (h > 1) { h >>= 1; ++d; }
  return d;
}
int o_border(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const int32_t* vperm,
             const int32_t* part, const int32_t* node_heap, const int32_t* node_vptr, int32_t n_nodes, int32_t P,
             int32_t b, int32_t* vperm_out) {
  if (k < 1 || P < 1 || b < 0 || b > 15 || n_nodes < 1 || n_nodes > 4 * P) return -1;
  for (int32_t i = 0; i < k; ++i) vperm_out[i] = vperm[i];
  if (b == 0) return 0;
  /* the node (heap id) each vertex ends in */
  int32_t* leaf_heap = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  int32_t* vh = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  uint32_t* word = (uint32_t*)calloc((size_t)k, sizeof(uint32_t));
  for (int32_t p = 0; p < P; ++p) leaf_heap[p] = 0;
  for (int32_t r = 0; r < n_nodes; ++r)
    for (int32_t i = node_vptr[r]; i < node_vptr[r + 1]; ++i)
      if (part[vperm[i]] < P) leaf_heap[part[vperm[i]]] = node_heap[r];
  for (int32_t v = 0; v < k; ++v) vh[v] = part[v] >= P ? part[v] - P : leaf_heap[part[v]];
  /* the words: every edge, seen from each end that lies in a separator */
  for (int32_t e = 0; e < l; ++e) {
    if (ptr[e + 1] - ptr[e] != 2) continue;
    for (int s = 0; s < 2; ++s) {
      const int32_t w = pins[ptr[e] + s], v = pins[ptr[e] + 1 - s];
      if (part[w] < P) continue;  /* w is not a separator vertex */
      const int32_t h = vh[w], d = heap_depth(h);
      const int32_t hv = vh[v], D = heap_depth(hv);
      if (D <= d || (hv >> (D - d)) != h) continue;  /* v is not below h */
      for (int32_t i = 1; i <= b; ++i) {
        if (D < d + i + 1) break;  /* v stopped at or above depth d + i */
        const int32_t second = (hv >> (D - d - i - 1)) & 1;  /* which part of the split at depth d + i */
        word[w] |= (uint32_t)(second ? 2 : 1) << (2 * (b - i));
      }
    }
  }
  /* stable sort of each separator block by the words (insertion sort) */
  for (int32_t r = 0; r < n_nodes; ++r) {
    const int32_t lo = node_vptr[r], hi = node_vptr[r + 1];
    if (hi - lo < 2 || part[vperm[lo]] < P) continue;
    for (int32_t i = lo + 1; i < hi; ++i) {
      const int32_t v = vperm_out[i];
      int32_t j = i - 1;
      while (j >= lo && word[vperm_out[j]] > word[v]) { vperm_out[j + 1] = vperm_out[j]; --j; }
      vperm_out[j + 1] = v;
    }
  }
  free(leaf_heap);
  free(vh);
  free(word);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Schur-complement recursion [Sec. 4.2, the paragraph on the freedom in the
   rows and columns of V3: Algorithm 7 applied recursively to G3 = (V3, E'3),
   E'3 the edges with both ends in V3, as for G1 and G2; the middle
   partitioning of the figure on matrix partitionings].  Input: a graph-mode
   ordering as o_border takes it, its coordinates x [4][k], and P3 >= 1.  The
   vertex block of every separator S_h (h internal) with at least two
   vertices is reordered by the recursive graph-mode BBD ordering (o_order,
   P3 parts, t_max, draws keyed by job = h) of the graph (S_h, edges inside
   S_h): local vertex i is the i-th vertex of the block as given, the edges
   keep their net order with local ends ascending, the coordinates are the
   vertices' own.  One level: the separators of these orderings are not
   recursed again.  Leaf blocks, part ids and node tables do not change.
   Returns 0 or <0. */
int o_schur(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* x, const int32_t* mu,
            const int32_t* vperm, const int32_t* part, const int32_t* node_heap, const int32_t* node_vptr,
            int32_t n_nodes, int32_t P, int32_t P3, uint64_t seed, int32_t t_max, int32_t* vperm_out) {
  if (k < 1 || P < 1 || P3 < 1 || n_nodes < 1 || n_nodes > 4 * P) return -1;
  if (mu && check_mu(k, l, ptr, pins, mu)) return -1;
  for (int32_t i = 0; i < k; ++i) vperm_out[i] = vperm[i];
  int32_t* loc = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t v = 0; v < k; ++v) loc[v] = -1;
  int rc = 0;
  for (int32_t r = 0; r < n_nodes && rc == 0; ++r) {
    const int32_t lo = node_vptr[r], hi = node_vptr[r + 1], m = hi - lo;
    if (m < 2 || part[vperm[lo]] < P) continue;  /* a leaf block, or too small */
    const int32_t h = node_heap[r];
    for (int32_t i = 0; i < m; ++i) loc[vperm[lo + i]] = i;
    /* the edges inside the block, in net order */
    int32_t l3 = 0;
    for (int32_t e = 0; e < l; ++e)
      if (ptr[e + 1] - ptr[e] == 2 && loc[pins[ptr[e]]] >= 0 && loc[pins[ptr[e] + 1]] >= 0) ++l3;
    int64_t* ptr3 = (int64_t*)malloc(sizeof(int64_t) * ((size_t)l3 + 1));
    int32_t* pins3 = (int32_t*)malloc(sizeof(int32_t) * (2 * (size_t)l3 + 1));
    int32_t t = 0;
    ptr3[0] = 0;
    for (int32_t e = 0; e < l; ++e) {
      if (ptr[e + 1] - ptr[e] != 2) continue;
      const int32_t a = loc[pins[ptr[e]]], b = loc[pins[ptr[e] + 1]];
      if (a < 0 || b < 0) continue;
      pins3[2 * t] = a < b ? a : b;
      pins3[2 * t + 1] = a < b ? b : a;
      ++t;
      ptr3[t] = 2 * (int64_t)t;
    }
    float* x3 = (float*)malloc(sizeof(float) * 4 * (size_t)m);
    for (int d = 0; d < 4; ++d)
      for (int32_t i = 0; i < m; ++i) x3[(size_t)d * m + i] = x[(size_t)d * k + vperm[lo + i]];
    /* the strengthened diagonal restricted to the block (partners outside
       the block are dropped) */
    int32_t* mu3 = NULL;
    if (mu) {
      mu3 = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
      for (int32_t i = 0; i < m; ++i) {
        const int32_t w = mu[vperm[lo + i]];
        mu3[i] = w >= 0 ? loc[w] : -1;
      }
    }
    int32_t* v3 = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    int32_t* p3 = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    int32_t* heap3 = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)P3);
    int32_t* vptr3 = (int32_t*)malloc(sizeof(int32_t) * (4 * (size_t)P3 + 1));
    double* sc3 = (double*)malloc(sizeof(double) * 4 * (size_t)P3);
    int32_t nn3 = 0;
    rc = o_order_mu(m, l3, ptr3, pins3, NULL, 1, 1, x3, mu3, P3, seed, (uint64_t)h, t_max, v3, NULL, p3, heap3,
                    vptr3, NULL, sc3, &nn3);
    if (rc == 0)
      for (int32_t i = 0; i < m; ++i) vperm_out[lo + i] = vperm[lo + v3[i]];
    for (int32_t i = 0; i < m; ++i) loc[vperm[lo + i]] = -1;
    free(ptr3); free(pins3); free(x3); free(mu3); free(v3); free(p3); free(heap3); free(vptr3); free(sc3);
  }
  free(loc);
  return rc;
}

/* ========================================================================= */
/* Layout (Section 2).                                                        */

typedef struct {
  uint64_t seed;
  int32_t coarsest_iters, level_iters, min_coarse, max_levels, leaf_cap, match_max_net;
  float theta, step0_frac, decay, jitter, stall, pack_gap;
} o_layout_params;

/* ---- coarsening ---------------------------------------------------------- */
typedef struct { int32_t u, v; double om; uint64_t hs; } OPair;

static int cmp_pair_uv(const void* a, const void* b) {
  const OPair* x = (const OPair*)a; const OPair* y = (const OPair*)b;
  if (x->u != y->u) return x->u < y->u ? -1 : 1;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  if (x->om != y->om) return x->om > y->om ? -1 : 1;
  return 0;
}
/* priority: larger omega first, then larger hash, then smaller (u, v) */
static int cmp_pair_prio(const void* a, const void* b) {
  const OPair* x = (const OPair*)a; const OPair* y = (const OPair*)b;
  if (x->om != y->om) return x->om > y->om ? -1 : 1;
  if (x->hs != y->hs) return x->hs > y->hs ? -1 : 1;
  if (x->u != y->u) return x->u < y->u ? -1 : 1;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  return 0;
}

typedef struct { int32_t e, len; const int32_t* p; } ONetImg;
static int cmp_img(const void* a, const void* b) {
  const ONetImg* x = (const ONetImg*)a; const ONetImg* y = (const ONetImg*)b;
  int32_t m = x->len < y->len ? x->len : y->len;
  for (int32_t i = 0; i < m; ++i) if (x->p[i] != y->p[i]) return x->p[i] < y->p[i] ? -1 : 1;
  if (x->len != y->len) return x->len < y->len ? -1 : 1;
  return (x->e > y->e) - (x->e < y->e);
}
typedef struct { int32_t rep, len; const int32_t* p; float c; } OCNet;
static int cmp_cnet(const void* a, const void* b) {
  const OCNet* x = (const OCNet*)a; const OCNet* y = (const OCNet*)b;
  return (x->rep > y->rep) - (x->rep < y->rep);
}

/* One coarsening step (Sec. 2.3).  Candidate pairs share a net e with
   2 <= |e| <= match_max; omega(pair) = max over shared candidate nets of
   c(e)/(|e|-1).  Greedy maximal matching in decreasing priority (omega, hash,
   then smaller ids); then each unmatched vertex with exactly one candidate
   neighbour joins that neighbour's group.  Groups are numbered by their
   smallest member.  Coarse weight = sum of member weights (ascending member
   id); a net's image is the set of its members' groups; images of size < 2
   are dropped, equal images merge with summed cost (ascending net id) and
   are ordered by their smallest net id.
   Outputs: pi[k]; *kc, *lc; cptr[l+1], cpins[ptr[l]], cw[k], cc[l] (upper
   bounds on size; caller allocates). */
int o_coarsen(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
              const float* c, uint64_t seed, uint64_t comp, int32_t level, int32_t match_max,
              int32_t* pi, int32_t* kc_out, int32_t* lc_out, int64_t* cptr, int32_t* cpins,
              float* cw, float* cc) {
  /* candidate pairs */
  int64_t np = 0;
  for (int32_t e = 0; e < l; ++e) {
    int64_t s = ptr[e + 1] - ptr[e];
    if (s >= 2 && s <= match_max) np += s * (s - 1) / 2;
  }
  OPair* pr = (OPair*)malloc(sizeof(OPair) * (size_t)(np > 0 ? np : 1));
  int64_t t = 0;
  for (int32_t e = 0; e < l; ++e) {
    int64_t s = ptr[e + 1] - ptr[e];
    if (s < 2 || s > match_max) continue;
    double om = (double)(c ? c[e] : 1.0f) / (double)(s - 1);
    for (int64_t i = 0; i < s; ++i)
      for (int64_t j = i + 1; j < s; ++j) {
        pr[t].u = pins[ptr[e] + i]; pr[t].v = pins[ptr[e] + j]; pr[t].om = om; ++t;
      }
  }
  qsort(pr, (size_t)np, sizeof(OPair), cmp_pair_uv);
  int64_t nu = 0;
  for (int64_t i = 0; i < np; ++i)
    if (nu == 0 || pr[i].u != pr[nu - 1].u || pr[i].v != pr[nu - 1].v) pr[nu++] = pr[i];
  uint64_t mkey = TAG_MATCH | ((uint64_t)level << 8) | (comp << 32);
  int32_t* nbr_cnt = (int32_t*)calloc((size_t)k, sizeof(int32_t));
  int32_t* nbr_one = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int64_t i = 0; i < nu; ++i) {
    pr[i].hs = o_rng(seed, mkey, (uint64_t)pr[i].u, (uint64_t)pr[i].v);
    nbr_cnt[pr[i].u]++; nbr_one[pr[i].u] = pr[i].v;
    nbr_cnt[pr[i].v]++; nbr_one[pr[i].v] = pr[i].u;
  }
  qsort(pr, (size_t)nu, sizeof(OPair), cmp_pair_prio);
  int32_t* mate = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t v = 0; v < k; ++v) mate[v] = -1;
  for (int64_t i = 0; i < nu; ++i)
    if (mate[pr[i].u] < 0 && mate[pr[i].v] < 0) { mate[pr[i].u] = pr[i].v; mate[pr[i].v] = pr[i].u; }
  /* group roots */
  int32_t* root = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t v = 0; v < k; ++v) root[v] = mate[v] >= 0 ? (v < mate[v] ? v : mate[v]) : v;
  for (int32_t v = 0; v < k; ++v)
    if (mate[v] < 0 && nbr_cnt[v] == 1) {
      int32_t u = nbr_one[v];
      root[v] = mate[u] >= 0 ? (u < mate[u] ? u : mate[u]) : u;
    }
  int32_t* gmin = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t v = 0; v < k; ++v) gmin[v] = k;
  for (int32_t v = 0; v < k; ++v) if (v < gmin[root[v]]) gmin[root[v]] = v;
  int32_t* cid = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int32_t kc = 0;
  for (int32_t v = 0; v < k; ++v) cid[v] = -1;
  for (int32_t v = 0; v < k; ++v) if (gmin[root[v]] == v) cid[v] = kc++;
  for (int32_t v = 0; v < k; ++v) pi[v] = cid[gmin[root[v]]];
  for (int32_t g = 0; g < kc; ++g) cw[g] = 0.0f;
  for (int32_t v = 0; v < k; ++v) cw[pi[v]] = cw[pi[v]] + (w ? w[v] : 1.0f);
  /* net images */
  int32_t* img = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ptr[l] > 0 ? ptr[l] : 1));
  ONetImg* im = (ONetImg*)malloc(sizeof(ONetImg) * (size_t)(l > 0 ? l : 1));
  int32_t nim = 0;
  for (int32_t e = 0; e < l; ++e) {
    int64_t s = ptr[e + 1] - ptr[e];
    int32_t* b = img + ptr[e];
    for (int64_t i = 0; i < s; ++i) b[i] = pi[pins[ptr[e] + i]];
    qsort(b, (size_t)s, sizeof(int32_t), cmp_i32);
    int32_t u = 0;
    for (int64_t i = 0; i < s; ++i) if (u == 0 || b[i] != b[u - 1]) b[u++] = b[i];
    if (u >= 2) { im[nim].e = e; im[nim].len = u; im[nim].p = b; ++nim; }
  }
  qsort(im, (size_t)nim, sizeof(ONetImg), cmp_img);
  OCNet* cn = (OCNet*)malloc(sizeof(OCNet) * (size_t)(nim > 0 ? nim : 1));
  int32_t ncn = 0;
  for (int32_t i = 0; i < nim; ++i) {
    int same = ncn > 0 && cn[ncn - 1].len == im[i].len &&
               memcmp(cn[ncn - 1].p, im[i].p, sizeof(int32_t) * (size_t)im[i].len) == 0;
    float ce = c ? c[im[i].e] : 1.0f;
    if (same) { cn[ncn - 1].c = cn[ncn - 1].c + ce; }
    else { cn[ncn].rep = im[i].e; cn[ncn].len = im[i].len; cn[ncn].p = im[i].p; cn[ncn].c = ce; ++ncn; }
  }
  qsort(cn, (size_t)ncn, sizeof(OCNet), cmp_cnet);
  cptr[0] = 0;
  for (int32_t j = 0; j < ncn; ++j) {
    memcpy(cpins + cptr[j], cn[j].p, sizeof(int32_t) * (size_t)cn[j].len);
    cptr[j + 1] = cptr[j] + cn[j].len;
    cc[j] = cn[j].c;
  }
  *kc_out = kc; *lc_out = ncn;
  free(pr); free(nbr_cnt); free(nbr_one); free(mate); free(root); free(gmin); free(cid);
  free(img); free(im); free(cn);
  return 0;
}

/* ---- 2^d-tree ------------------------------------------------------------ */
/* Node layout in pre-order.  A node at depth L covers one cell of side
   2^(16-L) key units of a 2^16 grid over the bounding cube of the points
   (side = largest bbox side).  It is a leaf if it holds <= leaf_cap points or
   L = 16; otherwise its children are its non-empty sub-cells in Morton digit
   order.  next = index just after the node's subtree (n_nodes = end).
   Charges: W = sum of weights, X = weighted mean, both summed bottom-up in
   FP64 (leaf: its points in sorted order; internal: its children in order). */
typedef struct {
  int32_t first, count, depth, leaf, next;
  int32_t cell2[4];   /* cell centre x 2, key units */
  float W, X[4];
  double Wd, Sd[4];
} OTNode;

typedef struct {
  int32_t k, n, cap, nalloc;
  uint32_t* kq;        /* [4][k] 16-bit key coordinates, by vertex        */
  uint64_t* key;       /* [k] Morton key, by vertex                       */
  int32_t* order;      /* [k] vertices sorted by (key, id)                */
  OTNode* nd;
} OTree;

static const uint64_t* g_sort_keys;
static int cmp_by_key(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  uint64_t kx = g_sort_keys[x], ky = g_sort_keys[y];
  if (kx != ky) return kx < ky ? -1 : 1;
  return (x > y) - (x < y);
}

static int digit_of(uint64_t key, int depth) { return (int)((key >> (4 * (16 - depth))) & 15u); }

static int32_t tree_build_rec(OTree* T, int32_t first, int32_t count, int depth, const float* x,
                              const float* w) {
  if (T->n == T->nalloc) {
    T->nalloc = 2 * T->nalloc + 64;
    T->nd = (OTNode*)realloc(T->nd, sizeof(OTNode) * (size_t)T->nalloc);
  }
  int32_t me = T->n++;
  OTNode* N = &T->nd[me];
  N->first = first; N->count = count; N->depth = depth;
  int32_t side = 1 << (16 - depth);
  int32_t v0 = T->order[first];
  for (int d = 0; d < 4; ++d) {
    int32_t lo = (int32_t)((T->kq[(size_t)d * T->k + v0] >> (16 - depth)) << (16 - depth));
    if (depth == 0) lo = 0;
    N->cell2[d] = 2 * lo + side;
  }
  double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
  if (count <= T->cap || depth == 16) {
    N->leaf = 1;
    for (int32_t i = first; i < first + count; ++i) {
      int32_t v = T->order[i];
      double wv = (double)w[v];
      Wd += wv;
      for (int d = 0; d < 4; ++d) Sd[d] += wv * (double)x[(size_t)d * T->k + v];
    }
  } else {
    N->leaf = 0;
    int32_t i = first;
    while (i < first + count) {
      int dg = digit_of(T->key[T->order[i]], depth + 1);
      int32_t j = i;
      while (j < first + count && digit_of(T->key[T->order[j]], depth + 1) == dg) ++j;
      int32_t ch = tree_build_rec(T, i, j - i, depth + 1, x, w);
      Wd += T->nd[ch].Wd;
      for (int d = 0; d < 4; ++d) Sd[d] += T->nd[ch].Sd[d];
      i = j;
    }
    N = &T->nd[me];
  }
  N->Wd = Wd;
  for (int d = 0; d < 4; ++d) N->Sd[d] = Sd[d];
  N->W = (float)Wd;
  for (int d = 0; d < 4; ++d) N->X[d] = (float)(Sd[d] / Wd);
  N->next = T->n;
  return me;
}

static int otree_build(OTree* T, int32_t k, const float* x, const float* w, int32_t cap) {
  T->k = k; T->cap = cap; T->n = 0;
  T->kq = (uint32_t*)malloc(sizeof(uint32_t) * 4 * (size_t)k);
  T->key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)k);
  T->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  T->nalloc = 2 * k + 64;
  T->nd = (OTNode*)malloc(sizeof(OTNode) * (size_t)T->nalloc);
  float lo[4], hi[4];
  for (int d = 0; d < 4; ++d) {
    lo[d] = hi[d] = x[(size_t)d * k];
    for (int32_t i = 0; i < k; ++i) {
      float v = x[(size_t)d * k + i];
      if (!isfinite(v)) return -1;
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  }
  double ext = 0.0;
  for (int d = 0; d < 4; ++d) { double e = (double)hi[d] - (double)lo[d]; if (e > ext) ext = e; }
  double s = ext > 0.0 ? 65536.0 / ext : 0.0;
  for (int32_t i = 0; i < k; ++i) {
    uint64_t key = 0;
    uint32_t kq[4];
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
      if (s > 0.0) {
        double f = floor(((double)x[(size_t)d * k + i] - (double)lo[d]) * s);
        v = f >= 65535.0 ? 65535u : (uint32_t)f;
      }
      kq[d] = v;
      T->kq[(size_t)d * k + i] = v;
    }
    for (int b = 15; b >= 0; --b)
      for (int d = 0; d < 4; ++d) key = (key << 1) | ((kq[d] >> b) & 1u);
    T->key[i] = key;
    T->order[i] = i;
  }
  g_sort_keys = T->key;
  qsort(T->order, (size_t)k, sizeof(int32_t), cmp_by_key);
  tree_build_rec(T, 0, k, 0, x, w);
  return 0;
}
static void otree_free(OTree* T) { free(T->kq); free(T->key); free(T->order); free(T->nd); }

/* Exported for tree parity: node fields in pre-order.  ints[n][8] = first,
   count, depth, leaf, next, and three zeros; cell2[n][4]; flt[n][5] = W, X0..X3.
   order_out[k] = vertices in sorted order.  Returns the node count, <0 error. */
int o_tree(int32_t k, const float* x, const float* w, int32_t cap, int32_t* ints, int32_t* cell2,
           float* flt, int32_t* order_out, int32_t max_nodes) {
  OTree T;
  if (otree_build(&T, k, x, w, cap)) { otree_free(&T); return -1; }
  if (T.n > max_nodes) { otree_free(&T); return -2; }
  for (int32_t t = 0; t < T.n; ++t) {
    OTNode* N = &T.nd[t];
    int32_t* r = ints + 8 * (size_t)t;
    r[0] = N->first; r[1] = N->count; r[2] = N->depth; r[3] = N->leaf; r[4] = N->next;
    r[5] = r[6] = r[7] = 0;
    for (int d = 0; d < 4; ++d) cell2[4 * (size_t)t + d] = N->cell2[d];
    flt[5 * (size_t)t] = N->W;
    for (int d = 0; d < 4; ++d) flt[5 * (size_t)t + 1 + d] = N->X[d];
  }
  for (int32_t i = 0; i < k; ++i) order_out[i] = T.order[i];
  int32_t n = T.n;
  otree_free(&T);
  return n;
}

/* Interaction of point n with charge W at X: (d-2) W w_n |X-x|^-4 (X-x).
   The squared distance and the accumulation into y use fused multiply-adds
   (fmaf: one rounding each), the rest one rounding per operation. */
static void interact(float* y, const float* xn, float wn, const float* X, float W) {
  float dx[4];
  for (int d = 0; d < 4; ++d) dx[d] = X[d] - xn[d];
  float r2 = dx[0] * dx[0];
  r2 = fmaf(dx[1], dx[1], r2);
  r2 = fmaf(dx[2], dx[2], r2);
  r2 = fmaf(dx[3], dx[3], r2);
  if (!(r2 > 0.0f)) return;
  float num = 2.0f * W;
  num = num * wn;
  float den = r2 * r2;
  float f = num / den;
  for (int d = 0; d < 4; ++d) y[d] = fmaf(f, dx[d], y[d]);
}

static int node_far(const OTNode* N, const int32_t* p2, double th2) {
  if (!(th2 > 0.0)) return 0;
  int64_t D2 = 0;
  for (int d = 0; d < 4; ++d) { int64_t t = (int64_t)p2[d] - (int64_t)N->cell2[d]; D2 += t * t; }
  int64_t s2 = (int64_t)2 << (16 - N->depth);
  return (double)(s2 * s2) < th2 * (double)D2;
}

/* Depth-first walk: far node -> one cluster charge; near internal node ->
   its children in order; near leaf -> every other point of the leaf. */
static void walk_rec(const OTree* T, int32_t t, int32_t n, const float* xn, float wn,
                     const int32_t* p2, double th2, const float* x, const float* w, float* y, int64_t* cnt) {
  const OTNode* N = &T->nd[t];
  if (node_far(N, p2, th2)) { interact(y, xn, wn, N->X, N->W); ++*cnt; return; }
  if (!N->leaf) {
    int32_t ch = t + 1;
    while (ch != N->next) { walk_rec(T, ch, n, xn, wn, p2, th2, x, w, y, cnt); ch = T->nd[ch].next; }
    return;
  }
  for (int32_t i = N->first; i < N->first + N->count; ++i) {
    int32_t v = T->order[i];
    if (v == n) continue;
    float xv[4];
    for (int d = 0; d < 4; ++d) xv[d] = x[(size_t)d * T->k + v];
    interact(y, xn, wn, xv, w[v]);
    ++*cnt;
  }
}

/* Repulsion of point n, added to yn (STRICT order).  The walk's
   interactions are summed in two levels of parts.  A root that is a leaf or
   far from the point is a single part.  Otherwise each child c of the root
   gives one part, added to yn in child order; the part of a child that is a
   leaf or far from the point is its walk summed from zero, and the part of
   any other child is the sum, in child order and from zero, of the walks over
   its own children, each summed from zero.  The paper fixes no summation
   order; this one is frozen as the strict mode that the GPU reproduces bit
   for bit (it lets the walks over the cells of the first two levels run
   independently).  The plain evaluation of the same definition, with no
   parts, is o_gradient_plain below.  *cnt += interactions evaluated. */
static void repulsion(const OTree* T, int32_t n, const float* xn, float wn, const int32_t* p2, double th2,
                      const float* x, const float* w, float* yn, int64_t* cnt) {
  const OTNode* R = &T->nd[0];
  if (R->leaf || node_far(R, p2, th2)) {
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    walk_rec(T, 0, n, xn, wn, p2, th2, x, w, acc, cnt);
    for (int d = 0; d < 4; ++d) yn[d] = yn[d] + acc[d];
    return;
  }
  for (int32_t c1 = 1; c1 != R->next; c1 = T->nd[c1].next) {
    const OTNode* N1 = &T->nd[c1];
    float acc1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (N1->leaf || node_far(N1, p2, th2)) {
      walk_rec(T, c1, n, xn, wn, p2, th2, x, w, acc1, cnt);
    } else {
      for (int32_t c2 = c1 + 1; c2 != N1->next; c2 = T->nd[c2].next) {
        float acc2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        walk_rec(T, c2, n, xn, wn, p2, th2, x, w, acc2, cnt);
        for (int d = 0; d < 4; ++d) acc1[d] = acc1[d] + acc2[d];
      }
    }
    for (int d = 0; d < 4; ++d) yn[d] = yn[d] + acc1[d];
  }
}

/* Net centres z_j = (sum of pins) / |e_j|, pins summed in CSR order. */
static void centres(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* x, float* z) {
  for (int32_t e = 0; e < l; ++e) {
    int64_t s = ptr[e + 1] - ptr[e];
    for (int d = 0; d < 4; ++d) {
      float a = 0.0f;
      for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) a = a + x[(size_t)d * k + pins[p]];
      z[(size_t)d * l + e] = s > 0 ? a / (float)s : 0.0f;
    }
  }
}

/* Interactions evaluated by the tree walks of every gradient since the last
   reset (all levels and steps of a layout). */
static int64_t g_interactions;
void o_interactions_reset(void) { g_interactions = 0; }
int64_t o_interactions(void) { return g_interactions; }

/* Gradient (eq. 7): attraction over the vertex's nets in ascending net
   order, then the tree walk.  y is [4][k].  The per-vertex loops are
   independent (each vertex's terms and their order are its own), so they run
   on all host threads without changing a bit of the result. */
static int gradient(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
                    const float* c, const float* x, float theta, int32_t cap, float* y) {
  float* z = (float*)malloc(sizeof(float) * 4 * (size_t)(l > 0 ? l : 1));
  centres(k, l, ptr, pins, x, z);
  int64_t* dptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k + 1));
  int32_t* dp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ptr[l] > 0 ? ptr[l] : 1));
  o_dual(k, l, ptr, pins, dptr, dp);
#pragma omp parallel for schedule(static)
  for (int32_t n = 0; n < k; ++n) {
    for (int d = 0; d < 4; ++d) {
      float a = 0.0f;
      for (int64_t t = dptr[n]; t < dptr[n + 1]; ++t) {
        int32_t e = dp[t];
        float ce = c ? c[e] : 1.0f;
        float df = x[(size_t)d * k + n] - z[(size_t)d * l + e];
        a = a + ce * df;
      }
      y[(size_t)d * k + n] = a;
    }
  }
  free(z); free(dptr); free(dp);
  OTree T;
  if (otree_build(&T, k, x, w, cap)) { otree_free(&T); return -1; }
  double th2 = (double)theta * (double)theta;
  int64_t nint = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nint)
  for (int32_t n = 0; n < k; ++n) {
    float xn[4], yn[4];
    int32_t p2[4];
    for (int d = 0; d < 4; ++d) {
      xn[d] = x[(size_t)d * k + n];
      yn[d] = y[(size_t)d * k + n];
      p2[d] = 2 * (int32_t)T.kq[(size_t)d * k + n] + 1;
    }
    repulsion(&T, n, xn, w[n], p2, th2, x, w, yn, &nint);
    for (int d = 0; d < 4; ++d) y[(size_t)d * k + n] = yn[d];
  }
  g_interactions += nint;
  otree_free(&T);
  return 0;
}

/* Exported gradient for parity of the attraction/repulsion kernels. */
int o_gradient(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
               const float* c, const float* x, float theta, int32_t cap, float* y, float* z) {
  if (z) centres(k, l, ptr, pins, x, z);
  return gradient(k, l, ptr, pins, w, c, x, theta, cap, y);
}

/* First step length of a level: step0 * V^(1/4), V = volume of the bounding
   box of x (if V = 0, the largest side replaces V^(1/4)), in FP64. */
static double step_length0(int32_t k, const float* x, const o_layout_params* P) {
  float lo[4], hi[4];
  for (int d = 0; d < 4; ++d) {
    lo[d] = hi[d] = x[(size_t)d * k];
    for (int32_t i = 0; i < k; ++i) {
      float v = x[(size_t)d * k + i];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  }
  double V = 1.0, ext = 0.0;
  for (int d = 0; d < 4; ++d) {
    double e = (double)hi[d] - (double)lo[d];
    V = V * e;
    if (e > ext) ext = e;
  }
  double side = V > 0.0 ? sqrt(sqrt(V)) : ext;
  return (double)P->step0_frac * side;
}

/* One steepest-descent step (Algorithm 3).  it = step index at this level;
   *alpha carries the step length between calls: at it == 0 it is set by
   step_length0, afterwards alpha <- decay * alpha.  Each vertex is then moved
   a distance alpha against its own gradient: x_n <- x_n - (alpha / |y_n|) y_n
   (vertices with y_n = 0 stay).  Sec. 2.3 sets the step by weighing the size
   of the bounding box against the vertices' own gradients; this is read as
   the step rule of the force-directed method the paper cites (Hu 2005): a
   fixed length for every vertex, shrinking by a constant factor per step. */
int o_layout_iter(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
                  const float* c, float* x, const o_layout_params* P, int32_t it, double* alpha,
                  float* y_out) {
  float* y = (float*)malloc(sizeof(float) * 4 * (size_t)k);
  if (gradient(k, l, ptr, pins, w, c, x, P->theta, P->leaf_cap, y)) { free(y); return -1; }
  if (it == 0) *alpha = step_length0(k, x, P);
  else *alpha = *alpha * (double)P->decay;
  for (int32_t i = 0; i < k; ++i) {
    float yv[4];
    for (int d = 0; d < 4; ++d) yv[d] = y[(size_t)d * k + i];
    float n2 = yv[0] * yv[0];
    n2 = n2 + yv[1] * yv[1];
    n2 = n2 + yv[2] * yv[2];
    n2 = n2 + yv[3] * yv[3];
    if (!(n2 > 0.0f)) continue;
    float f = (float)(*alpha / sqrt((double)n2));
    for (int d = 0; d < 4; ++d) {
      float t = f * yv[d];
      x[(size_t)d * k + i] = x[(size_t)d * k + i] - t;
    }
  }
  if (y_out) memcpy(y_out, y, sizeof(float) * 4 * (size_t)k);
  free(y);
  return 0;
}

/* Random start of the coarsest level: x = (u - 1/2) k^(1/4), u a 24-bit
   uniform in [0,1). */
void o_layout_init(int32_t k, uint64_t seed, uint64_t comp, int32_t level, float* x) {
  float a = (float)sqrt(sqrt((double)k));
  uint64_t key = TAG_INIT | ((uint64_t)level << 8) | (comp << 32);
  for (int32_t v = 0; v < k; ++v)
    for (int d = 0; d < 4; ++d) {
      uint64_t r = o_rng(seed, key, (uint64_t)v, (uint64_t)d);
      float u = (float)(uint32_t)(r >> 40) * 0x1p-24f;
      x[(size_t)d * k + v] = (u - 0.5f) * a;
    }
}

/* Prolongation (Algorithm 2): x_f(v) = sigma x_c(pi(v)) + eps u, sigma =
   (k_f/k_c)^(1/4), eps = jitter * (largest side of x_c) / k_c^(1/4),
   u uniform in [-1, 1) (24-bit grid), keyed by the fine level index. */
void o_layout_prolong(int32_t kf, int32_t kc, const int32_t* pi, const float* xc, uint64_t seed,
                      uint64_t comp, int32_t flevel, float jitter, float* xf) {
  float lo[4], hi[4];
  for (int d = 0; d < 4; ++d) {
    lo[d] = hi[d] = xc[(size_t)d * kc];
    for (int32_t i = 0; i < kc; ++i) {
      float v = xc[(size_t)d * kc + i];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  }
  double ext = 0.0;
  for (int d = 0; d < 4; ++d) { double e = (double)hi[d] - (double)lo[d]; if (e > ext) ext = e; }
  float sigma = (float)sqrt(sqrt((double)kf / (double)kc));
  double epsd = (double)jitter * ext;
  float eps = (float)(epsd / sqrt(sqrt((double)kc)));
  uint64_t key = TAG_PROLONG | ((uint64_t)flevel << 8) | (comp << 32);
  for (int32_t v = 0; v < kf; ++v)
    for (int d = 0; d < 4; ++d) {
      uint64_t r = o_rng(seed, key, (uint64_t)v, (uint64_t)d);
      float u = (float)(uint32_t)(r >> 40) * 0x1p-23f;
      u = u - 1.0f;
      float a = sigma * xc[(size_t)d * kc + pi[v]];
      float b = eps * u;
      xf[(size_t)d * kf + v] = a + b;
    }
}

typedef struct { int32_t k, l; int64_t* ptr; int32_t* pins; float* w; float* c; int32_t* pi; } OLvl;

/* Multilevel layout of one connected hypergraph (Algorithm 2). */
static int layout_component(OLvl* G0, const o_layout_params* P, uint64_t comp, float* xout) {
  int32_t cap_levels = P->max_levels + 1;
  OLvl* L = (OLvl*)calloc((size_t)cap_levels, sizeof(OLvl));
  L[0] = *G0;
  int32_t J = 0;
  while (L[J].k > P->min_coarse && J < P->max_levels) {
    OLvl* F = &L[J];
    OLvl C;
    C.pi = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->k);
    C.ptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(F->l + 1));
    C.pins = (int32_t*)malloc(sizeof(int32_t) * (size_t)(F->ptr[F->l] > 0 ? F->ptr[F->l] : 1));
    C.w = (float*)malloc(sizeof(float) * (size_t)F->k);
    C.c = (float*)malloc(sizeof(float) * (size_t)(F->l > 0 ? F->l : 1));
    o_coarsen(F->k, F->l, F->ptr, F->pins, F->w, F->c, P->seed, comp, J, P->match_max_net, C.pi,
              &C.k, &C.l, C.ptr, C.pins, C.w, C.c);
    if ((double)C.k > (double)P->stall * (double)F->k) {
      free(C.pi); free(C.ptr); free(C.pins); free(C.w); free(C.c);
      break;
    }
    F->pi = C.pi;
    C.pi = NULL;
    L[J + 1] = C;
    ++J;
  }
  float* x = (float*)malloc(sizeof(float) * 4 * (size_t)L[J].k);
  o_layout_init(L[J].k, P->seed, comp, J, x);
  for (int32_t j = J; j >= 0; --j) {
    int32_t iters = j == J ? P->coarsest_iters : P->level_iters;
    double alpha = 0.0;
    for (int32_t it = 0; it < iters; ++it)
      if (o_layout_iter(L[j].k, L[j].l, L[j].ptr, L[j].pins, L[j].w, L[j].c, x, P, it, &alpha, NULL))
        return -1;
    if (j > 0) {
      float* xf = (float*)malloc(sizeof(float) * 4 * (size_t)L[j - 1].k);
      o_layout_prolong(L[j - 1].k, L[j].k, L[j - 1].pi, x, P->seed, comp, j - 1, P->jitter, xf);
      free(x);
      x = xf;
    }
  }
  memcpy(xout, x, sizeof(float) * 4 * (size_t)G0->k);
  free(x);
  for (int32_t j = 1; j <= J; ++j) { free(L[j].ptr); free(L[j].pins); free(L[j].w); free(L[j].c); free(L[j].pi); }
  free(L[0].pi);
  free(L);
  return 0;
}

/* Full layout: components (minimum-id labels, ascending), each laid out
   alone, then packed side by side along the first axis with gap
   pack_gap * (largest component side).  x is [4][k]. */
int o_layout(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
             const float* c, const o_layout_params* P, float* x) {
  int32_t* label = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  if (o_components(k, l, ptr, pins, label)) { free(label); return -1; }
  int32_t* local = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int32_t* csize = (int32_t*)calloc((size_t)k, sizeof(int32_t));
  for (int32_t v = 0; v < k; ++v) local[v] = csize[label[v]]++;
  float* xl = (float*)malloc(sizeof(float) * 4 * (size_t)k);
  /* per component layout into xl (component-local SoA blocks at offset) */
  int32_t* coff = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int32_t off = 0;
  for (int32_t v = 0; v < k; ++v) if (label[v] == v) { coff[v] = off; off += csize[v]; }
  int rc = 0;
  for (int32_t r = 0; r < k && rc == 0; ++r) {
    if (label[r] != r) continue;
    int32_t kc = csize[r];
    float* xc = xl + 4 * (size_t)coff[r];
    if (kc == 1) { for (int d = 0; d < 4; ++d) xc[d] = 0.0f; continue; }
    OLvl G;
    memset(&G, 0, sizeof G);
    G.k = kc;
    int32_t nl = 0;
    int64_t npins = 0;
    for (int32_t e = 0; e < l; ++e)
      if (ptr[e + 1] > ptr[e] && label[pins[ptr[e]]] == r) { nl++; npins += ptr[e + 1] - ptr[e]; }
    G.l = nl;
    G.ptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nl + 1));
    G.pins = (int32_t*)malloc(sizeof(int32_t) * (size_t)(npins > 0 ? npins : 1));
    G.w = (float*)malloc(sizeof(float) * (size_t)kc);
    G.c = (float*)malloc(sizeof(float) * (size_t)(nl > 0 ? nl : 1));
    G.ptr[0] = 0;
    int32_t j = 0;
    for (int32_t e = 0; e < l; ++e) {
      if (!(ptr[e + 1] > ptr[e] && label[pins[ptr[e]]] == r)) continue;
      for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) G.pins[G.ptr[j] + (p - ptr[e])] = local[pins[p]];
      G.ptr[j + 1] = G.ptr[j] + (ptr[e + 1] - ptr[e]);
      G.c[j] = c ? c[e] : 1.0f;
      ++j;
    }
    for (int32_t v = 0; v < k; ++v) if (label[v] == r) G.w[local[v]] = w ? w[v] : 1.0f;
    rc = layout_component(&G, P, (uint64_t)r, xc);
    free(G.ptr); free(G.pins); free(G.w); free(G.c);
  }
  if (rc == 0) {
    /* packing */
    double maxext = 0.0;
    for (int32_t r = 0; r < k; ++r) {
      if (label[r] != r) continue;
      int32_t kc = csize[r];
      float* xc = xl + 4 * (size_t)coff[r];
      for (int d = 0; d < 4; ++d) {
        float lo = xc[(size_t)d * kc], hi = lo;
        for (int32_t i = 0; i < kc; ++i) { float v = xc[(size_t)d * kc + i]; if (v < lo) lo = v; if (v > hi) hi = v; }
        double e = (double)hi - (double)lo;
        if (e > maxext) maxext = e;
      }
    }
    double gap = (double)P->pack_gap * maxext;
    double offx = 0.0;
    for (int32_t r = 0; r < k; ++r) {
      if (label[r] != r) continue;
      int32_t kc = csize[r];
      float* xc = xl + 4 * (size_t)coff[r];
      float lo[4];
      double ext = 0.0;
      for (int d = 0; d < 4; ++d) {
        float a = xc[(size_t)d * kc], b = a;
        for (int32_t i = 0; i < kc; ++i) { float v = xc[(size_t)d * kc + i]; if (v < a) a = v; if (v > b) b = v; }
        lo[d] = a;
        double e = (double)b - (double)a;
        if (e > ext) ext = e;
      }
      for (int32_t v = 0; v < k; ++v) {
        if (label[v] != r) continue;
        int32_t i = local[v];
        double t0 = (double)xc[i] - (double)lo[0];
        x[v] = (float)(t0 + offx);
        for (int d = 1; d < 4; ++d) x[(size_t)d * k + v] = (float)((double)xc[(size_t)d * kc + i] - (double)lo[d]);
      }
      offx = offx + ext;
      offx = offx + gap;
    }
  }
  free(label); free(local); free(csize); free(xl); free(coff);
  return rc;
}

/* Gradient at a sample of vertices (for checks at full size): y[4][ns] for
   the vertices ids[0..ns), plus the number of charge interactions each one's
   walk performed (far nodes + leaf pairs, zero-distance pairs included). */
int o_gradient_sample(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
                      const float* c, const float* x, float theta, int32_t cap, int32_t ns,
                      const int32_t* ids, float* y, int64_t* nint) {
  float* z = (float*)malloc(sizeof(float) * 4 * (size_t)(l > 0 ? l : 1));
  centres(k, l, ptr, pins, x, z);
  int64_t* dptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k + 1));
  int32_t* dp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ptr[l] > 0 ? ptr[l] : 1));
  o_dual(k, l, ptr, pins, dptr, dp);
  OTree T;
  if (otree_build(&T, k, x, w, cap)) { otree_free(&T); free(z); free(dptr); free(dp); return -1; }
  double th2 = (double)theta * (double)theta;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t s = 0; s < ns; ++s) {
    int32_t n = ids[s];
    float xn[4], yn[4];
    int32_t p2[4];
    for (int d = 0; d < 4; ++d) {
      float a = 0.0f;
      for (int64_t t = dptr[n]; t < dptr[n + 1]; ++t) {
        int32_t e = dp[t];
        float ce = c ? c[e] : 1.0f;
        float df = x[(size_t)d * k + n] - z[(size_t)d * l + e];
        a = a + ce * df;
      }
      yn[d] = a;
      xn[d] = x[(size_t)d * k + n];
      p2[d] = 2 * (int32_t)T.kq[(size_t)d * k + n] + 1;
    }
    int64_t cnt = 0;
    repulsion(&T, n, xn, w[n], p2, th2, x, w, yn, &cnt);
    for (int d = 0; d < 4; ++d) y[(size_t)d * ns + s] = yn[d];
    if (nint) nint[s] = cnt;
  }
  otree_free(&T); free(z); free(dptr); free(dp);
  return 0;
}

/* ---- plain evaluation of eq. (7) ------------------------------------------ */
/* The gradient of eq. (6) as eq. (7) states it, evaluated plainly: every
   operation in FP64 (one rounding each, no fused multiply-add), net centres
   z_e = (sum of the pins' coordinates) / |e|, the attraction
   sum_e c_e (x_n - z_e) over the vertex's nets in ascending net order, then
   the repulsion as ONE running sum per point over the depth-first walk of
   Algorithm 3 from the root: a far node adds one term with the node's charge
   W at its weighted centre X (the tree as built above: integer far test,
   theta, leaf size; charges W and X as stored), a near internal node is
   entered child by child, a near leaf adds a term for each of its other
   points.  One term is (d - 2) W w_n (X - x_n) / |X - x_n|^4 with d = 4; a
   term at zero distance is left out (the point itself, coincident points).
   Nothing here follows the GPU's division of the walk into parts.

   s (per point and coordinate) is the magnitude against which the FP32
   evaluation's rounding is measured: for each attraction term
   c_e (|x_n| + mean over the pins of |x_p|) (the operands of the centre and
   of the difference), and for each repulsion term its absolute value.  An
   FP32 evaluation of the same terms in any order differs from y by a few
   units of 2^-24 times s, times a factor that grows with the number of
   terms. */
static void plain_term(double* y, double* s, const float* xn, double wn, const float* X, double W) {
  double dx[4], r2 = 0.0;
  for (int d = 0; d < 4; ++d) {
    dx[d] = (double)X[d] - (double)xn[d];
    r2 = r2 + dx[d] * dx[d];
  }
  if (!(r2 > 0.0)) return;
  double f = 2.0 * W * wn / (r2 * r2);
  for (int d = 0; d < 4; ++d) {
    double t = f * dx[d];
    y[d] = y[d] + t;
    s[d] = s[d] + fabs(t);
  }
}

static void walk_plain(const OTree* T, int32_t t, int32_t n, const float* xn, double wn, const int32_t* p2,
                       double th2, const float* x, const float* w, double* y, double* s, int64_t* cnt) {
  const OTNode* N = &T->nd[t];
  if (node_far(N, p2, th2)) { plain_term(y, s, xn, wn, N->X, (double)N->W); ++*cnt; return; }
  if (!N->leaf) {
    for (int32_t ch = t + 1; ch != N->next; ch = T->nd[ch].next)
      walk_plain(T, ch, n, xn, wn, p2, th2, x, w, y, s, cnt);
    return;
  }
  for (int32_t i = N->first; i < N->first + N->count; ++i) {
    int32_t v = T->order[i];
    if (v == n) continue;
    float xv[4];
    for (int d = 0; d < 4; ++d) xv[d] = x[(size_t)d * T->k + v];
    plain_term(y, s, xn, wn, xv, (double)w[v]);
    ++*cnt;
  }
}

/* Plain gradient at the vertices ids[0..ns) (ids == NULL: all k, ns = k).
   y, s: [4][ns] FP64; nint (or NULL): [ns] interactions of each walk. */
int o_gradient_plain(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
                     const float* c, const float* x, float theta, int32_t cap, int32_t ns, const int32_t* ids,
                     double* y, double* s, int64_t* nint) {
  if (!ids) ns = k;
  double* z = (double*)malloc(sizeof(double) * 4 * (size_t)(l > 0 ? l : 1));
  double* za = (double*)malloc(sizeof(double) * 4 * (size_t)(l > 0 ? l : 1));
  for (int32_t e = 0; e < l; ++e) {
    double sz = (double)(ptr[e + 1] - ptr[e]);
    for (int d = 0; d < 4; ++d) {
      double a = 0.0, b = 0.0;
      for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) {
        double v = (double)x[(size_t)d * k + pins[p]];
        a = a + v;
        b = b + fabs(v);
      }
      z[(size_t)d * l + e] = sz > 0.0 ? a / sz : 0.0;
      za[(size_t)d * l + e] = sz > 0.0 ? b / sz : 0.0;
    }
  }
  int64_t* dptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k + 1));
  int32_t* dp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ptr[l] > 0 ? ptr[l] : 1));
  o_dual(k, l, ptr, pins, dptr, dp);
  OTree T;
  if (otree_build(&T, k, x, w, cap)) { otree_free(&T); free(z); free(za); free(dptr); free(dp); return -1; }
  double th2 = (double)theta * (double)theta;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < ns; ++i) {
    int32_t n = ids ? ids[i] : i;
    double yn[4], sn[4];
    float xn[4];
    int32_t p2[4];
    for (int d = 0; d < 4; ++d) {
      double xv = (double)x[(size_t)d * k + n];
      double a = 0.0, b = 0.0;
      for (int64_t t = dptr[n]; t < dptr[n + 1]; ++t) {
        int32_t e = dp[t];
        double ce = c ? (double)c[e] : 1.0;
        a = a + ce * (xv - z[(size_t)d * l + e]);
        b = b + ce * (fabs(xv) + za[(size_t)d * l + e]);
      }
      yn[d] = a;
      sn[d] = b;
      xn[d] = x[(size_t)d * k + n];
      p2[d] = 2 * (int32_t)T.kq[(size_t)d * k + n] + 1;
    }
    int64_t cnt = 0;
    walk_plain(&T, 0, n, xn, (double)w[n], p2, th2, x, w, yn, sn, &cnt);
    for (int d = 0; d < 4; ++d) {
      y[(size_t)d * ns + i] = yn[d];
      s[(size_t)d * ns + i] = sn[d];
    }
    if (nint) nint[i] = cnt;
  }
  otree_free(&T); free(z); free(za); free(dptr); free(dp);
  return 0;
}

/* One descent step (Algorithm 3) with the plain gradient: the step length is
   set as in o_layout_iter, and each vertex moves by it along -y_n/|y_n| in
   FP64, the new coordinates rounded to FP32.  y_out (or NULL): [4][k] FP64,
   s_out (or NULL): the magnitudes of o_gradient_plain. */
int o_layout_iter_plain(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
                        const float* c, float* x, const o_layout_params* P, int32_t it, double* alpha,
                        double* y_out, double* s_out) {
  double* y = (double*)malloc(sizeof(double) * 4 * (size_t)k);
  double* s = (double*)malloc(sizeof(double) * 4 * (size_t)k);
  if (o_gradient_plain(k, l, ptr, pins, w, c, x, P->theta, P->leaf_cap, k, NULL, y, s, NULL)) {
    free(y); free(s);
    return -1;
  }
  if (it == 0) *alpha = step_length0(k, x, P);
  else *alpha = *alpha * (double)P->decay;
  for (int32_t i = 0; i < k; ++i) {
    double n2 = 0.0;
    for (int d = 0; d < 4; ++d) n2 = n2 + y[(size_t)d * k + i] * y[(size_t)d * k + i];
    if (!(n2 > 0.0)) continue;
    double f = *alpha / sqrt(n2);
    for (int d = 0; d < 4; ++d)
      x[(size_t)d * k + i] = (float)((double)x[(size_t)d * k + i] - f * y[(size_t)d * k + i]);
  }
  if (y_out) memcpy(y_out, y, sizeof(double) * 4 * (size_t)k);
  if (s_out) memcpy(s_out, s, sizeof(double) * 4 * (size_t)k);
  free(y); free(s);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Strengthened diagonal [Sec. 4.2, permutations with a perfect bipartite
   matching; Sec. 5, a heavy edge matching of the bipartite representation
   augmented to a perfect matching by Hopcroft-Karp].  The bipartite graph of
   an m x n pattern has rows 0..m-1 and columns m..m+n-1; nonzero e = (i, j)
   is the edge {i, m + j}.  mrow[i] = the column matched to row i or -1,
   mcol[j] = the row matched to column j or -1. */

/* MurmurHash3's 32-bit finalizer (Appleby): a bijection of 32-bit words. */
static uint32_t o_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

/* Priority of nonzero e: the bits of |a_e| (of 1.0 when a is NULL) above the
   scrambled index fmix32(e + seed).  Non-negative floats order as their bits,
   and the low word is a bijection of e, so no two nonzeros tie. */
uint64_t o_match_key(const float* a, int64_t e, uint32_t seed) {
  const float w = a ? fabsf(a[e]) : 1.0f;
  uint32_t wb;
  memcpy(&wb, &w, 4);
  return ((uint64_t)wb << 32) | o_fmix32((uint32_t)e + seed);
}

static const uint64_t* g_match_keys;
static int cmp_key_desc(const void* pa, const void* pb) {
  const uint64_t a = g_match_keys[*(const int64_t*)pa], b = g_match_keys[*(const int64_t*)pb];
  return a < b ? 1 : (a > b ? -1 : 0);
}

/* Heavy edge matching: nonzeros visited by decreasing priority, each taken
   when its row and its column are both free.  Returns the matching size, or
   -1 for bad input (a value not finite). */
int64_t o_match_heavy(int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* a,
                      uint32_t seed, int32_t* mrow, int32_t* mcol) {
  const int64_t nnz = rowptr[m];
  if (a)
    for (int64_t e = 0; e < nnz; ++e)
      if (!isfinite(a[e])) return -1;
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  int32_t* row = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  for (int32_t i = 0; i < m; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) row[e] = i;
  for (int64_t e = 0; e < nnz; ++e) { key[e] = o_match_key(a, e, seed); idx[e] = e; }
  g_match_keys = key;
  qsort(idx, (size_t)nnz, sizeof(int64_t), cmp_key_desc);
  for (int32_t i = 0; i < m; ++i) mrow[i] = -1;
  for (int32_t j = 0; j < n; ++j) mcol[j] = -1;
  int64_t size = 0;
  for (int64_t t = 0; t < nnz; ++t) {
    const int64_t e = idx[t];
    const int32_t i = row[e], j = col[e];
    if (mrow[i] < 0 && mcol[j] < 0) { mrow[i] = j; mcol[j] = i; ++size; }
  }
  free(key); free(idx); free(row);
  return size;
}

/* Hopcroft-Karp: each phase layers the rows by breadth-first search from the
   free rows (ascending) along alternating paths, then takes vertex-disjoint
   shortest augmenting paths by depth-first search from every free row in
   ascending order, columns in row order; phases repeat until no augmenting
   path is left.  Returns the final matching size. */
typedef struct {
  const int64_t* rowptr; const int32_t* col;
  int32_t *mrow, *mcol, *dist; int64_t* it; int32_t found;
} OHK;
#define HK_INF 0x7fffffff
static int hk_dfs(OHK* H, int32_t u) {
  for (; H->it[u] < H->rowptr[u + 1]; ++H->it[u]) {
    const int32_t j = H->col[H->it[u]], r = H->mcol[j];
    int ok;
    if (r < 0) ok = H->dist[u] + 1 == H->found;
    else ok = H->dist[r] == H->dist[u] + 1 && hk_dfs(H, r);
    if (ok) { H->mrow[u] = j; H->mcol[j] = u; ++H->it[u]; return 1; }
  }
  H->dist[u] = HK_INF;
  return 0;
}
int64_t o_match_augment(int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, int32_t* mrow,
                        int32_t* mcol) {
  OHK H;
  H.rowptr = rowptr; H.col = col; H.mrow = mrow; H.mcol = mcol;
  H.dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  H.it = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  for (;;) {
    int32_t qh = 0, qt = 0;
    for (int32_t i = 0; i < m; ++i) {
      H.dist[i] = HK_INF;
      if (mrow[i] < 0) { H.dist[i] = 0; queue[qt++] = i; }
    }
    H.found = HK_INF;
    while (qh < qt) {
      const int32_t u = queue[qh++];
      if (H.dist[u] >= H.found) continue;
      for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) {
        const int32_t r = mcol[col[p]];
        if (r < 0) { if (H.dist[u] + 1 < H.found) H.found = H.dist[u] + 1; }
        else if (H.dist[r] == HK_INF) { H.dist[r] = H.dist[u] + 1; queue[qt++] = r; }
      }
    }
    if (H.found == HK_INF) break;
    for (int32_t i = 0; i < m; ++i) H.it[i] = rowptr[i];
    for (int32_t i = 0; i < m; ++i)
      if (mrow[i] < 0 && H.dist[i] == 0) hk_dfs(&H, i);
  }
  int64_t size = 0;
  for (int32_t i = 0; i < m; ++i) size += mrow[i] >= 0;
  (void)n;
  free(H.dist); free(H.it); free(queue);
  return size;
}

/* Row and column permutations of a square matrix from an ordering of its
   bipartite graph with a perfect strengthened diagonal mu: the rows in the
   order they appear in vperm, and the column matched to each (so the matching
   lies on the diagonal and every diagonal block is square).  Returns -1 if a
   row has no partner column. */
int o_matched_perms(int32_t m, const int32_t* vperm, const int32_t* mu, int32_t* rperm, int32_t* cperm) {
  int32_t t = 0;
  for (int32_t p = 0; p < 2 * m; ++p) {
    const int32_t v = vperm[p];
    if (v >= m) continue;
    if (mu[v] < m || mu[v] >= 2 * m || t >= m) return -1;
    rperm[t] = v;
    cperm[t] = mu[v] - m;
    ++t;
  }
  return t == m ? 0 : -1;
}

/* Finegrain coordinates [Sec. 4.2: each nonzero at the average of the points
   of its row and its column in a layout of the bipartite graph]: x holds
   m + n points (rows, then columns), [4][m+n]; xnz[d][e] for nonzero e. */
void o_finegrain(int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* x, float* xnz) {
  const size_t k = (size_t)m + (size_t)n, nnz = (size_t)rowptr[m];
  for (int32_t i = 0; i < m; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      for (int d = 0; d < 4; ++d)
        xnz[d * nnz + (size_t)e] = (x[d * k + (size_t)i] + x[d * k + (size_t)m + (size_t)col[e]]) * 0.5f;
}

/* ------------------------------------------------------------------------- */
/* Kernighan-Lin refinement [Sec. 3, the remark that partitionings made by
   Algorithm 4 improve under a few Kernighan-Lin iterations; Kernighan and Lin
   1970].  Graph mode (every net an edge {v, w}); every edge weighs 1, so
   parallel edges add up.  label[v] = 2 g + s puts v on side s (0 = A, 1 = B)
   of bisection g; label -1 leaves v out.  Each bisection is refined on its
   own, only edges inside it counting.  One pass: D(v) = (edges to the other
   side) - (edges to its own side); then min(|A|, |B|) times the unlocked pair
   (a in A, b in B) of largest gain D(a) + D(b) - 2 m(a, b) (m = edges joining
   them) is chosen, ties to the smallest a, then the smallest b; both are
   locked and the D of the unlocked vertices updated as if they had swapped.
   With G(j) the sum of the first j gains and j* the smallest j of largest
   G(j), the first j* pairs are swapped if G(j*) > 0, else the bisection is
   done.  At most `passes` passes.  gain[g] = the cut reduction (edges) of
   bisection g over all passes.  Returns -1 for bad input. */
static int32_t kl_mult(const int64_t* aptr, const int32_t* adj, int32_t a, int32_t b) {
  int32_t m = 0;
  for (int64_t p = aptr[a]; p < aptr[a + 1]; ++p) m += adj[p] == b;
  return m;
}
int o_refine_kl(int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, int32_t* label, int32_t passes,
                int64_t* gain) {
  if (k < 1 || l < 0 || passes < 0) return -1;
  for (int32_t e = 0; e < l; ++e)
    if (ptr[e + 1] - ptr[e] != 2 || pins[ptr[e]] >= pins[ptr[e] + 1] || pins[ptr[e]] < 0 || pins[ptr[e] + 1] >= k)
      return -1;
  int32_t G = 0;
  for (int32_t v = 0; v < k; ++v) {
    if (label[v] < -1) return -1;
    if (label[v] / 2 + 1 > G) G = label[v] / 2 + 1;
  }
  /* adjacency: the other end of every incident edge, edges in ascending order */
  int64_t* aptr = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
  int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (2 * (size_t)l + 1));
  for (int32_t e = 0; e < l; ++e) { aptr[pins[2 * e] + 1]++; aptr[pins[2 * e + 1] + 1]++; }
  for (int32_t v = 0; v < k; ++v) aptr[v + 1] += aptr[v];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  for (int32_t v = 0; v < k; ++v) fill[v] = aptr[v];
  for (int32_t e = 0; e < l; ++e) {
    const int32_t a = pins[2 * e], b = pins[2 * e + 1];
    adj[fill[a]++] = b;
    adj[fill[b]++] = a;
  }
  int64_t* D = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  char* locked = (char*)malloc((size_t)k);
  int32_t* mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int32_t* pa = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int32_t* pb = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int64_t* pg = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  for (int32_t g = 0; g < G; ++g) {
    gain[g] = 0;
    int32_t n = 0, nA = 0, nB = 0;
    for (int32_t v = 0; v < k; ++v)
      if (label[v] >= 0 && label[v] / 2 == g) {
        mem[n++] = v;
        if (label[v] % 2 == 0) ++nA; else ++nB;
      }
    const int32_t steps = nA < nB ? nA : nB;
    for (int32_t pass = 0; pass < passes && steps > 0; ++pass) {
      for (int32_t i = 0; i < n; ++i) {
        const int32_t v = mem[i];
        locked[v] = 0;
        D[v] = 0;
        for (int64_t p = aptr[v]; p < aptr[v + 1]; ++p) {
          const int32_t w = adj[p];
          if (label[w] < 0 || label[w] / 2 != g) continue;
          D[v] += (label[w] % 2 != label[v] % 2) ? 1 : -1;
        }
      }
      for (int32_t st = 0; st < steps; ++st) {
        int64_t best = INT64_MIN;
        int32_t ba = -1, bb = -1;
        for (int32_t i = 0; i < n; ++i) {
          const int32_t a = mem[i];
          if (locked[a] || label[a] % 2 != 0) continue;
          for (int32_t j = 0; j < n; ++j) {
            const int32_t b = mem[j];
            if (locked[b] || label[b] % 2 != 1) continue;
            const int64_t gv = D[a] + D[b] - 2 * (int64_t)kl_mult(aptr, adj, a, b);
            if (gv > best) { best = gv; ba = a; bb = b; }  /* ascending a, then b: first of equals wins */
          }
        }
        locked[ba] = locked[bb] = 1;
        pa[st] = ba; pb[st] = bb; pg[st] = best;
        /* D of the unlocked members as if ba (A -> B) and bb (B -> A) swapped */
        for (int s = 0; s < 2; ++s) {
          const int32_t x = s == 0 ? ba : bb;  /* x leaves side label[x] % 2 */
          for (int64_t p = aptr[x]; p < aptr[x + 1]; ++p) {
            const int32_t w = adj[p];
            if (label[w] < 0 || label[w] / 2 != g || locked[w]) continue;
            D[w] += (label[w] % 2 == label[x] % 2) ? 2 : -2;
          }
        }
      }
      int64_t run = 0, bestG = INT64_MIN;
      int32_t jstar = 0;
      for (int32_t st = 0; st < steps; ++st) {
        run += pg[st];
        if (run > bestG) { bestG = run; jstar = st + 1; }
      }
      if (bestG <= 0) break;
      for (int32_t st = 0; st < jstar; ++st) {
        label[pa[st]] = 2 * g + 1;
        label[pb[st]] = 2 * g;
      }
      gain[g] += bestG;
    }
  }
  free(aptr); free(adj); free(fill); free(D); free(locked); free(mem); free(pa); free(pb); free(pg);
  return 0;
}
