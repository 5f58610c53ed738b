// Schur-complement recursion (Sec. 4.2, the recursion on G3 = (V3, E'3)):
// every separator block of an ordering result with at least two vertices is
// reordered by the graph-mode BBD ordering (Algorithm 7) of the graph its
// vertices induce, with their own coordinates and P3 parts.  The induced graph
// of a block lists its vertices in block order (local id = position in the
// block) and the edges with both ends in the block in net order, the smaller
// local end first; its random draws are keyed by the heap id of the block's
// node as the job index.  With a strengthened diagonal mu, each block's job
// gets mu restricted to the block (partners outside it dropped), so matched
// pairs also stay together in the Schur complement.  One level of recursion:
// the result's own separator blocks are left as they come.
//
// All blocks are ordered together, as one batch of jobs of the ordering
// engine: a device pass marks the separator blocks, the vertices of each block
// get their local ids and their coordinates gathered per job, the edges inside
// blocks are grouped by block with one stable radix sort (net order kept), and
// the results are composed back into the outer order.
#include "order_engine.h"

namespace vmo {

constexpr int kST = 256;

static unsigned ssz(int64_t n) {
  int64_t b = (n + kST - 1) / kST;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}
#define SC_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// sep[r] = 1 for a block with >= 2 vertices whose first vertex is a separator
// vertex (part >= P).
__global__ void k_sc_mark(const int32_t* vperm, const int32_t* part, const int32_t* node_vptr, int32_t nn,
                          int32_t P, int32_t* sep) {
  SC_STRIDE(r, nn) {
    const int32_t lo = node_vptr[r], hi = node_vptr[r + 1];
    sep[r] = (hi - lo >= 2 && part[vperm[lo]] >= P) ? 1 : 0;
  }
}

// Block rank of position i: the last r with node_vptr[r] <= i.
__device__ __forceinline__ int32_t sc_rank(const int32_t* node_vptr, int32_t nn, int64_t i) {
  int32_t lo = 0, hi = nn;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (node_vptr[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Per position: the job of its block (-1 for blocks that stay), the vertex's
// local id and job, and its coordinates in the job's [4][m] array.
__global__ void k_sc_verts(const int32_t* vperm, const int32_t* node_vptr, int32_t nn, int32_t k,
                           const int32_t* job_of, const int64_t* jbase, const float* x, int32_t* loc, int32_t* vjob,
                           float* xs) {
  SC_STRIDE(i, k) {
    const int32_t r = sc_rank(node_vptr, nn, i);
    const int32_t j = job_of[r], v = vperm[i];
    vjob[v] = j;
    if (j < 0) continue;
    const int32_t lo = node_vptr[r], m = node_vptr[r + 1] - lo, t = (int32_t)i - lo;
    loc[v] = t;
    float* xj = xs + 4 * jbase[j];
    for (int d = 0; d < 4; ++d) xj[(int64_t)d * m + t] = x[(int64_t)d * k + v];
  }
}

// The strengthened diagonal of each job in local ids.
__global__ void k_sc_mu(const int32_t* vperm, const int32_t* node_vptr, int32_t nn, int32_t k, const int32_t* job_of,
                        const int64_t* jbase, const int32_t* mu, const int32_t* loc, const int32_t* vjob,
                        int32_t* mu3) {
  SC_STRIDE(i, k) {
    const int32_t r = sc_rank(node_vptr, nn, i);
    const int32_t j = job_of[r];
    if (j < 0) continue;
    const int32_t w = mu[vperm[i]];
    mu3[jbase[j] + (i - node_vptr[r])] = (w >= 0 && vjob[w] == j) ? loc[w] : -1;
  }
}

// Edge e goes to job j when both ends lie in j's block (key j, counted), else
// to the end of the order (key nb).
__global__ void k_sc_edge_keys(const int32_t* pins, int32_t l, const int32_t* vjob, int32_t nb, uint32_t* key,
                               int32_t* val, int32_t* count) {
  SC_STRIDE(e, l) {
    const int32_t ja = vjob[pins[2 * e]], jb = vjob[pins[2 * e + 1]];
    const bool in = ja >= 0 && ja == jb;
    key[e] = in ? (uint32_t)ja : (uint32_t)nb;
    val[e] = (int32_t)e;
    if (in) atomicAdd(&count[ja], 1);
  }
}

// The induced edges in local ids, smaller end first; edges [0, L3) of the
// sorted order are the ones inside blocks, grouped by job in net order.
__global__ void k_sc_pins(const int32_t* pins, const int32_t* val, int64_t L3, const int32_t* loc, int32_t* pins3) {
  SC_STRIDE(t, L3) {
    const int32_t e = val[t];
    const int32_t a = loc[pins[2 * e]], b = loc[pins[2 * e + 1]];
    pins3[2 * t] = a < b ? a : b;
    pins3[2 * t + 1] = a < b ? b : a;
  }
}

// Edge pointers of job j (one block per job): 2t for t in [0, count].
__global__ void k_sc_ptr(const int64_t* pbase, const int32_t* count, int64_t* ptr3) {
  const int32_t j = blockIdx.x;
  int64_t* p = ptr3 + pbase[j];
  for (int32_t t = threadIdx.x; t <= count[j]; t += blockDim.x) p[t] = 2 * (int64_t)t;
}

// Composition: position lo + t of a reordered block takes the outer vertex at
// position lo + v3[t] of the same block; other positions keep theirs.
__global__ void k_sc_compose(const int32_t* vperm, const int32_t* node_vptr, int32_t nn, int32_t k,
                             const int32_t* job_of, const int64_t* jbase, const int32_t* v3, int32_t* out) {
  SC_STRIDE(i, k) {
    const int32_t r = sc_rank(node_vptr, nn, i);
    const int32_t j = job_of[r];
    if (j < 0) {
      out[i] = vperm[i];
    } else {
      const int32_t lo = node_vptr[r];
      out[i] = vperm[lo + v3[jbase[j] + (i - lo)]];
    }
  }
}

void validate_mu(Ctx& c, const vmo_hypergraph* h, const int32_t* mu, hipStream_t s);

void order_schur(Ctx& c, const vmo_hypergraph* h, const float* x, const int32_t* mu, const vmo_order_out* in,
                 int32_t P, int32_t P3, uint64_t seed, int32_t t_max, int32_t* vperm_out, hipStream_t s) {
  VMO_REQUIRE(vperm_out != nullptr, "vperm_out is NULL");
  VMO_REQUIRE(P3 >= 1 && P3 <= (1 << 24), "P3 must be in [1, 2^24]");
  VMO_REQUIRE(t_max >= 0, "t_max must be >= 0");
  std::vector<int64_t> npins;
  validate_jobs(c, {JobCheck{h, x, true, true}}, npins, s);
  if (mu) validate_mu(c, h, mu, s);
  const int32_t k = h->k, l = h->l;
  const int32_t nn = check_ordering(c, k, P, in, s);
  // the separator blocks, on the host
  std::vector<int32_t> vptr(nn + 1), heap(nn), sep(nn);
  {
    Buf<int32_t> dsep(c.pool, nn);
    VMO_LAUNCH(k_sc_mark, ssz(nn), kST, 0, s, in->vperm, in->part, in->node_vptr, nn, P, dsep.p);
    VMO_HIP(hipMemcpyAsync(vptr.data(), in->node_vptr, sizeof(int32_t) * (nn + 1), hipMemcpyDeviceToHost, s));
    VMO_HIP(hipMemcpyAsync(heap.data(), in->node_heap, sizeof(int32_t) * nn, hipMemcpyDeviceToHost, s));
    VMO_HIP(hipMemcpyAsync(sep.data(), dsep.p, sizeof(int32_t) * nn, hipMemcpyDeviceToHost, s));
    VMO_HIP(hipStreamSynchronize(s));
  }
  std::vector<int32_t> job_of(nn, -1), jrank;
  std::vector<int64_t> jbase;
  int64_t M = 0;
  for (int32_t r = 0; r < nn; ++r) {
    if (!sep[r] || P3 == 1) continue;  // with one part the block keeps its order
    job_of[r] = (int32_t)jrank.size();
    jrank.push_back(r);
    jbase.push_back(M);
    M += vptr[r + 1] - vptr[r];
  }
  const int32_t nb = (int32_t)jrank.size();
  if (nb == 0) {
    VMO_HIP(hipMemcpyAsync(vperm_out, in->vperm, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, s));
    return;
  }
  const int64_t nper = 4 * (int64_t)P3;
  VMO_REQUIRE(nb * (nper + 1) < (int64_t(1) << 31), "too many tree nodes over the separator blocks");
  Buf<int32_t> djob(c.pool, nn);
  Buf<int64_t> djbase(c.pool, nb);
  VMO_HIP(hipMemcpyAsync(djob.p, job_of.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(djbase.p, jbase.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, s));
  // local ids, jobs and gathered coordinates
  Buf<int32_t> loc(c.pool, k), vjob(c.pool, k);
  Buf<float> xs(c.pool, 4 * M);
  VMO_LAUNCH(k_sc_verts, ssz(k), kST, 0, s, in->vperm, in->node_vptr, nn, k, djob.p, djbase.p, x, loc.p, vjob.p,
             xs.p);
  Buf<int32_t> mu3;
  if (mu) {
    mu3 = Buf<int32_t>(c.pool, M);
    VMO_LAUNCH(k_sc_mu, ssz(k), kST, 0, s, in->vperm, in->node_vptr, nn, k, djob.p, djbase.p, mu, loc.p, vjob.p,
               mu3.p);
  }
  // induced edges grouped by job, net order kept
  Buf<int32_t> count(c.pool, nb);
  fill_i32(count.p, 0, nb, s);
  std::vector<int32_t> hcount(nb);
  Buf<int32_t> val(c.pool, l > 0 ? l : 1);
  if (l > 0) {
    Buf<uint32_t> key(c.pool, l);
    VMO_LAUNCH(k_sc_edge_keys, ssz(l), kST, 0, s, h->pins, l, vjob.p, nb, key.p, val.p, count.p);
    radix_sort<uint32_t>(c, key.p, val.p, l, bits_for((uint64_t)nb), s);
  }
  VMO_HIP(hipMemcpyAsync(hcount.data(), count.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> ebase(nb), pbase(nb);
  int64_t L3 = 0;
  for (int32_t j = 0; j < nb; ++j) {
    ebase[j] = L3;
    pbase[j] = L3 + j;
    L3 += hcount[j];
  }
  Buf<int32_t> pins3(c.pool, 2 * (L3 > 0 ? L3 : 1));
  Buf<int64_t> ptr3(c.pool, L3 + nb), dpbase(c.pool, nb);
  if (L3 > 0) VMO_LAUNCH(k_sc_pins, ssz(L3), kST, 0, s, h->pins, val.p, L3, loc.p, pins3.p);
  VMO_HIP(hipMemcpyAsync(dpbase.p, pbase.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, s));
  VMO_LAUNCH(k_sc_ptr, (unsigned)nb, kST, 0, s, dpbase.p, count.p, ptr3.p);
  // one ordering job per block
  Buf<int32_t> v3(c.pool, M), p3(c.pool, M), heap3(c.pool, nb * nper), vptr3(c.pool, nb * (nper + 1)),
      nn3(c.pool, nb);
  Buf<double> sc3(c.pool, nb * nper);
  std::vector<JobHost> jobs(nb);
  std::vector<int64_t> jp(nb);
  for (int32_t j = 0; j < nb; ++j) {
    const int32_t r = jrank[j];
    JobHost& J = jobs[j];
    memset(&J, 0, sizeof J);
    J.h.k = vptr[r + 1] - vptr[r];
    J.h.l = hcount[j];
    J.h.net_ptr = ptr3.p + pbase[j];
    J.h.pins = pins3.p + 2 * ebase[j];
    J.mode = VMO_GRAPH;
    J.order = VMO_BBD;
    J.x = xs.p + 4 * jbase[j];
    J.P = P3;
    J.seed = seed;
    J.job_index = (uint64_t)heap[r];
    J.out.vperm = v3.p + jbase[j];
    J.out.part = p3.p + jbase[j];
    J.out.node_heap = heap3.p + nper * j;
    J.out.node_vptr = vptr3.p + (nper + 1) * j;
    J.out.split_cut = sc3.p + nper * j;
    J.out.n_nodes = nn3.p + j;
    J.mu = mu ? mu3.p + jbase[j] : nullptr;
    jp[j] = 2 * (int64_t)hcount[j];
  }
  Engine e(c, s);
  e.setup(jobs);
  e.set_edges(jobs, jp);
  e.run_levels(t_max, false);
  e.finish(jobs);
  // composition (through a buffer of its own: vperm_out may be in->vperm)
  Buf<int32_t> outb(c.pool, k);
  VMO_LAUNCH(k_sc_compose, ssz(k), kST, 0, s, in->vperm, in->node_vptr, nn, k, djob.p, djbase.p, v3.p, outb.p);
  VMO_HIP(hipMemcpyAsync(vperm_out, outb.p, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, s));
}

}  // namespace vmo
