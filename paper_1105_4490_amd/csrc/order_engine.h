// Segmented ordering engine shared by vmo_bisect, vmo_order and the batch and
// serving entry points.
#pragma once

#include <cstring>

#include "vmo_internal.h"

namespace vmo {

// Per-job constants, device resident.
struct JobDev {
  int64_t voff;        // first position / global vertex index of the job
  int32_t k, P;
  int32_t mode, ord;
  uint64_t seed, job_index;
  int64_t node_base;   // node-table offset (4P entries, indexed by heap id)
  float lo[4];         // quantization origin (exact FP32 minima)
  double scale;        // (2^20 - 1) / largest bounding-box side
  int64_t eoff;        // first edge (graph mode)
  int64_t noff;        // first net (net mode)
  int32_t nnets;
  int32_t pin_vadd;    // net mode: added to nets_pins[] to give global vertex ids
  // bases of this job in the index spaces of one emission call (vertices,
  // tree nodes, nets): a subset of jobs is emitted over the concatenation of
  // their ranges
  int64_t vk0, vn0, ve0;
  // net mode: the job's nets (pins of net u at nets_pins[nets_ptr[u] ..
  // nets_ptr[u + 1]]): the caller's arrays in a call, the arena in serving
  const int64_t* nets_ptr;
  const int32_t* nets_pins;
};

struct JobHost {
  vmo_hypergraph h;
  int32_t mode, order;
  const float* x;
  int32_t P;
  uint64_t seed, job_index;
  vmo_order_out out;
  const int32_t* mu;  // graph mode: strengthened diagonal (partner or -1), local ids; NULL = none
};

struct OutPtrs {
  int32_t* vperm;
  int32_t* nperm;
  int32_t* part;
  int32_t* node_heap;
  int32_t* node_vptr;
  int32_t* node_nptr;
  double* split_cut;
  int32_t* n_nodes;
};

enum : int32_t { kStIter = 0, kStDone = 1, kStLeaf = 2 };
enum : int32_t { kNodeNone = 0, kNodeLeaf = 1, kNodeInternal = 2, kNodePending = 3 };
// segment accumulators: sums of q (4), side-1 sums (4), side-1 count,
// changed count
constexpr int kAccF = 12, kAccTot = 0, kAccS1 = 4;

struct SegArrays {
  int64_t *beg, *end;
  int32_t *job, *h, *K, *p0, *state, *iters;
  int64_t* i1;
  int64_t* acc;
  double* plane;  // [5] r0..r3, delta
  double* cen;    // [8] c1, c2 (grid units)
};

struct SegBufs {
  Buf<int64_t> beg, end;
  Buf<int32_t> job, h, K, p0, state, iters;
  Buf<int64_t> i1, acc;
  Buf<double> plane, cen;
  int64_t cap = 0;
};

struct NodeArrays {
  int32_t *state, *K, *p0;
  int64_t *beg, *end;
};

class Engine {
 public:
  Engine(Ctx& c, hipStream_t s) : c(c), s(s) {}
  void setup(const std::vector<JobHost>& jobs);
  // jpins[j]: net_ptr[l] of job j (its pin count)
  void set_edges(const std::vector<JobHost>& jobs, const std::vector<int64_t>& jpins);
  void run_levels(int t_max, bool plain);
  void finish(const std::vector<JobHost>& jobs);
  // emission for the jobs `slots` of the job table (their work is done)
  void emit(const std::vector<int32_t>& slots, const std::vector<JobHost>& jobs);
  // k-means++ seeding and Lloyd iterations of segments [s0, s0+Sn) over
  // positions [p0, p1); tuned: the assignment's block size comes from the
  // context's online tuner (else 256)
  void two_means(int64_t s0, int64_t Sn, int64_t p0, int64_t p1, int t_max, bool tuned);

  Ctx& c;
  hipStream_t s;
  int32_t nj = 0;
  std::vector<JobDev> hj;
  Buf<JobDev> dj;
  int64_t N = 0, Np = 0, NT = 0, E = 0, L = 0, S = 0, npins_ = 0;
  Buf<uint32_t> q, q2;
  Buf<int32_t> id, id2, pos, segpos;
  Buf<int32_t> segpack;  // per aligned group of four positions: their shared segment (k_segpos)
  Buf<uint8_t> side;
  SegBufs cur;
  Buf<int32_t> nd_state, nd_K, nd_p0;
  Buf<int64_t> nd_beg, nd_end;
  Buf<int32_t> edges, npins_buf;
  Buf<int32_t> mu_g;  // partners in global vertex ids (-1: none), when a job has a strengthened diagonal
  bool has_mu = false;
  Buf<int64_t> nptr, jnoff;

  SegArrays view(SegBufs& b);
  NodeArrays nodes();

  // serving: fixed arenas, jobs admitted into ranges, one level per tick
  void arena_init(int64_t max_v, int64_t max_nodes, int64_t max_edges, int64_t max_nets, int64_t max_pins,
                  int32_t max_jobs);
  void arena_admit(int32_t slot, const JobHost& h, int64_t voff, int64_t node_base, int64_t eoff, int64_t noff,
                   int64_t pinoff);
  void arena_release(int32_t slot);
  void tick(int t_max);
  std::vector<int32_t> segment_jobs();

 private:
  void alloc_segments(SegBufs& b, int64_t cap);
  void copy_segments(SegBufs& a, SegBufs& b, int64_t n);
  void separator(int64_t s0, int64_t Sn, int64_t p0, int64_t p1, int64_t e0, int64_t e1);
  int64_t partition(int64_t s0, int64_t Sn, int64_t p0, int64_t p1, SegBufs& nx, int64_t t0);
  void launch_offset_copy_i32(const int32_t* in, int32_t* out, int64_t n, int32_t add);
  void launch_offset_copy_ptr(const int64_t* in, int64_t* out, int64_t n, int64_t add);
  void append_root(int32_t slot);
};

// bisect output helpers (order.hip)
void bisect_outputs(Engine& e, uint8_t* side, float* centres, int split);

}  // namespace vmo
