// Recursive SBD/BBD ordering on the GPU: quantization, segmented k-means++
// seeding and Lloyd iterations (Algorithm 4 with m = 2), the plane and
// separator of Algorithm 7, the stable three-way partition of every split,
// and the emission of permutations (Sec. 4.1, 4.2, 5).
//
// Every level of the recursion, for every job of a batch, is one segment list;
// each kernel below covers all segments of a level in one launch (the plain
// per-subproblem form reuses the same kernels with one segment per launch).
#include <algorithm>

#include "order_engine.h"

namespace vmo {

constexpr uint32_t kQMax = 1048575u;  // 2^20 - 1 grid
constexpr int kT = 256;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// -------------------------------------------------------- device helpers ----
// s(v) = x(v).r - delta, products and sums rounded one by one, left to right.
__device__ __forceinline__ double plane_eval(uint32_t q0, uint32_t q1, uint32_t q2, uint32_t q3,
                                             const double* pl) {
  double a0 = (double)q0 * pl[0];
  double a1 = (double)q1 * pl[1];
  double a2 = (double)q2 * pl[2];
  double a3 = (double)q3 * pl[3];
  double t = a0 + a1;
  t = t + a2;
  t = t + a3;
  return t - pl[4];
}
// r = c2 - c1, delta = ((c1 + c2) / 2) . r with the same rounding discipline.
__device__ __forceinline__ void plane_from(const double* c1, const double* c2, double* pl) {
  double m[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pl[d] = c2[d] - c1[d];
    double s = c1[d] + c2[d];
    m[d] = s * 0.5;
  }
  double a0 = m[0] * pl[0];
  double a1 = m[1] * pl[1];
  double a2 = m[2] * pl[2];
  double a3 = m[3] * pl[3];
  double t = a0 + a1;
  t = t + a2;
  t = t + a3;
  pl[4] = t;
}

__device__ __forceinline__ int32_t find_job(const JobDev* jobs, int32_t nj, int64_t pos) {
  int32_t lo = 0, hi = nj;
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    if (jobs[mid].voff <= pos) lo = mid; else hi = mid;
  }
  return lo;
}

// Job of a virtual index u (emission): the last job whose base is <= u.
__device__ __forceinline__ int32_t find_v(const JobDev* jobs, int32_t nj, int64_t u, int which) {
  int32_t lo = 0, hi = nj;
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    int64_t b = which == 0 ? jobs[mid].vk0 : (which == 1 ? jobs[mid].vn0 : jobs[mid].ve0);
    if (b <= u) lo = mid; else hi = mid;
  }
  return lo;
}

// Sum over the 64 lanes (all active) by DPP row shifts and row broadcasts;
// lane 63 ends with the total.
__device__ __forceinline__ int32_t wave_sum_dpp(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Segmented sum across a wavefront.  Lanes hold (key, v[F]); equal keys form
// contiguous lane runs.  Afterwards the first lane of each run holds the run's
// total and returns true.  key < 0 = no segment.
template <int F>
__device__ __forceinline__ bool wave_seg_sum(int key, int64_t (&v)[F]) {
  int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int ok = __shfl_down(key, off, 64);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      int64_t o = __shfl_down(v[f], off, 64);
      if (lane + off < 64 && ok == key) v[f] += o;
    }
  }
  int prev = __shfl_up(key, 1, 64);
  return key >= 0 && (lane == 0 || prev != key);
}

// --------------------------------------------------------- setup kernels ----
__global__ void k_gather_x(const JobDev* jobs, int32_t nj, const float* const* xptr, int64_t N,
                           int64_t Np, float* xs, int32_t* id, int32_t* pos) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Np; i += (int64_t)gridDim.x * blockDim.x) {
    if (i >= N) {
      for (int d = 0; d < 4; ++d) xs[d * Np + i] = 0.0f;
      id[i] = -1;
      continue;
    }
    int32_t j = find_job(jobs, nj, i);
    int64_t loc = i - jobs[j].voff;
    const float* x = xptr[j];
    for (int d = 0; d < 4; ++d) xs[d * Np + i] = x[(int64_t)d * jobs[j].k + loc];
    id[i] = (int32_t)i;
    pos[i] = (int32_t)i;
  }
}

// Per-job bounding box (exact FP32 min / max through ordered integer keys).
__global__ void k_bbox(const JobDev* jobs, int32_t nj, const float* xs, int64_t N, int64_t Np, uint32_t* box) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1;
  uint32_t mn[4], mx[4];
  for (int d = 0; d < 4; ++d) { mn[d] = 0xffffffffu; mx[d] = 0u; }
  if (i < N) {
    key = find_job(jobs, nj, i);
    for (int d = 0; d < 4; ++d) mn[d] = mx[d] = fkey(xs[d * Np + i]);
  }
  int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int ok = __shfl_down(key, off, 64);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t a = __shfl_down(mn[d], off, 64), b = __shfl_down(mx[d], off, 64);
      if (lane + off < 64 && ok == key) {
        mn[d] = a < mn[d] ? a : mn[d];
        mx[d] = b > mx[d] ? b : mx[d];
      }
    }
  }
  int prev = __shfl_up(key, 1, 64);
  if (key >= 0 && (lane == 0 || prev != key))
    for (int d = 0; d < 4; ++d) {
      atomicMin(&box[key * 8 + d], mn[d]);
      atomicMax(&box[key * 8 + 4 + d], mx[d]);
    }
}

// Per job: lo = exact FP32 minimum, scale = (2^20 - 1) / largest side (FP64).
__global__ void k_job_scale(JobDev* jobs, int32_t nj, const uint32_t* box) {
  int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nj) return;
  double ext = 0.0;
  for (int d = 0; d < 4; ++d) {
    float lo = fkey_inv(box[j * 8 + d]), hi = fkey_inv(box[j * 8 + 4 + d]);
    jobs[j].lo[d] = lo;
    double e = (double)hi - (double)lo;
    if (e > ext) ext = e;
  }
  jobs[j].scale = ext > 0.0 ? (double)kQMax / ext : 0.0;
}

__global__ void k_quantize(const JobDev* jobs, int32_t nj, const float* xs, int64_t N, int64_t Np, uint32_t* q) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Np; i += (int64_t)gridDim.x * blockDim.x) {
    if (i >= N) {
      for (int d = 0; d < 4; ++d) q[d * Np + i] = 0;
      continue;
    }
    int32_t j = find_job(jobs, nj, i);
    double s = jobs[j].scale;
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
      if (s > 0.0) {
        double t = ((double)xs[d * Np + i] - (double)jobs[j].lo[d]) * s;
        double f = floor(t);
        v = f >= (double)kQMax ? kQMax : (uint32_t)f;
      }
      q[d * Np + i] = v;
    }
  }
}

// --------------------------------------------------------- level kernels ----
// Segment of every position in [p0, p1) for segments [s0, s0 + S).
// Segment of every position in [p0, p1) (-1: none; segments sorted by
// position), and per aligned group of four positions the one value its four
// positions share (kPackMixed when they differ or reach outside [p0, p1)), so
// that the Lloyd passes read one word per four positions.
constexpr int32_t kPackMixed = -2;
__global__ void k_segpos(const int64_t* sbeg, const int64_t* send, int64_t s0, int64_t S, int64_t p0,
                         int64_t p1, int32_t* segpos, int32_t* segpack) {
  const int64_t g0 = p0 >> 2, g1 = (p1 + 3) >> 2;
  for (int64_t g = g0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < g1;
       g += (int64_t)gridDim.x * blockDim.x) {
    int32_t first = 0;
    bool uni = true;
    for (int u = 0; u < 4; ++u) {
      const int64_t i = 4 * g + u;
      if (i < p0 || i >= p1) {
        uni = false;
        continue;
      }
      int32_t v = -1;
      int64_t lo = s0, hi = s0 + S;
      if (S > 0 && sbeg[lo] <= i) {
        while (hi - lo > 1) {
          int64_t mid = (lo + hi) >> 1;
          if (sbeg[mid] <= i) lo = mid; else hi = mid;
        }
        v = i < send[lo] ? (int32_t)lo : -1;
      }
      segpos[i] = v;
      if (u == 0) first = v;
      else if (v != first) uni = false;
    }
    segpack[g] = uni ? first : kPackMixed;
  }
}

// z1: uniform member of the segment; clears the accumulators.
__global__ void k_seed1(const JobDev* jobs, SegArrays sg, int64_t s0, int64_t S) {
  int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= s0 + S) return;
  const JobDev& J = jobs[sg.job[s]];
  uint64_t n = (uint64_t)(sg.end[s] - sg.beg[s]);
  uint64_t r0 = rng3(J.seed, kTagKmeans | (J.job_index << 8), (uint64_t)sg.h[s], 0);
  sg.i1[s] = sg.beg[s] + (int64_t)__umul64hi(r0, n);
  for (int f = 0; f < kAccF; ++f) sg.acc[s * kAccF + f] = 0;
  sg.state[s] = kStIter;
  sg.iters[s] = 0;
}

// D^2 = |q - q(z1)|^2 (exact int64) per position, and the segment sums of q.
__global__ __launch_bounds__(kT) void k_d2(SegArrays sg, const int32_t* segpos, const uint32_t* q, int64_t Np,
                                           int64_t p0, int64_t p1, U128* dd) {
  int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1;
  int64_t v[4] = {0, 0, 0, 0};
  if (i < p1) {
    int32_t s = segpos[i];
    U128 out{0, 0};
    if (s >= 0) {
      key = s;
      int64_t j = sg.i1[s];
      uint64_t d2 = 0;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        int64_t a = (int64_t)q[d * Np + i];
        int64_t df = a - (int64_t)q[d * Np + j];
        d2 += (uint64_t)(df * df);
        v[d] = a;
      }
      out.lo = d2;
    }
    dd[i] = out;
  }
  if (wave_seg_sum<4>(key, v))
    for (int d = 0; d < 4; ++d) atomicAdd((unsigned long long*)&sg.acc[key * kAccF + kAccTot + d], (unsigned long long)v[d]);
}

// z2 by the D^2 draw: t = floor(r1 T / 2^64) (exact), z2 = first position whose
// inclusive prefix exceeds t.  T = 0 -> the node cannot split.
__global__ void k_seed2(const JobDev* jobs, SegArrays sg, int64_t s0, int64_t S, const U128* pre,
                        const uint32_t* q, int64_t Np) {
  int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= s0 + S) return;
  const JobDev& J = jobs[sg.job[s]];
  int64_t b = sg.beg[s], e = sg.end[s];
  U128 base = pre[b];
  U128 T = u128_sub(pre[e], base);
  if (u128_zero(T)) { sg.state[s] = kStLeaf; return; }
  uint64_t r1 = rng3(J.seed, kTagKmeans | (J.job_index << 8), (uint64_t)sg.h[s], 1);
  // t = (r1 * T.lo >> 64) + r1 * T.hi
  U128 t;
  t.lo = r1 * T.hi;
  t.hi = __umul64hi(r1, T.hi);
  t = u128_add(t, U128{__umul64hi(r1, T.lo), 0});
  U128 target = u128_add(base, t);
  int64_t lo = b + 1, hi = e;  // smallest j in [b+1, e] with pre[j] > target
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (u128_gt(pre[mid], target)) hi = mid; else lo = mid + 1;
  }
  int64_t i2 = lo - 1, i1 = sg.i1[s];
  double c1[4], c2[4];
  for (int d = 0; d < 4; ++d) {
    c1[d] = (double)q[d * Np + i1];
    c2[d] = (double)q[d * Np + i2];
    sg.cen[s * 8 + d] = c1[d];
    sg.cen[s * 8 + 4 + d] = c2[d];
  }
  plane_from(c1, c2, &sg.plane[s * 5]);
}

// Segmented sum across a wavefront of int32 values (exact here: every value
// is below 2^29), as wave_seg_sum.
template <int F>
__device__ __forceinline__ bool wave_seg_sum32(int key, int32_t (&v)[F]) {
  int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int ok = __shfl_down(key, off, 64);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      int32_t o = __shfl_down(v[f], off, 64);
      if (lane + off < 64 && ok == key) v[f] += o;
    }
  }
  int prev = __shfl_up(key, 1, 64);
  return key >= 0 && (lane == 0 || prev != key);
}

// One Lloyd assignment: side by the plane, and the segment's side-1 sums,
// side-1 count and changed count.  PPT (4 or 8) consecutive positions per
// thread (Np is a multiple of 4 and the arrays are 16-byte aligned): 16-byte
// loads of each grid coordinate and of the segment ids, 4-byte loads and
// stores of the sides.  Bytes of a pack outside [p0, p1) or in segments that
// do not iterate are written back unchanged (one thread owns each pack).
// A thread sums its positions of the pack's first segment in int32 (at most
// PPT coordinates below 2^20 each); positions of a later segment in the same
// pack (a segment boundary inside the pack, once per segment at most) go to
// the segment's accumulators directly.  A wavefront whose threads all hold
// one segment adds up by DPP, else by a segmented shuffle sum (int32: below
// 64 PPT 2^20 = 2^29); the block adds equal segments before the atomics.
// prev: segments still iterating after the previous iteration (NULL: run);
// when none is, this iteration would skip every segment, so it returns.
template <int PPT>
__global__ __launch_bounds__(1024) void k_assign(SegArrays sg, const int32_t* segpos, const int32_t* segpack,
                                                 const uint32_t* q, int64_t Np,
                                                 int64_t p0, int64_t p1, int it, uint8_t* side,
                                                 unsigned long long* work, const int32_t* prev) {
  if (prev && *prev == 0) return;
  const int64_t b = (p0 & ~int64_t(3)) + PPT * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  int kt = -1;          // the pack's first iterating segment
  int32_t acc[6] = {0, 0, 0, 0, 0, 0};
  // state and plane of the segment of the previous position (a pack meets
  // one segment, rarely two): loaded once per segment, not per position
  int32_t cs = -1;
  bool citer = false;
  double pl[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int32_t scanned = 0;  // positions read (for the timing's byte count)
#pragma unroll
  for (int h = 0; h < PPT / 4; ++h) {
    const int64_t bh = b + 4 * h;
    if (bh >= p1) break;
    // the four positions' segments: one word when they share it; four
    // positions of a segment that no longer iterates are neither read nor
    // written
    const int32_t pk = segpack[bh >> 2];
    if (pk != kPackMixed && (pk < 0 || sg.state[pk] != kStIter)) continue;
    scanned += (int32_t)(min(bh + 4, p1) - max(bh, p0));
    int4 sp = make_int4(pk, pk, pk, pk);
    if (pk == kPackMixed) sp = *reinterpret_cast<const int4*>(segpos + bh);
    const uint4 q0 = *reinterpret_cast<const uint4*>(q + bh);
    const uint4 q1 = *reinterpret_cast<const uint4*>(q + Np + bh);
    const uint4 q2 = *reinterpret_cast<const uint4*>(q + 2 * Np + bh);
    const uint4 q3 = *reinterpret_cast<const uint4*>(q + 3 * Np + bh);
    const uchar4 so = *reinterpret_cast<const uchar4*>(side + bh);
    const int spa[4] = {sp.x, sp.y, sp.z, sp.w};
    const uint32_t a0[4] = {q0.x, q0.y, q0.z, q0.w}, a1[4] = {q1.x, q1.y, q1.z, q1.w};
    const uint32_t a2[4] = {q2.x, q2.y, q2.z, q2.w}, a3[4] = {q3.x, q3.y, q3.z, q3.w};
    uint8_t sv[4] = {so.x, so.y, so.z, so.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = bh + u;
      const int32_t sgm = spa[u];
      if (i < p0 || i >= p1 || sgm < 0) continue;
      if (sgm != cs) {
        cs = sgm;
        citer = sg.state[sgm] == kStIter;
        if (citer)
          for (int f = 0; f < 5; ++f) pl[f] = sg.plane[sgm * 5 + f];
      }
      if (!citer) continue;
      const double e = plane_eval(a0[u], a1[u], a2[u], a3[u], pl);
      const uint8_t sd = e <= 0.0 ? 1 : 2;
      const int32_t chg = (it > 0 && sd != sv[u]) ? 1 : 0;
      sv[u] = sd;
      if (kt < 0) kt = sgm;
      if (sgm == kt) {
        if (sd == 1) {
          acc[0] += (int32_t)a0[u]; acc[1] += (int32_t)a1[u]; acc[2] += (int32_t)a2[u]; acc[3] += (int32_t)a3[u];
          acc[4] += 1;
        }
        acc[5] += chg;
      } else {
        unsigned long long* g = (unsigned long long*)&sg.acc[sgm * kAccF + kAccS1];
        if (sd == 1) {
          atomicAdd(g + 0, (unsigned long long)a0[u]); atomicAdd(g + 1, (unsigned long long)a1[u]);
          atomicAdd(g + 2, (unsigned long long)a2[u]); atomicAdd(g + 3, (unsigned long long)a3[u]);
          atomicAdd(g + 4, 1ull);
        }
        if (chg) atomicAdd(g + 5, 1ull);
      }
    }
    *reinterpret_cast<uchar4*>(side + bh) = make_uchar4(sv[0], sv[1], sv[2], sv[3]);
  }
  const int k0 = __builtin_amdgcn_readfirstlane(kt);
  // wavefronts with one segment leave their sums here; the block adds those
  // of equal segments before the atomics (a level's first segments hold
  // hundreds of thousands of positions, whose per-wavefront atomics would
  // queue on the same six words)
  __shared__ int skey[32];
  __shared__ long long ssum[32][6];
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (__all(kt == k0)) {
    if (k0 >= 0) {
      int32_t t[6];
#pragma unroll
      for (int f = 0; f < 6; ++f) t[f] = wave_sum_dpp(acc[f]);
      if (lane_id() == 63)
        for (int f = 0; f < 6; ++f) ssum[wv][f] = t[f];
    }
    if (lane_id() == 63) skey[wv] = k0;
  } else {
    if (lane_id() == 63) skey[wv] = -1;
    // the lanes' packs increase with the lane: equal keys are runs
    if (wave_seg_sum32<6>(kt, acc))
      for (int f = 0; f < 6; ++f)
        if (acc[f]) atomicAdd((unsigned long long*)&sg.acc[kt * kAccF + kAccS1 + f], (unsigned long long)acc[f]);
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    // field f: one atomic per run of wavefronts with the same segment
    const int f = threadIdx.x;
    int cur = -1;
    long long a = 0;
    for (int w = 0; w <= nw; ++w) {
      const int kw = w < nw ? skey[w] : -1;
      if (kw != cur) {
        if (cur >= 0 && a) atomicAdd((unsigned long long*)&sg.acc[cur * kAccF + kAccS1 + f], (unsigned long long)a);
        cur = kw;
        a = 0;
      }
      if (kw >= 0) a += ssum[w][f];
    }
  }
  if (work) {
    // 17 algorithmic bytes per position read (16 B coordinates, 1 B side)
    const int32_t tot = wave_sum_dpp(scanned);
    if (lane_id() == 63 && tot) atomicAdd(work, 17ull * (unsigned long long)tot);
  }
}

// End of a Lloyd iteration for segment s: new centres and plane, or the
// segment stops (converged, t_max reached, or a side came out empty).
__device__ __forceinline__ void lloyd_fin_seg(const SegArrays& sg, int64_t s, int it, int t_max, int32_t* active) {
  if (sg.state[s] != kStIter) return;
  int64_t* a = &sg.acc[s * kAccF];
  int64_t n = sg.end[s] - sg.beg[s];
  int64_t n1 = a[kAccS1 + 4], n2 = n - n1, ch = a[kAccS1 + 5];
  if (n1 == 0 || n2 == 0) { sg.state[s] = kStLeaf; return; }
  if ((it > 0 && ch == 0) || it >= t_max) { sg.state[s] = kStDone; return; }
  double m1[4], m2[4];
  for (int d = 0; d < 4; ++d) {
    int64_t S1 = a[kAccS1 + d];
    int64_t S2 = a[kAccTot + d] - S1;
    m1[d] = (double)S1 / (double)n1;
    m2[d] = (double)S2 / (double)n2;
    sg.cen[s * 8 + d] = m1[d];
    sg.cen[s * 8 + 4 + d] = m2[d];
  }
  plane_from(m1, m2, &sg.plane[s * 5]);
  sg.iters[s] = it + 1;
  for (int f = 0; f < 6; ++f) a[kAccS1 + f] = 0;
  atomicAdd(active, 1);
}

__global__ void k_lloyd_fin(SegArrays sg, int64_t s0, int64_t S, int it, int t_max, int32_t* active,
                            const int32_t* prev) {
  if (prev && *prev == 0) return;
  int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < s0 + S) lloyd_fin_seg(sg, s, it, t_max, active);
}

// ------------------------------------------------------------- separator ----
// Cut edges of splitting segments: both ends in the segment, sides differ.
// Only segments [s0, s0 + S) count: positions outside them may hold segment
// ids of other launches, which are never dereferenced.
__global__ void k_cutedges(const int32_t* edges, int64_t e0, int64_t e1, const int32_t* pos, const int32_t* segpos,
                           int64_t s0, int64_t S, const int32_t* state, const uint8_t* side, int32_t* flag) {
  for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t pa = pos[edges[2 * e]], pb = pos[edges[2 * e + 1]];
    int32_t sa = segpos[pa], sb = segpos[pb];
    int ok = sa >= s0 && sa < s0 + S && sa == sb;
    ok = ok && state[sa] == kStDone && side[pa] != side[pb];
    flag[e] = ok;
  }
}
__global__ void k_compact_edges(const int32_t* flag, const int32_t* scan, const int32_t* edges, int64_t e0,
                                int64_t e1, const int32_t* pos, const int32_t* segpos, int32_t* cand,
                                uint32_t* candseg) {
  for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[e]) continue;
    int32_t o = scan[e];
    cand[o] = (int32_t)e;
    candseg[o] = (uint32_t)segpos[pos[edges[2 * e]]];
  }
}
__global__ void k_cbounds(const uint32_t* candseg, int64_t nc, int64_t* cbeg, int64_t* cend) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t s = candseg[i];
    if (i == 0 || candseg[i - 1] != s) cbeg[s] = i;
    if (i == nc - 1 || candseg[i + 1] != s) cend[s] = i + 1;
  }
}

// Position of the partner of the vertex at each position of [p0, p1) under
// the strengthened diagonal (-1: none).
__global__ void k_mate_pos(const int32_t* id, const int32_t* pos, const int32_t* mu_g, int64_t p0, int64_t p1,
                           int32_t* mate) {
  for (int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p1; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = id[i];  // -1 at the padding positions
    const int32_t w = v >= 0 ? mu_g[v] : -1;
    mate[i] = w >= 0 ? pos[w] : -1;
  }
}

// Algorithm 7 separator loop, one wavefront per segment.  Its cut edges come in
// edge order, 64 at a time; edges already touching S are dropped; inside a
// chunk, edges are resolved in order with ballots: once an edge puts its end
// nearer the plane (smaller |s|; ties to the first end) into S, every later
// edge of the chunk touching that vertex is dropped.  With a strengthened
// diagonal (mate != NULL) the chosen end's partner enters S with it, and later
// edges touching either are dropped.
__global__ __launch_bounds__(kT) void k_separator(SegArrays sg, int64_t s0, int64_t S, const int64_t* cbeg,
                                                  const int64_t* cend, const int32_t* cand, const int32_t* edges,
                                                  const int32_t* pos, const uint32_t* q, int64_t Np,
                                                  const int32_t* mate, int32_t* sep) {
  int64_t s = s0 + (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (s >= s0 + S) return;
  int lane = lane_id();
  int64_t b = cbeg[s], e = cend[s];
  if (b >= e) return;
  const double* pl = &sg.plane[s * 5];
  for (int64_t base = b; base < e; base += 64) {
    int64_t idx = base + lane;
    bool valid = idx < e;
    int32_t pa = -1, pb = -1, ch = -1, chm = -1;
    bool alive = false;
    if (valid) {
      int32_t ed = cand[idx];
      pa = pos[edges[2 * ed]];
      pb = pos[edges[2 * ed + 1]];
      double sa = fabs(plane_eval(q[pa], q[Np + pa], q[2 * Np + pa], q[3 * Np + pa], pl));
      double sb = fabs(plane_eval(q[pb], q[Np + pb], q[2 * Np + pb], q[3 * Np + pb], pl));
      ch = sa <= sb ? pa : pb;
      if (mate) chm = mate[ch];
      int ia = __hip_atomic_load(&sep[pa], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int ib = __hip_atomic_load(&sep[pb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      alive = !ia && !ib;
    }
    uint64_t mask = __ballot(valid && alive);
    uint64_t rem = mask;
    while (rem) {
      int j = __builtin_ctzll(rem);
      rem &= rem - 1;
      int32_t cj = __shfl(ch, j, 64);
      int32_t mj = __shfl(chm, j, 64);
      uint64_t kill = __ballot(valid && lane > j && (pa == cj || pb == cj || (mj >= 0 && (pa == mj || pb == mj))));
      mask &= ~kill;
      rem &= ~kill;
    }
    if (valid && ((mask >> lane) & 1ull)) {
      __hip_atomic_store(&sep[ch], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (chm >= 0) __hip_atomic_store(&sep[chm], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the next chunk's reads see these stores: the positions of a segment are
    // read and written by this wavefront only, so the order is needed among
    // its own lanes (workgroup scope: a wait for the stores, no cache write-back)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
}

__global__ void k_mark_sep(const int32_t* sep, int64_t p0, int64_t p1, uint8_t* side) {
  for (int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p1; i += (int64_t)gridDim.x * blockDim.x)
    if (sep[i]) side[i] = 3;
}

// ------------------------------------------------------------- partition ----
__global__ void k_classes(const int32_t* segpos, const int32_t* state, const uint8_t* side, int64_t p0, int64_t p1,
                          uint64_t* cls) {
  for (int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p1; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t s = segpos[i];
    uint64_t v = 0;
    if (s >= 0 && state[s] == kStDone) v = side[i] == 1 ? 1ull : (side[i] == 2 ? (1ull << 32) : 0ull);
    cls[i] = v;
  }
}

struct Counts3 {
  int64_t n1, n2, n3;
};
__device__ __forceinline__ Counts3 seg_counts(const uint64_t* pre, int64_t b, int64_t e) {
  uint64_t d = pre[e] - pre[b];
  Counts3 c;
  c.n1 = (int64_t)(d & 0xffffffffull);
  c.n2 = (int64_t)(d >> 32);
  c.n3 = (e - b) - c.n1 - c.n2;
  return c;
}

// Stable three-way partition of every split segment: part 1, then part 2 and
// the separator (BBD: 1 | 2 | S; SBD: 1 | S | 2), ascending within each.
__global__ __launch_bounds__(kT) void k_partition(const JobDev* jobs, SegArrays sg, const int32_t* segpos,
                                                  const uint8_t* side, const uint64_t* pre, const uint32_t* q,
                                                  const int32_t* id, int64_t Np, int64_t p0, int64_t p1,
                                                  uint32_t* q2, int32_t* id2, int32_t* pos) {
  for (int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p1; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t s = segpos[i];
    int64_t dest = i;
    if (s >= 0 && sg.state[s] == kStDone) {
      int64_t b = sg.beg[s], e = sg.end[s];
      Counts3 c = seg_counts(pre, b, e);
      uint64_t d = pre[i] - pre[b];
      int64_t r1 = (int64_t)(d & 0xffffffffull), r2 = (int64_t)(d >> 32), r3 = (i - b) - r1 - r2;
      bool bbd = jobs[sg.job[s]].ord == VMO_BBD;
      uint8_t sd = side[i];
      if (sd == 1) dest = b + r1;
      else if (sd == 2) dest = bbd ? b + c.n1 + r2 : b + c.n1 + c.n3 + r2;
      else dest = bbd ? b + c.n1 + c.n2 + r3 : b + c.n1 + r3;
      pos[id[i]] = (int32_t)dest;
    }
    for (int d = 0; d < 4; ++d) q2[d * Np + dest] = q[d * Np + i];
    id2[dest] = id[i];
  }
}

// Per processed segment: node-table entries for the node and its children;
// the number of children that go on splitting.
__global__ void k_children(const JobDev* jobs, SegArrays sg, int64_t s0, int64_t S, const uint64_t* pre, NodeArrays nd,
                           int32_t* nnext) {
  int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= s0 + S) return;
  const JobDev& J = jobs[sg.job[s]];
  int64_t nb = J.node_base;
  int32_t h = sg.h[s];
  int64_t b = sg.beg[s], e = sg.end[s];
  int32_t cnt = 0;
  if (sg.state[s] != kStDone) {
    nd.state[nb + h] = kNodeLeaf;
    nd.beg[nb + h] = b;
    nd.end[nb + h] = e;
  } else {
    Counts3 c = seg_counts(pre, b, e);
    bool bbd = J.ord == VMO_BBD;
    nd.state[nb + h] = kNodeInternal;
    nd.beg[nb + h] = bbd ? b + c.n1 + c.n2 : b + c.n1;
    nd.end[nb + h] = nd.beg[nb + h] + c.n3;
    int32_t K = sg.K[s], K1 = (K + 1) / 2, K2 = K / 2;
    int64_t cb[2] = {b, bbd ? b + c.n1 : b + c.n1 + c.n3};
    int64_t cn[2] = {c.n1, c.n2};
    int32_t ck[2] = {K1, K2}, cp[2] = {sg.p0[s], sg.p0[s] + K1};
    for (int t = 0; t < 2; ++t) {
      int32_t hc = 2 * h + t;
      nd.K[nb + hc] = ck[t];
      nd.p0[nb + hc] = cp[t];
      nd.beg[nb + hc] = cb[t];
      nd.end[nb + hc] = cb[t] + cn[t];
      if (ck[t] == 1 || cn[t] < 2) nd.state[nb + hc] = kNodeLeaf;
      else { nd.state[nb + hc] = kNodePending; ++cnt; }
    }
  }
  nnext[s - s0] = cnt;
}

__global__ void k_children_write(SegArrays sg, int64_t s0, int64_t S, const int32_t* nscan, const JobDev* jobs,
                                 NodeArrays nd, SegArrays nx, int64_t t0) {
  int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= s0 + S || sg.state[s] != kStDone) return;
  int64_t o = t0 + nscan[s - s0];
  int64_t nb = jobs[sg.job[s]].node_base;
  for (int t = 0; t < 2; ++t) {
    int32_t hc = 2 * sg.h[s] + t;
    if (nd.state[nb + hc] != kNodePending) continue;
    nx.beg[o] = nd.beg[nb + hc];
    nx.end[o] = nd.end[nb + hc];
    nx.job[o] = sg.job[s];
    nx.h[o] = hc;
    nx.K[o] = nd.K[nb + hc];
    nx.p0[o] = nd.p0[nb + hc];
    ++o;
  }
}

// ------------------------------------------------------------- emission ----
// Leaf vertices get the leaf's first part; separator vertices P + heap id.
__global__ void k_node_fill(const JobDev* jobs, int32_t nj, NodeArrays nd, int64_t NTv, const int32_t* id,
                            int32_t* const* part_out, int32_t* leafh) {
  for (int64_t u = blockIdx.x; u < NTv; u += gridDim.x) {
    int32_t j = find_v(jobs, nj, u, 1);
    const JobDev& J = jobs[j];
    int64_t g = J.node_base + (u - J.vn0);
    int32_t st = nd.state[g];
    if (st != kNodeLeaf && st != kNodeInternal) continue;
    int32_t h = (int32_t)(g - J.node_base);
    int32_t pv = st == kNodeLeaf ? nd.p0[g] : J.P + h;
    int32_t* part = part_out[j];
    for (int64_t i = nd.beg[g] + threadIdx.x; i < nd.end[g]; i += blockDim.x) {
      int32_t v = id[i];
      if (part) part[v - J.voff] = pv;
      leafh[v] = h;
    }
  }
}

__global__ void k_vperm(const JobDev* jobs, int32_t nj, const int32_t* id, int64_t Nv, int32_t* const* vperm) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < Nv; u += (int64_t)gridDim.x * blockDim.x) {
    int32_t j = find_v(jobs, nj, u, 0);
    int64_t i = jobs[j].voff + (u - jobs[j].vk0);
    vperm[j][u - jobs[j].vk0] = (int32_t)(id[i] - jobs[j].voff);
  }
}

// Emission ranks, one block per job: the order is in-order (SBD: left, node,
// right) or post-order (BBD: left, right, node) over the heap tree.  Subtree
// sizes go bottom-up and the rank of each subtree's first node top-down, one
// heap level per pass (sz and off are scratch, one word per node slot).
constexpr int kEmitT = 256;
__global__ __launch_bounds__(kEmitT) void k_emit(const JobDev* jobs, int32_t nj, NodeArrays nd, const OutPtrs* outs,
                                                 int32_t* rank_of, int32_t* sz, int32_t* off) {
  const int32_t j = blockIdx.x;
  if (j >= nj) return;  // the whole block
  const JobDev& J = jobs[j];
  const OutPtrs& O = outs[j];
  const int64_t nb = J.node_base;
  const int32_t nmax = 4 * J.P;
  const bool post = J.ord == VMO_BBD;
  const int dmax = 31 - __clz(nmax - 1);  // deepest heap level below nmax
  auto state = [&](int32_t h) { return h < nmax ? nd.state[nb + h] : kNodeNone; };
  auto size = [&](int32_t h) { return h < nmax ? sz[nb + h] : 0; };
  for (int d = dmax; d >= 0; --d) {
    const int32_t h1 = min(2 << d, nmax);
    for (int32_t h = (1 << d) + threadIdx.x; h < h1; h += kEmitT) {
      const int32_t st = state(h);
      int32_t n = 0;
      if (st == kNodeLeaf) n = 1;
      else if (st == kNodeInternal) n = 1 + size(2 * h) + size(2 * h + 1);
      sz[nb + h] = n;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) off[nb + 1] = 0;
  __syncthreads();
  for (int d = 0; d < dmax; ++d) {
    const int32_t h1 = min(2 << d, nmax);
    for (int32_t h = (1 << d) + threadIdx.x; h < h1; h += kEmitT) {
      if (state(h) != kNodeInternal) continue;
      const int32_t o = off[nb + h];
      if (2 * h < nmax) off[nb + 2 * h] = o;
      if (2 * h + 1 < nmax) off[nb + 2 * h + 1] = o + size(2 * h) + (post ? 0 : 1);
    }
    __syncthreads();
  }
  const int32_t nn = sz[nb + 1];
  for (int32_t h = 1 + threadIdx.x; h < nmax; h += kEmitT) {
    const int32_t st = state(h);
    if (st != kNodeLeaf && st != kNodeInternal) continue;
    const bool leaf = st == kNodeLeaf;
    const int32_t o = off[nb + h];
    const int32_t r = leaf ? o : (post ? o + size(2 * h) + size(2 * h + 1) : o + size(2 * h));
    O.node_heap[r] = h;
    O.node_vptr[r] = (int32_t)(nd.beg[nb + h] - J.voff);
    O.split_cut[r] = (!leaf && J.mode == VMO_GRAPH) ? (double)(nd.end[nb + h] - nd.beg[nb + h]) : 0.0;
    rank_of[nb + h] = r;
  }
  for (int32_t t = nn + threadIdx.x; t < nmax; t += kEmitT) {
    O.node_heap[t] = -1;
    O.node_vptr[t] = J.k;
    O.split_cut[t] = 0.0;
  }
  if (threadIdx.x == 0) {
    O.node_vptr[nmax] = J.k;
    O.n_nodes[0] = nn;
  }
  if (O.node_nptr) {
    // filled after the net sort; pad here
    for (int32_t t = threadIdx.x; t <= nmax + 1; t += kEmitT) O.node_nptr[t] = J.nnets;
  }
}

__device__ __forceinline__ int32_t heap_lca(int32_t a, int32_t b) {
  // bring to equal depth, then climb together
  int da = 31 - __clz(a), db = 31 - __clz(b);
  if (da > db) a >>= (da - db); else b >>= (db - da);
  while (a != b) { a >>= 1; b >>= 1; }
  return a;
}

// Net mode: a net belongs to the lowest common ancestor of its pins' leaves.
// kNetG lanes per net: each takes every kNetG-th pin (consecutive lanes read
// consecutive pins), and the group combines its lanes' ancestors (the lowest
// common ancestor of a set does not depend on the order it is formed in).  A
// wavefront takes kNetRun consecutive runs of 64 / kNetG consecutive nets, so
// its nets mostly belong to one job, whose range it keeps.
constexpr int kNetG = 16, kNetRun = 16;
__global__ void k_net_node(const JobDev* jobs, int32_t nj, int64_t Lv, const int32_t* leafh, const int32_t* rank_of,
                           const OutPtrs* outs, const int64_t* keybase, uint32_t* key, int32_t* val) {
  constexpr int kPerWave = 64 / kNetG;
  const int gl = threadIdx.x & (kNetG - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t u0 = wave * kPerWave * kNetRun + ((threadIdx.x & 63) / kNetG);
  int32_t j = -1;
  int64_t jlo = 0, jhi = 0;  // nets of job j: [jlo, jhi)
  for (int r = 0; r < kNetRun; ++r) {
    const int64_t u = u0 + (int64_t)r * kPerWave;
    if (u >= Lv) break;
    if (u < jlo || u >= jhi) {
      j = find_v(jobs, nj, u, 2);
      jlo = jobs[j].ve0;
      jhi = j + 1 < nj ? jobs[j + 1].ve0 : Lv;
    }
    const JobDev& J = jobs[j];
    const int64_t ul = u - jlo;
    const int64_t b = J.nets_ptr[ul], e = J.nets_ptr[ul + 1];
    const int32_t* pins = J.nets_pins;
    const int32_t va = J.pin_vadd;
    int32_t node = 0;  // none yet (heap ids start at 1)
    for (int64_t p = b + gl; p < e; p += kNetG) {
      const int32_t h = leafh[pins[p] + va];
      node = node ? heap_lca(node, h) : h;
    }
    for (int off = kNetG / 2; off > 0; off >>= 1) {
      const int32_t o = __shfl_xor(node, off, kNetG);
      if (o) node = node ? heap_lca(node, o) : o;
    }
    if (gl != 0) continue;
    const int32_t rk = b == e ? outs[j].n_nodes[0] : rank_of[J.node_base + node];
    key[u] = (uint32_t)(keybase[j] + rk);
    val[u] = (int32_t)ul;
  }
}

// Nets per key (counting sort of the nets by node): a wavefront adds each
// run of equal keys among its lanes with one atomic (the nets of a node are
// mostly consecutive).
__global__ void k_net_count(const uint32_t* key, int64_t Lv, int64_t* keycount) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < Lv; base += stride) {
    const int64_t u = base + lane;
    const int nvalid = Lv - base < 64 ? (int)(Lv - base) : 64;
    const uint32_t k = u < Lv ? key[u] : 0xffffffffu;
    const uint32_t pk = __shfl_up(k, 1);
    const bool head = lane < nvalid && (lane == 0 || pk != k);
    const uint64_t heads = __ballot(head);
    if (head) {
      const uint64_t after = lane == 63 ? 0ull : heads >> (lane + 1);
      const int next = after ? lane + __ffsll((unsigned long long)after) : nvalid;
      atomicAdd((unsigned long long*)&keycount[k], (unsigned long long)(next - lane));
    }
  }
}

// Cut of every split (Table 4) in net mode: the costs of the nets of an
// internal node, summed in FP64 one by one in ascending net id (the nets are
// sorted by node, stably: their order within a node is the input order); one
// wavefront per node.
__global__ __launch_bounds__(kT) void k_net_split(const JobDev* jobs, int32_t nj, const int64_t* keybase, int64_t kt,
                                                  const int64_t* kc, const int32_t* val, NodeArrays nd,
                                                  float* const* costs, const OutPtrs* outs) {
  __shared__ __align__(16) float stage[kT / 64][64];
  const int wv = threadIdx.x >> 6;
  for (int64_t kk = (int64_t)blockIdx.x * (kT / 64) + wv; kk < kt; kk += (int64_t)gridDim.x * (kT / 64)) {
    int32_t lo = 0, hi = nj;  // the last job whose keys begin at or before kk
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (keybase[mid] <= kk) lo = mid; else hi = mid;
    }
    const int32_t j = lo;
    const OutPtrs& O = outs[j];
    const int64_t r = kk - keybase[j];
    if (jobs[j].mode != VMO_NET || r >= O.n_nodes[0]) continue;  // the bucket of empty nets
    const int32_t h = O.node_heap[r];
    if (nd.state[jobs[j].node_base + h] != kNodeInternal) continue;
    const double sum = wave_ordered_cost_sum(costs[j], val, kc[kk], kc[kk + 1], stage[wv]);
    if ((threadIdx.x & 63) == 0) O.split_cut[r] = sum;
  }
}

__global__ void k_net_out(const JobDev* jobs, int32_t nj, int64_t Lv, const int32_t* val, const OutPtrs* outs) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < Lv; u += (int64_t)gridDim.x * blockDim.x) {
    int32_t j = find_v(jobs, nj, u, 2);
    if (outs[j].nperm) outs[j].nperm[u - jobs[j].ve0] = val[u];
  }
}

__global__ void k_net_ptr(const JobDev* jobs, int32_t nj, const int64_t* keyscan, const int64_t* keybase,
                          const OutPtrs* outs) {
  int32_t j = blockIdx.x;
  if (j >= nj) return;
  const OutPtrs& O = outs[j];
  if (!O.node_nptr) return;
  int32_t n = O.n_nodes[0];
  for (int32_t r = threadIdx.x; r <= n; r += blockDim.x)
    O.node_nptr[r] = (int32_t)(keyscan[keybase[j] + r] - jobs[j].ve0);
}

__global__ void k_bisect_out(const JobDev* jobs, SegArrays sg, const uint8_t* side, int64_t k, uint8_t* out,
                             int split) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = split ? (uint8_t)(side[i] - 1) : (uint8_t)0;
}

__global__ void k_bisect_centres(const JobDev* jobs, SegArrays sg, float* cen, int split) {
  int t = threadIdx.x;
  if (t >= 8) return;
  int d = t & 3;
  cen[t] = split ? (float)((double)jobs[0].lo[d] + sg.cen[t] / jobs[0].scale) : 0.0f;
}

__global__ void k_init_roots(const JobDev* jobs, int32_t nj, NodeArrays nd) {
  int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nj) return;
  int64_t g = jobs[j].node_base + 1;
  nd.state[g] = (jobs[j].k < 2 || jobs[j].P == 1) ? kNodeLeaf : kNodePending;
  nd.beg[g] = jobs[j].voff;
  nd.end[g] = jobs[j].voff + jobs[j].k;
  nd.K[g] = jobs[j].P;
  nd.p0[g] = 0;
}

// ---------------------------------------------------------------- engine ----
static unsigned gsz(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

void Engine::alloc_segments(SegBufs& b, int64_t cap) {
  b.beg = Buf<int64_t>(c.pool, cap);
  b.end = Buf<int64_t>(c.pool, cap);
  b.job = Buf<int32_t>(c.pool, cap);
  b.h = Buf<int32_t>(c.pool, cap);
  b.K = Buf<int32_t>(c.pool, cap);
  b.p0 = Buf<int32_t>(c.pool, cap);
  b.state = Buf<int32_t>(c.pool, cap);
  b.iters = Buf<int32_t>(c.pool, cap);
  b.i1 = Buf<int64_t>(c.pool, cap);
  b.acc = Buf<int64_t>(c.pool, cap * kAccF);
  b.plane = Buf<double>(c.pool, cap * 5);
  b.cen = Buf<double>(c.pool, cap * 8);
  b.cap = cap;
}

SegArrays Engine::view(SegBufs& b) {
  SegArrays v;
  v.beg = b.beg.p; v.end = b.end.p; v.job = b.job.p; v.h = b.h.p; v.K = b.K.p; v.p0 = b.p0.p;
  v.state = b.state.p; v.iters = b.iters.p; v.i1 = b.i1.p; v.acc = b.acc.p; v.plane = b.plane.p; v.cen = b.cen.p;
  return v;
}

void Engine::setup(const std::vector<JobHost>& jobs) {
  nj = (int32_t)jobs.size();
  hj.resize(nj);
  int64_t voff = 0, nbase = 0, eoff = 0, noff = 0;
  std::vector<const float*> xp(nj);
  for (int32_t j = 0; j < nj; ++j) {
    const JobHost& H = jobs[j];
    JobDev& D = hj[j];
    memset(&D, 0, sizeof D);
    D.voff = voff; D.k = H.h.k; D.P = H.P; D.mode = H.mode; D.ord = H.order;
    D.seed = H.seed; D.job_index = H.job_index; D.node_base = nbase; D.nnets = H.h.l;
    D.eoff = eoff; D.noff = noff;
    voff += H.h.k;
    nbase += 4 * (int64_t)H.P;
    if (H.mode == VMO_GRAPH) eoff += H.h.l; else noff += H.h.l;
    xp[j] = H.x;
  }
  N = voff;
  Np = (N + 3) & ~int64_t(3);
  NT = nbase;
  E = eoff;
  L = noff;
  VMO_REQUIRE(N < (int64_t(1) << 31) - 8, "too many vertices in one call");
  dj = Buf<JobDev>(c.pool, nj);
  VMO_HIP(hipMemcpyAsync(dj.p, hj.data(), sizeof(JobDev) * nj, hipMemcpyHostToDevice, s));
  Buf<const float*> dxp(c.pool, nj);
  VMO_HIP(hipMemcpyAsync(dxp.p, xp.data(), sizeof(void*) * nj, hipMemcpyHostToDevice, s));
  // coordinates -> concatenated SoA, ids, positions
  Buf<float> xs(c.pool, 4 * Np);
  q = Buf<uint32_t>(c.pool, 4 * Np);
  q2 = Buf<uint32_t>(c.pool, 4 * Np);
  id = Buf<int32_t>(c.pool, Np);
  id2 = Buf<int32_t>(c.pool, Np);
  pos = Buf<int32_t>(c.pool, Np);
  side = Buf<uint8_t>(c.pool, Np);
  segpos = Buf<int32_t>(c.pool, Np);
  segpack = Buf<int32_t>(c.pool, (Np >> 2) + 2);
  VMO_LAUNCH(k_gather_x, gsz(Np), kT, 0, s, dj.p, nj, dxp.p, N, Np, xs.p, id.p, pos.p);
  Buf<uint32_t> box(c.pool, 8 * (size_t)nj);
  std::vector<uint32_t> hbox(8 * (size_t)nj);
  for (int32_t j = 0; j < nj; ++j)
    for (int d = 0; d < 4; ++d) { hbox[8 * j + d] = 0xffffffffu; hbox[8 * j + 4 + d] = 0u; }
  VMO_HIP(hipMemcpyAsync(box.p, hbox.data(), sizeof(uint32_t) * hbox.size(), hipMemcpyHostToDevice, s));
  VMO_LAUNCH(k_bbox, nblocks(N, kT), kT, 0, s, dj.p, nj, xs.p, N, Np, box.p);
  VMO_LAUNCH(k_job_scale, nblocks(nj, 64), 64, 0, s, dj.p, nj, box.p);
  VMO_LAUNCH(k_quantize, gsz(Np), kT, 0, s, dj.p, nj, xs.p, N, Np, q.p);
  VMO_HIP(hipMemcpyAsync(hj.data(), dj.p, sizeof(JobDev) * nj, hipMemcpyDeviceToHost, s));
  // node tables
  nd_state = Buf<int32_t>(c.pool, NT);
  nd_K = Buf<int32_t>(c.pool, NT);
  nd_p0 = Buf<int32_t>(c.pool, NT);
  nd_beg = Buf<int64_t>(c.pool, NT);
  nd_end = Buf<int64_t>(c.pool, NT);
  fill_i32(nd_state.p, kNodeNone, NT, s);
  // level-0 segments: one per job root that can split
  std::vector<int64_t> b0, e0;
  std::vector<int32_t> j0, h0, K0, p00;
  for (int32_t j = 0; j < nj; ++j) {
    bool leaf = hj[j].k < 2 || hj[j].P == 1;
    if (!leaf) {
      b0.push_back(hj[j].voff); e0.push_back(hj[j].voff + hj[j].k);
      j0.push_back(j); h0.push_back(1); K0.push_back(hj[j].P); p00.push_back(0);
    }
  }
  VMO_LAUNCH(k_init_roots, nblocks(nj, 64), 64, 0, s, dj.p, nj, nodes());
  S = (int64_t)b0.size();
  alloc_segments(cur, S > 0 ? S : 1);
  if (S > 0) {
    VMO_HIP(hipMemcpyAsync(cur.beg.p, b0.data(), 8 * S, hipMemcpyHostToDevice, s));
    VMO_HIP(hipMemcpyAsync(cur.end.p, e0.data(), 8 * S, hipMemcpyHostToDevice, s));
    VMO_HIP(hipMemcpyAsync(cur.job.p, j0.data(), 4 * S, hipMemcpyHostToDevice, s));
    VMO_HIP(hipMemcpyAsync(cur.h.p, h0.data(), 4 * S, hipMemcpyHostToDevice, s));
    VMO_HIP(hipMemcpyAsync(cur.K.p, K0.data(), 4 * S, hipMemcpyHostToDevice, s));
    VMO_HIP(hipMemcpyAsync(cur.p0.p, p00.data(), 4 * S, hipMemcpyHostToDevice, s));
  }
  VMO_HIP(hipStreamSynchronize(s));
}

// Copies of many arrays with an offset added, one launch per element type: a
// table of (source, destination offset, count, add) with cumulative counts.
struct OffCopy {
  const void* src;
  int64_t dst, n, add;
};
// A wavefront copies 64 * 16 consecutive elements of the concatenation: one
// table lookup per lane for its first element, then forward steps.
template <class T>
__global__ void k_offset_copy_all(const OffCopy* tab, const int64_t* cum, int32_t nt, int64_t total, T* out) {
  constexpr int kPer = 16;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  for (int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63)) * kPer; w0 < total;
       w0 += nthr * kPer) {
    int64_t i = w0 + lane;  // elements w0 + lane + 64 r, r < kPer: coalesced across the lanes
    if (i >= total) continue;
    int32_t lo = 0, hi = nt;  // last t with cum[t] <= i
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (cum[mid] <= i) lo = mid; else hi = mid;
    }
    int32_t t = lo;
    for (int r = 0; r < kPer && i < total; ++r, i += 64) {
      while (t + 1 < nt && cum[t + 1] <= i) ++t;
      const OffCopy& c = tab[t];
      const int64_t e = i - cum[t];
      out[c.dst + e] = static_cast<const T*>(c.src)[e] + (T)c.add;
    }
  }
}

template <class T>
static void offset_copy_all(Ctx& c, const std::vector<OffCopy>& tab, T* out, hipStream_t s) {
  if (tab.empty()) return;
  const int32_t nt = (int32_t)tab.size();
  std::vector<int64_t> cum(nt);
  int64_t tot = 0;
  for (int32_t t = 0; t < nt; ++t) { cum[t] = tot; tot += tab[t].n; }
  if (tot == 0) return;
  Buf<OffCopy> dt(c.pool, nt);
  Buf<int64_t> dc(c.pool, nt);
  VMO_HIP(hipMemcpyAsync(dt.p, tab.data(), sizeof(OffCopy) * nt, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(dc.p, cum.data(), 8 * nt, hipMemcpyHostToDevice, s));
  VMO_LAUNCH((k_offset_copy_all<T>), nblocks((tot + 15) / 16, kT), kT, 0, s, dt.p, dc.p, nt, tot, out);
}

__global__ void k_mu_global(const int32_t* mu, int32_t k, int64_t voff, int32_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = mu[i] >= 0 ? (int32_t)(mu[i] + voff) : -1;
}

void Engine::set_edges(const std::vector<JobHost>& jobs, const std::vector<int64_t>& jpins) {
  // graph-mode edges, global vertex ids; net-mode nets, global pins
  // (net-mode nets stay in the caller's arrays: the emission reads them
  // through the job table)
  edges = Buf<int32_t>(c.pool, 2 * (E > 0 ? E : 1));
  int64_t npins = 0;
  for (int32_t j = 0; j < nj; ++j)
    if (jobs[j].mode == VMO_NET) npins += jpins[j];
  npins_ = npins;
  jnoff = Buf<int64_t>(c.pool, nj);
  std::vector<int64_t> hnoff(nj);
  std::vector<OffCopy> c32;
  for (int32_t j = 0; j < nj; ++j) {
    const JobHost& H = jobs[j];
    hnoff[j] = hj[j].noff;
    if (H.mode == VMO_GRAPH) {
      if (H.h.l > 0) c32.push_back(OffCopy{H.h.pins, 2 * hj[j].eoff, 2 * (int64_t)H.h.l, hj[j].voff});
    } else {
      hj[j].nets_ptr = H.h.net_ptr;
      hj[j].nets_pins = H.h.pins;
      hj[j].pin_vadd = (int32_t)hj[j].voff;
    }
  }
  offset_copy_all<int32_t>(c, c32, edges.p, s);
  VMO_HIP(hipMemcpyAsync(jnoff.p, hnoff.data(), 8 * nj, hipMemcpyHostToDevice, s));
  // strengthened diagonals, in global vertex ids
  has_mu = false;
  for (int32_t j = 0; j < nj; ++j) has_mu = has_mu || (jobs[j].mode == VMO_GRAPH && jobs[j].mu);
  if (has_mu) {
    mu_g = Buf<int32_t>(c.pool, N);
    fill_i32(mu_g.p, -1, N, s);
    for (int32_t j = 0; j < nj; ++j)
      if (jobs[j].mode == VMO_GRAPH && jobs[j].mu)
        VMO_LAUNCH(k_mu_global, gsz(hj[j].k), kT, 0, s, jobs[j].mu, hj[j].k, hj[j].voff, mu_g.p + hj[j].voff);
  }
}

__global__ void k_offset_copy_i32(const int32_t* in, int32_t* out, int64_t n, int32_t add) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i] + add;
}
__global__ void k_offset_copy_ptr(const int64_t* in, int64_t* out, int64_t n, int64_t add) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i] + add;
}
void Engine::launch_offset_copy_i32(const int32_t* in, int32_t* out, int64_t n, int32_t add) {
  VMO_LAUNCH(k_offset_copy_i32, gsz(n), kT, 0, s, in, out, n, add);
}
void Engine::launch_offset_copy_ptr(const int64_t* in, int64_t* out, int64_t n, int64_t add) {
  VMO_LAUNCH(k_offset_copy_ptr, gsz(n), kT, 0, s, in, out, n, add);
}

constexpr int kLloydCheck = 8;

// Seeding and Lloyd iterations for segments [s0, s0+Sn) over positions [p0, p1).
void Engine::two_means(int64_t s0, int64_t Sn, int64_t p0, int64_t p1, int t_max, bool tuned) {
  SegArrays sg = view(cur);
  int64_t np = p1 - p0;
  VMO_LAUNCH(k_segpos, gsz((np >> 2) + 2), kT, 0, s, cur.beg.p, cur.end.p, s0, Sn, p0, p1, segpos.p, segpack.p);
  VMO_LAUNCH(k_seed1, nblocks(Sn, kT), kT, 0, s, dj.p, sg, s0, Sn);
  Buf<U128> dd(c.pool, Np + 1);
  VMO_LAUNCH(k_d2, nblocks(np, kT), kT, 0, s, sg, segpos.p, q.p, Np, p0, p1, dd.p);
  scan_exclusive<U128>(c, dd.p + p0, dd.p + p0, np, dd.p + p1, s);
  VMO_LAUNCH(k_seed2, nblocks(Sn, kT), kT, 0, s, dj.p, sg, s0, Sn, dd.p, q.p, Np);
  // The assignment's launch shape is tuned online per size bucket in the
  // batched form (every candidate gives the same result): block size x
  // positions per thread (4 or 8, so 256 or 512 positions per wavefront,
  // which sets how many small segments share one wavefront's reduction).
  static const int kBlocks[4] = {128, 256, 512, 1024};
  const int bucket = bits_for((uint64_t)np);
  Buf<int32_t> active(c.pool, (size_t)t_max + 1);  // one counter per iteration, cleared once
  fill_i32(active.p, 0, (int64_t)t_max + 1, s);
  for (int it = 0; it <= t_max; ++it) {
    bool timed = false;
    const int cfg = tuned ? tune_pick(c, kTuneAssign, bucket, 8, &timed) : 1;
    const int B = kBlocks[cfg & 3], ppt = cfg < 4 ? 4 : 8;
    unsigned long long* tw = timed ? tune_begin(c, kTuneAssign, bucket, cfg, s) : nullptr;
    int ph = prof_begin(c, "assign", 17.0 * (double)np, s, nullptr);
    const int64_t packs = (p1 - (p0 & ~int64_t(3)) + ppt - 1) / ppt;
    // after an iteration that left no segment iterating the rest return at
    // once, except the launches that are timed (tuner, profile), which run
    const int32_t* prev = it > 0 ? active.p + it - 1 : nullptr;
    if (ppt == 4)
      VMO_LAUNCH(k_assign<4>, nblocks(packs, B), B, 0, s, sg, segpos.p, segpack.p, q.p, Np, p0, p1, it, side.p, tw,
                 timed || ph >= 0 ? nullptr : prev);
    else
      VMO_LAUNCH(k_assign<8>, nblocks(packs, B), B, 0, s, sg, segpos.p, segpack.p, q.p, Np, p0, p1, it, side.p, tw,
                 timed || ph >= 0 ? nullptr : prev);
    prof_end(c, ph, s);
    if (timed) tune_end(c, s);
    VMO_LAUNCH(k_lloyd_fin, nblocks(Sn, kT), kT, 0, s, sg, s0, Sn, it, t_max, active.p + it, prev);
    // one host check every kLloydCheck iterations: an iteration after the
    // last segment stopped skips every segment, so the extra ones change nothing
    if ((it % kLloydCheck == kLloydCheck - 1 || it == t_max) && read1(active.p + it, s) == 0) break;
  }
}

// Separator (graph mode) for segments [s0, s0+Sn) using edges [e0, e1).
void Engine::separator(int64_t s0, int64_t Sn, int64_t p0, int64_t p1, int64_t e0, int64_t e1) {
  if (e1 <= e0) return;
  SegArrays sg = view(cur);
  int64_t ne = e1 - e0;
  Buf<int32_t> flag(c.pool, E + 1), scn(c.pool, E + 1);
  VMO_LAUNCH(k_cutedges, gsz(ne), kT, 0, s, edges.p, e0, e1, pos.p, segpos.p, s0, Sn, cur.state.p, side.p, flag.p);
  scan_exclusive<int32_t>(c, flag.p + e0, scn.p + e0, ne, scn.p + E, s);
  int32_t nc = read1(scn.p + E, s);
  // positions' separator flags
  Buf<int32_t> sep(c.pool, Np);
  fill_i32(sep.p + p0, 0, p1 - p0, s);
  if (nc > 0) {
    Buf<int32_t> cand(c.pool, nc);
    Buf<uint32_t> cseg(c.pool, nc);
    VMO_LAUNCH(k_compact_edges, gsz(ne), kT, 0, s, flag.p, scn.p, edges.p, e0, e1, pos.p, segpos.p, cand.p, cseg.p);
    radix_sort<uint32_t>(c, cseg.p, cand.p, nc, bits_for((uint64_t)(s0 + Sn)), s);
    Buf<int64_t> cb(c.pool, s0 + Sn), ce(c.pool, s0 + Sn);
    fill_i64(cb.p + s0, 0, Sn, s);
    fill_i64(ce.p + s0, 0, Sn, s);
    VMO_LAUNCH(k_cbounds, gsz(nc), kT, 0, s, cseg.p, (int64_t)nc, cb.p, ce.p);
    Buf<int32_t> mate;
    if (has_mu) {
      mate = Buf<int32_t>(c.pool, Np);
      VMO_LAUNCH(k_mate_pos, gsz(p1 - p0), kT, 0, s, id.p, pos.p, mu_g.p, p0, p1, mate.p);
    }
    VMO_LAUNCH(k_separator, nblocks(Sn, kT / 64), kT, 0, s, sg, s0, Sn, cb.p, ce.p, cand.p, edges.p, pos.p, q.p, Np,
               has_mu ? mate.p : nullptr, sep.p);
  }
  VMO_LAUNCH(k_mark_sep, gsz(p1 - p0), kT, 0, s, sep.p, p0, p1, side.p);
}

// Partition of segments [s0, s0+Sn), node table, next-level segments.
int64_t Engine::partition(int64_t s0, int64_t Sn, int64_t p0, int64_t p1, SegBufs& nx, int64_t t0) {
  SegArrays sg = view(cur);
  int64_t np = p1 - p0;
  Buf<uint64_t> cls(c.pool, Np + 1);
  VMO_LAUNCH(k_classes, gsz(np), kT, 0, s, segpos.p, cur.state.p, side.p, p0, p1, cls.p);
  scan_exclusive<uint64_t>(c, cls.p + p0, cls.p + p0, np, cls.p + p1, s);
  VMO_LAUNCH(k_partition, gsz(np), kT, 0, s, dj.p, sg, segpos.p, side.p, cls.p, q.p, id.p, Np, p0, p1, q2.p, id2.p,
             pos.p);
  // copy back the moved range (positions outside [p0,p1) are untouched in q2/id2)
  for (int d = 0; d < 4; ++d)
    VMO_HIP(hipMemcpyAsync(q.p + d * Np + p0, q2.p + d * Np + p0, 4 * np, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(id.p + p0, id2.p + p0, 4 * np, hipMemcpyDeviceToDevice, s));
  NodeArrays nd = nodes();
  Buf<int32_t> cnt(c.pool, Sn + 1);
  VMO_LAUNCH(k_children, nblocks(Sn, kT), kT, 0, s, dj.p, sg, s0, Sn, cls.p, nd, cnt.p);
  scan_exclusive<int32_t>(c, cnt.p, cnt.p, Sn, cnt.p + Sn, s);
  int32_t nn = read1(cnt.p + Sn, s);
  if (nn > 0) {
    if (t0 + nn > nx.cap) {
      SegBufs bigger;
      alloc_segments(bigger, 2 * (t0 + nn));
      if (t0 > 0) copy_segments(nx, bigger, t0);
      nx = std::move(bigger);
    }
    VMO_LAUNCH(k_children_write, nblocks(Sn, kT), kT, 0, s, sg, s0, Sn, cnt.p, dj.p, nd, view(nx), t0);
  }
  return nn;
}

void Engine::copy_segments(SegBufs& a, SegBufs& b, int64_t n) {
  VMO_HIP(hipMemcpyAsync(b.beg.p, a.beg.p, 8 * n, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(b.end.p, a.end.p, 8 * n, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(b.job.p, a.job.p, 4 * n, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(b.h.p, a.h.p, 4 * n, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(b.K.p, a.K.p, 4 * n, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(b.p0.p, a.p0.p, 4 * n, hipMemcpyDeviceToDevice, s));
}

NodeArrays Engine::nodes() {
  NodeArrays nd;
  nd.state = nd_state.p; nd.K = nd_K.p; nd.p0 = nd_p0.p; nd.beg = nd_beg.p; nd.end = nd_end.p;
  return nd;
}

void Engine::run_levels(int t_max, bool plain) {
  while (S > 0) {
    SegBufs nx;
    alloc_segments(nx, 2 * S);
    int64_t nn = 0;
    if (!plain) {
      two_means(0, S, 0, Np, t_max, true);
      separator(0, S, 0, Np, 0, E);
      nn = partition(0, S, 0, Np, nx, 0);
    } else {
      // one launch sequence per segment
      std::vector<int64_t> hb(S), he(S);
      std::vector<int32_t> hjob(S);
      VMO_HIP(hipMemcpyAsync(hb.data(), cur.beg.p, 8 * S, hipMemcpyDeviceToHost, s));
      VMO_HIP(hipMemcpyAsync(he.data(), cur.end.p, 8 * S, hipMemcpyDeviceToHost, s));
      VMO_HIP(hipMemcpyAsync(hjob.data(), cur.job.p, 4 * S, hipMemcpyDeviceToHost, s));
      VMO_HIP(hipStreamSynchronize(s));
      for (int64_t t = 0; t < S; ++t) {
        const JobDev& J = hj[hjob[t]];
        two_means(t, 1, hb[t], he[t], t_max, false);
        if (J.mode == VMO_GRAPH) separator(t, 1, hb[t], he[t], J.eoff, J.eoff + J.nnets);
        nn += partition(t, 1, hb[t], he[t], nx, nn);
      }
    }
    cur = std::move(nx);
    S = nn;
  }
}

void Engine::finish(const std::vector<JobHost>& jobs) {
  std::vector<int32_t> all(nj);
  for (int32_t j = 0; j < nj; ++j) all[j] = j;
  emit(all, jobs);
}

// Emission of the jobs `slots` (indices into the job table); jobs[i] holds the
// outputs of slots[i].
void Engine::emit(const std::vector<int32_t>& slots, const std::vector<JobHost>& jobs) {
  int32_t m = (int32_t)slots.size();
  if (m == 0) return;
  std::vector<JobDev> sub(m);
  std::vector<OutPtrs> ho(m);
  std::vector<int32_t*> hpart(m), hvperm(m);
  std::vector<float*> hcost(m);
  std::vector<int64_t> kb(m);
  int64_t Nv = 0, NTv = 0, Lv = 0, kt = 0;
  for (int32_t i = 0; i < m; ++i) {
    JobDev J = hj[slots[i]];
    J.vk0 = Nv; J.vn0 = NTv; J.ve0 = Lv;
    Nv += J.k;
    NTv += 4 * (int64_t)J.P;
    if (J.mode == VMO_NET) Lv += J.nnets;
    sub[i] = J;
    kb[i] = kt;
    kt += J.mode == VMO_NET ? 4 * (int64_t)J.P + 1 : 0;
    const vmo_order_out& o = jobs[i].out;
    ho[i].vperm = o.vperm; ho[i].nperm = o.nperm; ho[i].part = o.part; ho[i].node_heap = o.node_heap;
    ho[i].node_vptr = o.node_vptr; ho[i].node_nptr = J.mode == VMO_NET ? o.node_nptr : nullptr;
    ho[i].split_cut = o.split_cut; ho[i].n_nodes = o.n_nodes;
    hpart[i] = o.part; hvperm[i] = o.vperm;
    hcost[i] = const_cast<float*>(jobs[i].h.c);
  }
  VMO_REQUIRE(kt < (int64_t(1) << 32), "too many tree nodes in one call");
  Buf<JobDev> dsub(c.pool, m);
  Buf<OutPtrs> douts(c.pool, m);
  Buf<int32_t*> dpart(c.pool, m), dvperm(c.pool, m);
  Buf<float*> dcost(c.pool, m);
  Buf<int64_t> keybase(c.pool, m);
  VMO_HIP(hipMemcpyAsync(dsub.p, sub.data(), sizeof(JobDev) * m, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(douts.p, ho.data(), sizeof(OutPtrs) * m, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(dpart.p, hpart.data(), sizeof(void*) * m, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(dvperm.p, hvperm.data(), sizeof(void*) * m, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(dcost.p, hcost.data(), sizeof(void*) * m, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(keybase.p, kb.data(), 8 * m, hipMemcpyHostToDevice, s));
  NodeArrays nd = nodes();
  Buf<int32_t> leafh(c.pool, Np);
  VMO_LAUNCH(k_node_fill, (unsigned)(NTv < 65536 ? (NTv > 0 ? NTv : 1) : 65536), kT, 0, s, dsub.p, m, nd, NTv, id.p,
             dpart.p, leafh.p);
  VMO_LAUNCH(k_vperm, gsz(Nv), kT, 0, s, dsub.p, m, id.p, Nv, dvperm.p);
  Buf<int32_t> rank_of(c.pool, NT), esz(c.pool, NT), eoff(c.pool, NT);
  VMO_LAUNCH(k_emit, m, kEmitT, 0, s, dsub.p, m, nd, douts.p, rank_of.p, esz.p, eoff.p);
  if (Lv > 0) {
    Buf<uint32_t> key(c.pool, Lv);
    Buf<int32_t> val(c.pool, Lv);
    const int64_t nwaves = (Lv + (64 / kNetG) * kNetRun - 1) / ((64 / kNetG) * kNetRun);
    VMO_LAUNCH(k_net_node, (unsigned)((nwaves + kT / 64 - 1) / (kT / 64)), kT, 0, s, dsub.p, m, Lv, leafh.p,
               rank_of.p, douts.p, keybase.p, key.p, val.p);
    Buf<int64_t> kc(c.pool, kt + 1);
    fill_i64(kc.p, 0, kt + 1, s);
    VMO_LAUNCH(k_net_count, gsz(Lv), kT, 0, s, key.p, Lv, kc.p);
    scan_exclusive<int64_t>(c, kc.p, kc.p, kt, kc.p + kt, s);
    radix_sort<uint32_t>(c, key.p, val.p, Lv, bits_for((uint64_t)kt), s);
    VMO_LAUNCH(k_net_split, gsz(kt * 64), kT, 0, s, dsub.p, m, keybase.p, kt, kc.p, val.p, nd, dcost.p, douts.p);
    VMO_LAUNCH(k_net_out, gsz(Lv), kT, 0, s, dsub.p, m, Lv, val.p, douts.p);
    VMO_LAUNCH(k_net_ptr, m, kT, 0, s, dsub.p, m, kc.p, keybase.p, douts.p);
  }
}

}  // namespace vmo

namespace vmo {
void bisect_outputs(Engine& e, uint8_t* side, float* centres, int split) {
  SegArrays sg = e.view(e.cur);
  VMO_LAUNCH(k_bisect_out, gsz(e.N), kT, 0, e.s, e.dj.p, sg, e.side.p, e.N, side, split);
  VMO_LAUNCH(k_bisect_centres, 1, 64, 0, e.s, e.dj.p, sg, centres, split);
}
}  // namespace vmo

// ============================================================ serving ====
namespace vmo {

__global__ void k_quantize_range(const JobDev* jd, const float* x, int32_t k, int64_t voff, int64_t Np, uint32_t* q,
                                 int32_t* id, int32_t* pos) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    double s = jd->scale;
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
      if (s > 0.0) {
        double t = ((double)x[(int64_t)d * k + i] - (double)jd->lo[d]) * s;
        double f = floor(t);
        v = f >= (double)kQMax ? kQMax : (uint32_t)f;
      }
      q[d * Np + voff + i] = v;
    }
    id[voff + i] = (int32_t)(voff + i);
    pos[voff + i] = (int32_t)(voff + i);
  }
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

void Engine::arena_init(int64_t max_v, int64_t max_nodes, int64_t max_edges, int64_t max_nets, int64_t max_pins,
                        int32_t max_jobs) {
  N = max_v;
  Np = (N + 3) & ~int64_t(3);
  NT = max_nodes;
  E = max_edges;
  L = max_nets;
  npins_ = max_pins;
  nj = max_jobs;
  hj.assign(nj, JobDev());
  for (auto& J : hj) memset(&J, 0, sizeof J);
  dj = Buf<JobDev>(c.pool, nj);
  VMO_HIP(hipMemcpyAsync(dj.p, hj.data(), sizeof(JobDev) * nj, hipMemcpyHostToDevice, s));
  q = Buf<uint32_t>(c.pool, 4 * Np);
  q2 = Buf<uint32_t>(c.pool, 4 * Np);
  id = Buf<int32_t>(c.pool, Np);
  id2 = Buf<int32_t>(c.pool, Np);
  pos = Buf<int32_t>(c.pool, Np);
  side = Buf<uint8_t>(c.pool, Np);
  segpos = Buf<int32_t>(c.pool, Np);
  segpack = Buf<int32_t>(c.pool, (Np >> 2) + 2);
  VMO_LAUNCH(k_fill_u32, gsz(4 * Np), kT, 0, s, q.p, 0u, 4 * Np);
  iota_i32(id.p, Np, s);
  iota_i32(pos.p, Np, s);
  nd_state = Buf<int32_t>(c.pool, NT);
  nd_K = Buf<int32_t>(c.pool, NT);
  nd_p0 = Buf<int32_t>(c.pool, NT);
  nd_beg = Buf<int64_t>(c.pool, NT);
  nd_end = Buf<int64_t>(c.pool, NT);
  fill_i32(nd_state.p, kNodeNone, NT, s);
  edges = Buf<int32_t>(c.pool, 2 * (E > 0 ? E : 1));
  fill_i32(edges.p, 0, 2 * (E > 0 ? E : 1), s);
  nptr = Buf<int64_t>(c.pool, L + 1);
  fill_i64(nptr.p, 0, L + 1, s);
  npins_buf = Buf<int32_t>(c.pool, max_pins > 0 ? max_pins : 1);
  alloc_segments(cur, 1024);
  S = 0;
  VMO_HIP(hipStreamSynchronize(s));
}

void Engine::append_root(int32_t slot) {
  const JobDev& J = hj[slot];
  if (S + 1 > cur.cap) {
    SegBufs bigger;
    alloc_segments(bigger, 2 * (S + 1));
    if (S > 0) copy_segments(cur, bigger, S);
    cur = std::move(bigger);
  }
  int64_t b = J.voff, e = J.voff + J.k;
  int32_t jb = slot, h = 1, K = J.P, p0 = 0;
  VMO_HIP(hipMemcpyAsync(cur.beg.p + S, &b, 8, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.end.p + S, &e, 8, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.job.p + S, &jb, 4, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.h.p + S, &h, 4, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.K.p + S, &K, 4, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.p0.p + S, &p0, 4, hipMemcpyHostToDevice, s));
  VMO_HIP(hipStreamSynchronize(s));
  ++S;
  // the level kernels find a position's segment by binary search over the
  // segment starts: keep the list sorted (a reused low range may come last)
  std::vector<int64_t> hb(S), he(S);
  std::vector<int32_t> hjb(S), hh(S), hK(S), hp(S);
  VMO_HIP(hipMemcpyAsync(hb.data(), cur.beg.p, 8 * S, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipMemcpyAsync(he.data(), cur.end.p, 8 * S, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipMemcpyAsync(hjb.data(), cur.job.p, 4 * S, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipMemcpyAsync(hh.data(), cur.h.p, 4 * S, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipMemcpyAsync(hK.data(), cur.K.p, 4 * S, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipMemcpyAsync(hp.data(), cur.p0.p, 4 * S, hipMemcpyDeviceToHost, s));
  VMO_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> idx(S);
  for (int64_t i = 0; i < S; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return hb[a] < hb[b]; });
  std::vector<int64_t> sb(S), se(S);
  std::vector<int32_t> sj(S), sh(S), sK(S), sp(S);
  for (int64_t i = 0; i < S; ++i) {
    sb[i] = hb[idx[i]]; se[i] = he[idx[i]]; sj[i] = hjb[idx[i]]; sh[i] = hh[idx[i]]; sK[i] = hK[idx[i]];
    sp[i] = hp[idx[i]];
  }
  VMO_HIP(hipMemcpyAsync(cur.beg.p, sb.data(), 8 * S, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.end.p, se.data(), 8 * S, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.job.p, sj.data(), 4 * S, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.h.p, sh.data(), 4 * S, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.K.p, sK.data(), 4 * S, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cur.p0.p, sp.data(), 4 * S, hipMemcpyHostToDevice, s));
  VMO_HIP(hipStreamSynchronize(s));
}

void Engine::arena_admit(int32_t slot, const JobHost& H, int64_t voff, int64_t node_base, int64_t eoff, int64_t noff,
                         int64_t pinoff) {
  JobDev D;
  memset(&D, 0, sizeof D);
  D.voff = voff; D.k = H.h.k; D.P = H.P; D.mode = H.mode; D.ord = H.order;
  D.seed = H.seed; D.job_index = H.job_index; D.node_base = node_base; D.nnets = H.h.l;
  D.eoff = eoff; D.noff = noff;
  // quantization of this job alone
  Buf<JobDev> one(c.pool, 1);
  D.voff = 0;
  VMO_HIP(hipMemcpyAsync(one.p, &D, sizeof D, hipMemcpyHostToDevice, s));
  Buf<uint32_t> box(c.pool, 8);
  uint32_t hb[8] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u, 0u};
  VMO_HIP(hipMemcpyAsync(box.p, hb, sizeof hb, hipMemcpyHostToDevice, s));
  VMO_LAUNCH(k_bbox, nblocks(D.k, kT), kT, 0, s, one.p, 1, H.x, (int64_t)D.k, (int64_t)D.k, box.p);
  VMO_LAUNCH(k_job_scale, 1, 64, 0, s, one.p, 1, box.p);
  VMO_LAUNCH(k_quantize_range, gsz(D.k), kT, 0, s, one.p, H.x, D.k, voff, Np, q.p, id.p, pos.p);
  read_bytes(&D, one.p, sizeof D, s);
  D.voff = voff;
  hj[slot] = D;
  VMO_HIP(hipMemcpyAsync(dj.p + slot, &D, sizeof D, hipMemcpyHostToDevice, s));
  // node table of the job, root node
  fill_i32(nd_state.p + node_base, kNodeNone, 4 * (int64_t)D.P, s);
  VMO_LAUNCH(k_init_roots, 1, 64, 0, s, dj.p + slot, 1, nodes());
  // edges or nets with global (arena) vertex ids
  if (H.mode == VMO_GRAPH) {
    if (H.h.l > 0) launch_offset_copy_i32(H.h.pins, edges.p + 2 * eoff, 2 * (int64_t)H.h.l, (int32_t)voff);
  } else if (H.h.l > 0) {
    launch_offset_copy_ptr(H.h.net_ptr, nptr.p + noff, (int64_t)H.h.l + 1, pinoff);
    int64_t np = read1(H.h.net_ptr + H.h.l, s);
    if (np > 0) launch_offset_copy_i32(H.h.pins, npins_buf.p + pinoff, np, (int32_t)voff);
  }
  if (H.mode == VMO_NET) {
    // the emission reads the arena copies (global vertex ids already)
    hj[slot].nets_ptr = nptr.p + noff;
    hj[slot].nets_pins = npins_buf.p;
    hj[slot].pin_vadd = 0;
    VMO_HIP(hipMemcpyAsync(dj.p + slot, &hj[slot], sizeof(JobDev), hipMemcpyHostToDevice, s));
  }
  VMO_HIP(hipStreamSynchronize(s));
  if (D.k >= 2 && D.P > 1) append_root(slot);
}

void Engine::arena_release(int32_t slot) {
  const JobDev& J = hj[slot];
  if (J.mode == VMO_GRAPH && J.nnets > 0) fill_i32(edges.p + 2 * J.eoff, 0, 2 * (int64_t)J.nnets, s);
  fill_i32(nd_state.p + J.node_base, kNodeNone, 4 * (int64_t)J.P, s);
  VMO_HIP(hipStreamSynchronize(s));
  memset(&hj[slot], 0, sizeof(JobDev));
}

void Engine::tick(int t_max) {
  if (S == 0) return;
  // the arenas are sized for the whole budget: the level runs over the hull
  // of the position and edge ranges of the jobs that have segments, not over
  // the arenas (positions and edges inside the hull that belong to no segment
  // are passed over as in any level)
  std::vector<int32_t> sj = segment_jobs();
  std::sort(sj.begin(), sj.end());
  sj.erase(std::unique(sj.begin(), sj.end()), sj.end());
  int64_t p0 = Np, p1 = 0, e0 = E, e1 = 0;
  for (int32_t j : sj) {
    const JobDev& J = hj[j];
    p0 = std::min(p0, J.voff);
    p1 = std::max(p1, J.voff + (int64_t)J.k);
    if (J.mode == VMO_GRAPH && J.nnets > 0) {
      e0 = std::min(e0, J.eoff);
      e1 = std::max(e1, J.eoff + (int64_t)J.nnets);
    }
  }
  if (p1 <= p0) { p0 = 0; p1 = Np; }
  p1 = std::min(Np, (p1 + 3) & ~int64_t(3));
  if (e1 <= e0) { e0 = 0; e1 = 0; }
  SegBufs nx;
  alloc_segments(nx, 2 * S);
  two_means(0, S, p0, p1, t_max, true);
  separator(0, S, p0, p1, e0, e1);
  int64_t nn = partition(0, S, p0, p1, nx, 0);
  cur = std::move(nx);
  S = nn;
}

std::vector<int32_t> Engine::segment_jobs() {
  std::vector<int32_t> v(S);
  if (S > 0) {
    VMO_HIP(hipMemcpyAsync(v.data(), cur.job.p, 4 * S, hipMemcpyDeviceToHost, s));
    VMO_HIP(hipStreamSynchronize(s));
  }
  return v;
}

}  // namespace vmo
