// Multilevel layout on the GPU (Sec. 2): components (Algorithm 1),
// coarsening by greedy heavy-net matching (Sec. 2.3), the 2^d-tree with
// cluster charges and its sibling-link walk (Algorithm 3, Sec. 2.1), steepest
// descent steps (Algorithm 3), prolongation (Algorithm 2) and packing of the
// components side by side.
//
// Every floating-point step follows a fixed operation order (no contraction):
// net centres and attraction sum in CSR order, the walk visits nodes in
// pre-order, tree charges sum bottom-up in FP64, so one descent step gives the
// same bits as a sequential evaluation of the same definition.
#include <algorithm>
#include <type_traits>

#include "vmo_internal.h"

namespace vmo {

constexpr int kLT = 256;
constexpr int kParts = 16;  // a cell has at most 16 children
static unsigned gsz(int64_t n) {
  int64_t b = (n + kLT - 1) / kLT;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}
#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ================================================================= level ====
struct Level {
  int32_t k = 0, l = 0;
  int64_t np = 0;
  Buf<int64_t> ptr, dptr;
  Buf<int32_t> pins, dpins;
  Buf<float> w, c;
  Buf<int32_t> pi;  // map to the next coarser level
  // vertices of more than kHeavyDeg nets: [0] their count, then the vertices
  // (in no particular order); heavy_cap bounds the count (np / (kHeavyDeg+1))
  Buf<int32_t> heavy;
  int64_t heavy_cap = 0;
};

// A vertex of more than kHeavyDeg nets takes a wavefront of its own in the
// attraction and the matching: with one thread per vertex, the thread of a
// vertex of thousands of nets would hold its wavefront (and its kernel) long
// after the others are done.  The per-vertex results do not depend on which
// form computes them.
constexpr int32_t kHeavyDeg = 32;
constexpr int64_t kHeavyBlocks = 1024;  // most blocks of kLT / 64 wavefronts given to them
__global__ void k_heavy_list(const int64_t* dptr, int32_t k, int32_t* heavy) {
  GRID_STRIDE(v, k) {
    if (dptr[v + 1] - dptr[v] > kHeavyDeg) heavy[1 + atomicAdd(heavy, 1)] = (int32_t)v;
  }
}
// blocks of kLT threads for the heavy vertices of L (0: none can exist)
static int64_t heavy_blocks(const Level& L) {
  const int64_t nw = kLT / 64;
  return std::min(kHeavyBlocks, (L.heavy_cap + nw - 1) / nw);
}

static void make_dual(Ctx& C, Level& L, hipStream_t s) {
  L.dptr = Buf<int64_t>(C.pool, (size_t)L.k + 1);
  L.dpins = Buf<int32_t>(C.pool, L.np > 0 ? L.np : 1);
  csr_transpose(C, L.l, L.k, L.ptr.p, L.pins.p, L.dptr.p, L.dpins.p, s);
  // the degrees sum to np, so at most np / (kHeavyDeg + 1) vertices exceed it
  L.heavy_cap = std::min<int64_t>(L.k, L.np / (kHeavyDeg + 1));
  L.heavy = Buf<int32_t>(C.pool, (size_t)L.heavy_cap + 1);
  fill_i32(L.heavy.p, 0, 1, s);
  if (L.heavy_cap > 0) VMO_LAUNCH(k_heavy_list, gsz(L.k), kLT, 0, s, L.dptr.p, L.k, L.heavy.p);
}

// ============================================================ bounding box ==
__global__ __launch_bounds__(kLT) void k_box(const float4* x, int32_t k, uint32_t* box) {
  __shared__ uint32_t sm[kLT / 64][8];
  uint32_t mn[4], mx[4];
  for (int d = 0; d < 4; ++d) { mn[d] = 0xffffffffu; mx[d] = 0u; }
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    const float4 xv = x[v];
    const float c[4] = {xv.x, xv.y, xv.z, xv.w};
    for (int d = 0; d < 4; ++d) {
      uint32_t f = fkey(c[d]);
      mn[d] = f < mn[d] ? f : mn[d];
      mx[d] = f > mx[d] ? f : mx[d];
    }
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int d = 0; d < 4; ++d) {
      uint32_t a = __shfl_xor(mn[d], off, 64), b = __shfl_xor(mx[d], off, 64);
      mn[d] = a < mn[d] ? a : mn[d];
      mx[d] = b > mx[d] ? b : mx[d];
    }
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int d = 0; d < 4; ++d) { sm[w][d] = mn[d]; sm[w][4 + d] = mx[d]; }
  __syncthreads();
  if (threadIdx.x < 8) {
    int f = threadIdx.x;
    uint32_t r = sm[0][f];
    for (int i = 1; i < kLT / 64; ++i) r = f < 4 ? (sm[i][f] < r ? sm[i][f] : r) : (sm[i][f] > r ? sm[i][f] : r);
    if (f < 4) atomicMin(&box[f], r); else atomicMax(&box[f], r);
  }
}
__global__ void k_box_init(uint32_t* box) {
  int t = threadIdx.x;
  if (t < 4) box[t] = 0xffffffffu;
  else if (t < 8) box[t] = 0u;
}

struct HostBox {
  float lo[4], hi[4];
};

// reset: dbox already holds the empty box (the previous step's combine left it so)
static void box_of(const float4* x, int32_t k, uint32_t* dbox, hipStream_t s, bool reset = false) {
  if (!reset) VMO_LAUNCH(k_box_init, 1, 64, 0, s, dbox);
  // at most 128 blocks: the 8 atomics of every block meet on one cache line
  int64_t nb = nblocks(k, kLT);
  VMO_LAUNCH(k_box, (unsigned)(nb < 128 ? nb : 128), kLT, 0, s, x, k, dbox);
}
static HostBox read_box(const uint32_t* dbox, hipStream_t s) {
  uint32_t b[8];
  read_bytes(b, dbox, sizeof b, s);
  HostBox h;
  for (int d = 0; d < 4; ++d) { h.lo[d] = fkey_inv(b[d]); h.hi[d] = fkey_inv(b[4 + d]); }
  return h;
}

// =================================================================== tree ===
// Grid coordinate of a point: floor((x - lo) * 65536 / ext), clamped to
// 65535; ext = largest side of the bounding box (FP64).
__device__ __forceinline__ void grid_coords_of(const float4 xv, const uint32_t* box, uint32_t* kq) {
  const float c[4] = {xv.x, xv.y, xv.z, xv.w};
  double ext = 0.0;
  float lo[4];
  for (int d = 0; d < 4; ++d) {
    lo[d] = fkey_inv(box[d]);
    double e = (double)fkey_inv(box[4 + d]) - (double)lo[d];
    if (e > ext) ext = e;
  }
  double sc = ext > 0.0 ? 65536.0 / ext : 0.0;
  for (int d = 0; d < 4; ++d) {
    uint32_t a = 0;
    if (sc > 0.0) {
      double f = floor(((double)c[d] - (double)lo[d]) * sc);
      a = f >= 65535.0 ? 65535u : (uint32_t)f;
    }
    kq[d] = a;
  }
}
__device__ __forceinline__ void grid_coords(const float4* x, int64_t v, const uint32_t* box, uint32_t* kq) {
  grid_coords_of(x[v], box, kq);
}

// Bit b of x (b < 16) to bit 4b, and back (shift-and-mask stages).
__device__ __forceinline__ uint64_t spread4(uint32_t x) {
  uint64_t v = x & 0xffffu;
  v = (v | (v << 24)) & 0x000000ff000000ffull;
  v = (v | (v << 12)) & 0x000f000f000f000full;
  v = (v | (v << 6)) & 0x0303030303030303ull;
  v = (v | (v << 3)) & 0x1111111111111111ull;
  return v;
}
__device__ __forceinline__ uint32_t compact4(uint64_t v) {
  v &= 0x1111111111111111ull;
  v = (v | (v >> 3)) & 0x0303030303030303ull;
  v = (v | (v >> 6)) & 0x000f000f000f000full;
  v = (v | (v >> 12)) & 0x000000ff000000ffull;
  v = (v | (v >> 24)) & 0xffffull;
  return (uint32_t)v;
}
// Morton key: digit at depth L (1..16) = bits (16-L) of the four coordinates,
// dimension 0 most significant; depth-1 digit in the top nibble (bit b of
// coordinate d at bit 4b + 3 - d).
__device__ __forceinline__ uint64_t morton4(const uint32_t* kq) {
  return (spread4(kq[0]) << 3) | (spread4(kq[1]) << 2) | (spread4(kq[2]) << 1) | spread4(kq[3]);
}
__global__ void k_tree_keys(const float4* x, int32_t k, const uint32_t* box, uint64_t* key, int32_t* val) {
  GRID_STRIDE(v, k) {
    uint32_t kq[4];
    grid_coords(x, v, box, kq);
    key[v] = morton4(kq);
    val[v] = (int32_t)v;
  }
}

// Points in tree order: coordinates, weights and 2 kq + 1 (doubled grid units).
__global__ void k_tree_points(const float4* x, const float* w, int32_t k, const uint32_t* box, const int32_t* order,
                              float* xs, float* ws, int32_t* p2, float4* P) {
  GRID_STRIDE(j, k) {
    int32_t v = order[j];
    uint32_t kq[4];
    grid_coords(x, v, box, kq);
    const float4 xv = x[v];
    const float c[4] = {xv.x, xv.y, xv.z, xv.w};
    for (int d = 0; d < 4; ++d) {
      xs[(int64_t)d * k + j] = c[d];
      p2[(int64_t)d * k + j] = 2 * (int32_t)kq[d] + 1;
    }
    P[j] = make_float4(c[0], c[1], c[2], c[3]);
    ws[j] = w ? w[v] : 1.0f;
  }
}

constexpr int kCplB = 256;  // the prefix lengths are allocated in multiples of it

// End of the node of depth L beginning at position i: the first j > i whose
// key differs from key[i] in its first L digits (keys are sorted, so these
// positions form a suffix), found by doubling then bisection.
__device__ int32_t node_end(const uint64_t* key, int32_t k, int32_t i, int L) {
  if (L == 0) return k;
  const int sh = 64 - 4 * L;
  const uint64_t pre = key[i] >> sh;
  int32_t lo = i;  // key[lo] has the prefix
  int64_t step = 1;
  int32_t hi;
  while (true) {
    int64_t h = lo + step;
    if (h >= k) { hi = k; break; }
    if ((key[h] >> sh) != pre) { hi = (int32_t)h; break; }
    lo = (int32_t)h;
    step <<= 1;
  }
  while (hi - lo > 1) {
    int32_t mid = lo + (hi - lo) / 2;
    if ((key[mid] >> sh) == pre) lo = mid; else hi = mid;
  }
  return hi;
}

// Depth of the leaf holding point i: the smallest L whose run (the maximal
// interval of equal L-digit prefixes around i) has <= cap points, else 16.  A
// run of <= cap points lies inside [i-cap+1, i+cap].  Nodes beginning at i
// have depths cpl[i]+1 .. leaf depth.
// Leaf depth of position i (cap <= 16): the smallest L at which the depth-L
// cell holding i has at most cap points.  The cell at depth L is bounded by
// the nearest positions with cpl < L on each side; with ml(u) the minimum of
// cpl over [i - u, i] and mr(v) that over [i + 1, i + 1 + v] (both
// non-increasing), the cell fits when ml(u) < L and mr(v) < L for some
// u + v + 1 <= cap, so L = min over u of max(ml(u), mr(cap - 1 - u)) + 1
// (positions outside [lo, hi] left out), at most 16.  One pass each way.
template <class CplAt>
__device__ __forceinline__ int leaf_depth16(CplAt cpl_at, int32_t i, int32_t lo, int32_t hi, int32_t cap) {
  int r[16];
  int run = 127;
#pragma unroll
  for (int uu = 15; uu >= 0; --uu) {
    if (uu < cap) {
      const int32_t p = i + cap - uu;
      if (p <= hi) run = min(run, (int)cpl_at(p));
    }
    r[uu] = run;
  }
  int L = 127, runl = 127;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    if (u < cap && i - u >= lo) {
      runl = min(runl, (int)cpl_at(i - u));
      L = min(L, max(runl, r[u]) + 1);
    }
  }
  return L > 16 ? 16 : L;
}

// Common-prefix length cpl[i] of sorted keys i-1 and i in 4-bit digits (16
// when equal, -1 at 0 and k), and the leaf depth and the number of nodes
// beginning at each position, in one launch: a block forms the prefix lengths
// of its kLT positions and of cap positions on each side in LDS, writes its
// own and finds the leaf depths from LDS (cap <= kCplHalo, the largest leaf
// capacity).  nnp[b] = the node counts' sum over positions [b kLT, (b+1) kLT),
// for the scan of the counts.
constexpr int kCplHalo = 64;
static_assert(kLT == kScanPart, "a block's positions are one group of the scan");
__global__ __launch_bounds__(kLT) void k_cpl_ell(const uint64_t* key, int32_t k, int32_t cap, int8_t* cpl,
                                                int8_t* ell, int32_t* nn, int32_t* nnp) {
  __shared__ int8_t sc[kLT + 2 * kCplHalo];
  __shared__ int32_t wsum[kLT / 64];
  for (int64_t b0 = (int64_t)blockIdx.x * kLT; b0 <= k; b0 += (int64_t)gridDim.x * kLT) {
    const int64_t w0 = b0 - cap;  // sc[q] = cpl[w0 + q]
    for (int q = threadIdx.x; q < kLT + 2 * cap; q += kLT) {
      const int64_t p = w0 + q;
      int c = -1;  // positions 0 and k (and any outside [0, k], never read)
      if (p > 0 && p < k) {
        const uint64_t d = key[p - 1] ^ key[p];
        c = d == 0 ? 16 : (__clzll(d) >> 2);
      }
      sc[q] = (int8_t)c;
    }
    __syncthreads();
    const int64_t i64 = b0 + threadIdx.x;
    int32_t cnt = 0;
    if (i64 <= k) {
      const int32_t i = (int32_t)i64;
      auto cpl_at = [&](int64_t p) { return (int)sc[p - w0]; };
      cpl[i] = (int8_t)cpl_at(i);
      if (i == k) {
        nn[k] = 0;
      } else {
        const int lo = i - cap + 1 < 0 ? 0 : i - cap + 1;
        const int hi = i + cap > k ? k : i + cap;
        int L = 0;
        if (cap <= 16) {
          L = leaf_depth16([&](int32_t p) { return cpl_at(p); }, i, lo, hi, cap);
        } else {
          for (; L <= 16; ++L) {
            int b = -1, e = -1;
            for (int j = i; j >= lo; --j)
              if (cpl_at(j) < L) { b = j; break; }
            for (int j = i + 1; j <= hi; ++j)
              if (cpl_at(j) < L) { e = j; break; }
            if (b >= 0 && e >= 0 && e - b <= cap) break;
          }
          if (L > 16) L = 16;
        }
        ell[i] = (int8_t)L;
        const int ci = cpl_at(i);
        cnt = L >= ci + 1 ? L - ci : 0;
        nn[i] = cnt;
      }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t a = 0;
      for (int w = 0; w < kLT / 64; ++w) a += wsum[w];
      nnp[b0 / kLT] = a;
    }
    __syncthreads();
  }
}

// Far-field thresholds per depth: the node at depth L is far iff D2 >= T[L],
// D2 = squared distance point-to-cell-centre in doubled grid units (an exact
// integer below 2^40, so exact in FP64).  T[L] is the smallest integer D2
// for which s^2 < theta^2 D2 holds in FP64 (s = doubled cell side); the
// predicate is monotone in D2, so both forms decide every node alike.
struct FarTable {
  double T[17];
};
static FarTable far_table(double th2) {
  FarTable f;
  for (int L = 0; L <= 16; ++L) {
    int64_t s2 = (int64_t)2 << (16 - L);
    double lhs = (double)(s2 * s2);
    if (!(th2 > 0.0)) { f.T[L] = 1e300; continue; }
    int64_t lo = 0, hi = (int64_t)1 << 42;  // hi always satisfies the predicate
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (lhs < th2 * (double)mid) hi = mid; else lo = mid + 1;
    }
    f.T[L] = (double)lo;
  }
  return f;
}

// One tree node as the walk reads it (80 bytes, five 16-byte chunks).  The
// far test of a point q against the cell centre c (both in doubled grid
// units), |q - c|^2 >= T (T from the FarTable of the cell's depth), is kept
// as |q|^2 + A.q >= Tq with A = -2 c and Tq = T - |c|^2: every term is an
// integer below 2^42, so the FP64 fused multiply-adds are exact and the two
// forms decide every point alike.
struct alignas(16) TNode {
  double A[4];  // -2 c (chunks 0 and 1)
  int4 b;       // next, first, count, depth | leaf << 8 (chunk 2)
  float4 X;     // charge centre (chunk 3)
  double Tq;    // T - |c|^2 (chunk 4)
  float W;      // charge
  float pad;
};
static_assert(sizeof(TNode) == 80, "TNode is five 16-byte chunks");

// The cell geometry of a node: centre cc (doubled grid units), threshold T.
__device__ __forceinline__ void node_geom(TNode& nd, const int4& cc, double T) {
  const double c0 = cc.x, c1 = cc.y, c2 = cc.z, c3 = cc.w;
  nd.A[0] = -2.0 * c0; nd.A[1] = -2.0 * c1; nd.A[2] = -2.0 * c2; nd.A[3] = -2.0 * c3;
  nd.Tq = T - __builtin_fma(c3, c3, __builtin_fma(c2, c2, __builtin_fma(c1, c1, c0 * c0)));
}

// Far test of the point with coordinates qd (doubled grid units, as FP64)
// and q2 = |qd|^2 against a node: exact, as above.
__device__ __forceinline__ bool far_q(const double* qd, double q2, const double* A, double Tq) {
  double D = __builtin_fma(A[0], qd[0], q2);
  D = __builtin_fma(A[1], qd[1], D);
  D = __builtin_fma(A[2], qd[2], D);
  D = __builtin_fma(A[3], qd[3], D);
  return D >= Tq;
}
__device__ __forceinline__ double norm2_q(const double* qd) {
  return __builtin_fma(qd[3], qd[3], __builtin_fma(qd[2], qd[2], __builtin_fma(qd[1], qd[1], qd[0] * qd[0])));
}

struct NodeView {
  TNode* t;
  double* Wd;
  double* Sd;  // [n][4]
  int32_t* nch;
  int32_t* ctr;  // depth lists of the one-block build
  int32_t* cid;  // [n][16] children in order (a cell has at most 16 sub-cells)
  int32_t* plan;  // [kPlan] launch order of the walk's part rows (walk_plan)
};

// The walk's launch plan.  A part row of the walk (the root's child i1 and,
// spread, its child i2) has a node (that grandchild, or the child itself);
// the points inside it walk its whole subtree and are the longest walks.  The
// walk's grid first gives those points wavefronts of heavy_pts(k) (short unions,
// so the longest wavefronts shrink), rows with the most such points first,
// then the rows' other points in wavefronts of 64, rows in the same order and
// each row's blocks starting at its node's points.  Which wavefront walks which
// row and points changes no point's walk or sums.
// Points per heavy wavefront at a level of k points: few where the level's
// walk is bound by its longest wavefronts (the chip is not full), up to a whole
// wavefront where it fills the chip and shared unions save work (measured on
// the 64^3 hierarchy's levels).
__host__ __device__ constexpr int heavy_pts(int64_t k) {
  return k < 5000 ? 4 : k < 20000 ? 8 : k < 60000 ? 16 : k < 100000 ? 24 : k < 200000 ? 40 : 64;
}
// plan layout (ints): spread rows (256) then unspread rows (16) of each table
constexpr int kPlP = 0, kPlX = 272, kPlH = 544, kPlF = 818, kPlC = 1090, kPlan = 1362;
// rows in launch order [256 | 16]: kPlP; each row's first 64-point block
// [256 | 16]: kPlX; heavy wavefronts before each launch rank [257 | 17]:
// kPlH; each row's node's first point and point count [256 | 16]: kPlF, kPlC.
// Called by every thread of a block of at least 256 (the first 256 take
// part); sw: 704 ints of LDS.
__device__ void walk_plan(const NodeView& nd, int32_t* sw, int hpts) {
  const int t = threadIdx.x;
  int32_t w16 = -1, x16 = 0, f16 = 0;
  if (t < kParts * kParts) {
    const bool rleaf = (nd.t[0].b.w >> 8) & 1;
    const int n1 = rleaf ? 1 : min(nd.nch[0], kParts);
    const int i1 = t / kParts, i2 = t % kParts;
    if (i1 < n1) {
      const int32_t c1 = rleaf ? 0 : nd.cid[i1];
      const int4 b1 = nd.t[c1].b;
      if (i2 == 0) {
        sw[256 + i1] = b1.z;
        sw[272 + i1] = b1.y / 64;
        sw[288 + i1] = b1.y;
      }
      if ((b1.w >> 8) & 1) {
        if (i2 == 0) { w16 = b1.z; x16 = b1.y / 64; f16 = b1.y; }
      } else if (i2 < min(nd.nch[c1], kParts)) {
        const int4 b2 = nd.t[nd.cid[16 * (int64_t)c1 + i2]].b;
        w16 = b2.z;
        x16 = b2.y / 64;
        f16 = b2.y;
      }
    } else if (i2 == 0) {
      sw[256 + i1] = -1;
      sw[272 + i1] = 0;
      sw[288 + i1] = 0;
    }
    sw[t] = w16;
  }
  // launch order: rows bucketed by the bit length of their node's point
  // count, longest first (any order is correct; the order within a bucket is
  // whatever the atomics give); sw[320..] holds 33 + 33 bucket counts, then
  // the heavy wavefronts by launch rank
  int32_t* bc = sw + 320;   // [33] spread, [33] unspread: counts, then cursors
  int32_t* hc = sw + 400;   // [256] spread, [16] unspread
  if (t < 66) bc[t] = 0;
  __syncthreads();
  const int bk16 = w16 > 0 ? 32 - __clz(w16) : 0;  // 0: no points (last)
  int bk1 = 0;
  if (t < kParts * kParts) atomicAdd(&bc[32 - bk16], 1);
  if (t < kParts) {
    const int32_t w1 = sw[256 + t];
    bk1 = w1 > 0 ? 32 - __clz(w1) : 0;
    atomicAdd(&bc[33 + 32 - bk1], 1);
  }
  __syncthreads();
  if (t == 0) {
    int32_t a = 0;
    for (int i = 0; i < 33; ++i) { const int32_t c = bc[i]; bc[i] = a; a += c; }
    a = 0;
    for (int i = 33; i < 66; ++i) { const int32_t c = bc[i]; bc[i] = a; a += c; }
  }
  __syncthreads();
  if (t < kParts * kParts) {
    const int r = atomicAdd(&bc[32 - bk16], 1);
    nd.plan[kPlP + r] = t;
    nd.plan[kPlX + t] = x16;
    nd.plan[kPlF + t] = f16;
    nd.plan[kPlC + t] = w16 > 0 ? w16 : 0;
    hc[r] = w16 > 0 ? (w16 + hpts - 1) / hpts : 0;
  }
  if (t < kParts) {
    const int32_t w1 = sw[256 + t];
    const int r = atomicAdd(&bc[33 + 32 - bk1], 1);
    nd.plan[kPlP + 256 + r] = t;
    nd.plan[kPlX + 256 + t] = sw[272 + t];
    nd.plan[kPlF + 256 + t] = sw[288 + t];
    nd.plan[kPlC + 256 + t] = w1 > 0 ? w1 : 0;
    hc[256 + r] = w1 > 0 ? (w1 + hpts - 1) / hpts : 0;
  }
  __syncthreads();
  // exclusive prefix of the heavy wavefronts by launch rank: one wavefront,
  // four ranks per lane (spread), and lanes 0..15 (unspread)
  if (t < 64) {
    const int32_t h0 = hc[4 * t], h1 = hc[4 * t + 1], h2 = hc[4 * t + 2], h3 = hc[4 * t + 3];
    const int32_t tot = h0 + h1 + h2 + h3;
    int32_t inc = tot;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t u = __shfl_up(inc, off, 64);
      if (t >= off) inc += u;
    }
    const int32_t ex = inc - tot;
    nd.plan[kPlH + 4 * t] = ex;
    nd.plan[kPlH + 4 * t + 1] = ex + h0;
    nd.plan[kPlH + 4 * t + 2] = ex + h0 + h1;
    nd.plan[kPlH + 4 * t + 3] = ex + h0 + h1 + h2;
    if (t == 63) nd.plan[kPlH + 256] = inc;
    const int32_t g = t < kParts ? hc[256 + t] : 0;
    int32_t inc1 = g;
    for (int off = 1; off < kParts; off <<= 1) {
      const int32_t u = __shfl_up(inc1, off, 64);
      if (t >= off) inc1 += u;
    }
    if (t < kParts) nd.plan[kPlH + 257 + t] = inc1 - g;
    if (t == kParts - 1) nd.plan[kPlH + 257 + kParts] = inc1;
  }
}

// Nodes in pre-order: index = base[i] + (L - cpl[i] - 1) for the node of
// depth L beginning at point i; next = first node beginning at its end.
__global__ void k_tree_nodes(const int8_t* cpl, const uint64_t* key, const int8_t* ell, const int32_t* base,
                             const int32_t* p2, int32_t k, FarTable ft, NodeView nd) {
  GRID_STRIDE(i64, k) {
    int32_t i = (int32_t)i64;
    int ci = cpl[i], li = ell[i];
    if (li < ci + 1) continue;
    for (int L = ci + 1; L <= li; ++L) {
      int32_t t = base[i] + (L - ci - 1);
      int32_t end = node_end(key, k, i, L);
      int side = 1 << (16 - L);
      int4 cc;
      int kq0 = (p2[i] - 1) >> 1, kq1 = (p2[(int64_t)k + i] - 1) >> 1;
      int kq2 = (p2[2 * (int64_t)k + i] - 1) >> 1, kq3 = (p2[3 * (int64_t)k + i] - 1) >> 1;
      cc.x = 2 * ((kq0 >> (16 - L)) << (16 - L)) + side;
      cc.y = 2 * ((kq1 >> (16 - L)) << (16 - L)) + side;
      cc.z = 2 * ((kq2 >> (16 - L)) << (16 - L)) + side;
      cc.w = 2 * ((kq3 >> (16 - L)) << (16 - L)) + side;
      node_geom(nd.t[t], cc, ft.T[L]);
      nd.t[t].b = make_int4(base[end], i, end - i, L | ((L == li ? 1 : 0) << 8));
    }
  }
}

__global__ void k_tree_links(const int32_t* __restrict__ n_dev, NodeView nd) {
  const int32_t n = *n_dev;
  GRID_STRIDE(t64, n) {
    int32_t t = (int32_t)t64;
    int4 b = nd.t[t].b;
    int cnt = 0;
    if (!((b.w >> 8) & 1)) {
      int32_t ch = t + 1;
      while (ch != b.x) {
        if (cnt < 16) nd.cid[16 * (int64_t)t + cnt] = ch;  // a cell has at most 16 sub-cells
        ++cnt;
        ch = nd.t[ch].b.x;
      }
    }
    nd.nch[t] = cnt;
  }
}

__device__ __forceinline__ void node_finish(NodeView nd, int32_t t, double Wd, const double* Sd) {
  nd.Wd[t] = Wd;
  for (int d = 0; d < 4; ++d) nd.Sd[4 * (int64_t)t + d] = Sd[d];
  nd.t[t].W = (float)Wd;
  nd.t[t].X = make_float4((float)(Sd[0] / Wd), (float)(Sd[1] / Wd), (float)(Sd[2] / Wd), (float)(Sd[3] / Wd));
}

// Charge of a leaf: its points [first, first + count) in tree order, in FP64;
// point loads are issued eight points at a time.
__device__ __forceinline__ void leaf_sums(int32_t first, int32_t count, int32_t k, const float* xs, const float* ws,
                                          double& Wd, double* Sd) {
  for (int32_t j0 = first; j0 < first + count; j0 += 8) {
    float wb[8], xb[8][4];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (j0 + u < first + count) {
        wb[u] = ws[j0 + u];
        for (int d = 0; d < 4; ++d) xb[u][d] = xs[(int64_t)d * k + j0 + u];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (j0 + u < first + count) {
        const double wv = (double)wb[u];
        Wd += wv;
        for (int d = 0; d < 4; ++d) Sd[d] += wv * (double)xb[u][d];
      }
    }
  }
}

// Charge of an internal node: its nc children's charges in child order.  The
// children are loaded eight at a time.
__device__ __forceinline__ void child_sums(NodeView nd, int32_t p, int32_t nc, double& W2, double* S2) {
  const int4* cq = reinterpret_cast<const int4*>(nd.cid + 16 * (int64_t)p);
  for (int32_t r0 = 0; r0 < nc; r0 += 8) {
    const int4 c4a = cq[r0 >> 2], c4b = cq[(r0 >> 2) + 1];
    const int32_t cc[8] = {c4a.x, c4a.y, c4a.z, c4a.w, c4b.x, c4b.y, c4b.z, c4b.w};
    double wv[8], sv[8][4];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (r0 + u < nc) {
        wv[u] = nd.Wd[cc[u]];
        for (int d = 0; d < 4; ++d) sv[u][d] = nd.Sd[4 * (int64_t)cc[u] + d];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (r0 + u < nc) {
        W2 += wv[u];
        for (int d = 0; d < 4; ++d) S2[d] += sv[u][d];
      }
    }
  }
}

// Charges without cross-workgroup waits: workgroup (i1, i2, i3) takes the
// subtree of the node reached from the root through child i1, then child i2,
// then child i3 (a node range [r, next(r)) in pre-order), or the leaf met on
// the way when i1..i3 below it are zero, and forms its charges bottom-up:
// leaves first, then the internal nodes depth by depth, deepest first, with a
// barrier between depths.  k_moments_top then forms the charges of the
// internal nodes of depths 2, 1 and 0 (and one more workgroup of the first
// launch forms the walk's launch plan).  The sums and their order are those of
// the one-block build: a leaf sums its points in tree order, an internal node
// its children's charges in child order, in FP64.
constexpr int kMomT = 256;
constexpr int kMomD = 3;          // depth of the subtree roots
constexpr int kMomList = 4096;    // internal nodes listed in LDS
__global__ __launch_bounds__(kMomT) void k_moments_sub(int32_t k, const float* xs, const float* ws, NodeView nd) {
  if (blockIdx.x == kParts * kParts * kParts) {
    // the extra block: the walk's launch plan (nodes, counts and children
    // lists are final here; the plan needs no charges)
    __shared__ int32_t sw[704];
    walk_plan(nd, sw, heavy_pts(k));
    return;
  }
  const int idx[kMomD] = {(int)blockIdx.x / (kParts * kParts), (int)(blockIdx.x / kParts) % kParts,
                          (int)blockIdx.x % kParts};
  int32_t r = 0;
  for (int lv = 0; lv < kMomD; ++lv) {
    if ((nd.t[r].b.w >> 8) & 1) {
      for (int u = lv; u < kMomD; ++u)
        if (idx[u] != 0) return;  // the whole block
      break;
    }
    if (idx[lv] >= min(nd.nch[r], kParts)) return;  // the whole block
    r = nd.cid[16 * (int64_t)r + idx[lv]];
  }
  const int32_t lo = r, hi = nd.t[r].b.x;
  // the range's internal nodes are counted by depth while the leaves are
  // summed, then listed by depth in LDS (when they fit), so that each depth
  // of the bottom-up pass visits its own nodes only
  __shared__ int32_t dcnt[18], doff[18];
  __shared__ int32_t dl[kMomList];
  if (threadIdx.x < 18) dcnt[threadIdx.x] = 0;
  __syncthreads();
  for (int32_t t = lo + threadIdx.x; t < hi; t += kMomT) {
    const int4 b = nd.t[t].b;
    if ((b.w >> 8) & 1) {
      double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
      leaf_sums(b.y, b.z, k, xs, ws, Wd, Sd);
      node_finish(nd, t, Wd, Sd);
    } else {
      atomicAdd(&dcnt[b.w & 255], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t a = 0;
    for (int L = 0; L <= 16; ++L) {
      doff[L] = a;
      a += dcnt[L];
      dcnt[L] = doff[L];  // the cursors of the lists
    }
    doff[17] = a;
  }
  __syncthreads();
  const int L0 = nd.t[lo].b.w & 255;
  if (doff[17] <= kMomList) {
    for (int32_t t = lo + threadIdx.x; t < hi; t += kMomT) {
      const int w = nd.t[t].b.w;
      if (!((w >> 8) & 1)) dl[atomicAdd(&dcnt[w & 255], 1)] = t;
    }
    __syncthreads();
    for (int L = 16; L >= L0; --L) {
      if (doff[L] == doff[L + 1]) continue;  // uniform: doff is in LDS
      for (int32_t e = doff[L] + threadIdx.x; e < doff[L + 1]; e += kMomT) {
        const int32_t t = dl[e];
        double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
        child_sums(nd, t, nd.nch[t], Wd, Sd);
        node_finish(nd, t, Wd, Sd);
      }
      __syncthreads();
    }
  } else {
    for (int L = 16; L >= L0; --L) {
      if (doff[L] == doff[L + 1]) continue;
      for (int32_t t = lo + threadIdx.x; t < hi; t += kMomT) {
        const int4 b = nd.t[t].b;
        if ((b.w & 0x1ff) != L) continue;  // internal (leaf bit clear) at depth L
        double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
        child_sums(nd, t, nd.nch[t], Wd, Sd);
        node_finish(nd, t, Wd, Sd);
      }
      __syncthreads();
    }
  }
}

// Internal nodes of depths 2, 1, 0 (one block of kParts^2 threads).
__global__ __launch_bounds__(kParts * kParts) void k_moments_top(NodeView nd) {
  if ((nd.t[0].b.w >> 8) & 1) return;
  const int i1 = threadIdx.x / kParts, i2 = threadIdx.x % kParts;
  const int n1 = min(nd.nch[0], kParts);
  const int32_t c1 = i1 < n1 ? nd.cid[i1] : -1;
  const bool c1int = c1 >= 0 && !((nd.t[c1].b.w >> 8) & 1);
  if (c1int && i2 < min(nd.nch[c1], kParts)) {
    const int32_t c2 = nd.cid[16 * (int64_t)c1 + i2];
    if (!((nd.t[c2].b.w >> 8) & 1)) {
      double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
      child_sums(nd, c2, nd.nch[c2], Wd, Sd);
      node_finish(nd, c2, Wd, Sd);
    }
  }
  __syncthreads();
  if (i2 == 0 && c1int) {
    double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
    child_sums(nd, c1, nd.nch[c1], Wd, Sd);
    node_finish(nd, c1, Wd, Sd);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
    child_sums(nd, 0, nd.nch[0], Wd, Sd);
    node_finish(nd, 0, Wd, Sd);
  }
}

// ------------------------------------------------- attraction, by wavefront ----
// The attraction of eq. (7) for vertices that meet many nets (all the
// vertices of small levels, whose coarse vertices can meet thousands): one
// wavefront per vertex, the lanes form the terms c_e (x - z_e) of 64 nets at a
// time, and lanes 0..3 then sum one coordinate each over them in net order.
// The sum is one dependent chain per coordinate, so its cost per net is one
// add once the terms are staged (the 16-byte LDS reads run ahead of it).
struct AttractJob {
  const int64_t* dptr;
  const int32_t* dpins;
  int32_t k;
  const float* c;
  const float4* x;
  const float4* z;
  float4* y;
  const int32_t* heavy;  // NULL: every vertex; else the listed ones ([0]: count)
};
// staging of one wavefront: the 64 terms by coordinate, rows padded so that
// the four summing lanes read different banks
constexpr int kTbRow = 68;
using AttractStage = float[4][kTbRow];
// NW wavefronts per block; block blk of nblk (the blocks that take part).
template <int NW>
__device__ __forceinline__ void attract_waves(const AttractJob& aj, AttractStage* tb, int64_t blk, int64_t nblk) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nv = aj.heavy ? aj.heavy[0] : aj.k;
  const float* row = tb[wv][lane & 3];
  for (int64_t i = blk * NW + wv; i < nv; i += nblk * NW) {
    const int64_t v = aj.heavy ? aj.heavy[1 + i] : i;
    const int64_t b = aj.dptr[v], e = aj.dptr[v + 1];
    const float4 xv = aj.x[v];
    float acc = 0.0f;
    for (int64_t t0 = b; t0 < e; t0 += 64) {
      const int m = e - t0 < 64 ? (int)(e - t0) : 64;
      float4 term = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (lane < m) {
        const int32_t n = aj.dpins[t0 + lane];
        const float ce = aj.c ? aj.c[n] : 1.0f;
        const float4 zn = aj.z[n];
        const float d0 = xv.x - zn.x, d1 = xv.y - zn.y, d2 = xv.z - zn.z, d3 = xv.w - zn.w;
        term = make_float4(ce * d0, ce * d1, ce * d2, ce * d3);
      }
      // the previous chunk's reads are done before its rows are overwritten
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      tb[wv][0][lane] = term.x;
      tb[wv][1][lane] = term.y;
      tb[wv][2][lane] = term.z;
      tb[wv][3][lane] = term.w;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < 4) {
        if (m == 64) {
          const float4* r4 = reinterpret_cast<const float4*>(row);
#pragma unroll
          for (int q = 0; q < 16; q += 4) {
            const float4 u0 = r4[q], u1 = r4[q + 1], u2 = r4[q + 2], u3 = r4[q + 3];
            acc = acc + u0.x; acc = acc + u0.y; acc = acc + u0.z; acc = acc + u0.w;
            acc = acc + u1.x; acc = acc + u1.y; acc = acc + u1.z; acc = acc + u1.w;
            acc = acc + u2.x; acc = acc + u2.y; acc = acc + u2.z; acc = acc + u2.w;
            acc = acc + u3.x; acc = acc + u3.y; acc = acc + u3.z; acc = acc + u3.w;
          }
        } else {
          for (int j = 0; j < m; ++j) acc = acc + row[j];
        }
      }
    }
    if (lane < 4) reinterpret_cast<float*>(aj.y + v)[lane] = acc;
  }
}

// ------------------------------------------------- one-block tree build ----
// Levels with k <= 4096 build their tree in one 1024-thread block: the same
// keys, stable order, nodes and FP64 charges as the multi-kernel build, with
// the node count written to device memory, so an iteration of a small level
// needs no host round trip and a handful of launches.
constexpr int kSTB = 1024;
constexpr int kSmallK = 4096;

// grid coordinate of dimension d back from a Morton key (inverse of k_tree_keys)
__device__ __forceinline__ int32_t key_coord(uint64_t m, int d) { return (int32_t)compact4(m >> (3 - d)); }

__global__ __launch_bounds__(kSTB) void k_tree_small(const float4* __restrict__ x, const float* __restrict__ w,
                                                     int32_t k, int32_t cap, uint32_t* __restrict__ box,
                                                     FarTable ft, int32_t* __restrict__ order, float* __restrict__ xs,
                                                     float* __restrict__ ws, int32_t* __restrict__ p2,
                                                     float4* __restrict__ P, NodeView nd, int32_t* __restrict__ nn,
                                                     AttractJob aj) {
  // blocks after the first form the attraction of the same step (it does
  // not depend on the tree), on other CUs while block 0 builds the tree
  if (blockIdx.x > 0) {
    __shared__ __align__(16) AttractStage tb[kSTB / 64];
    attract_waves<kSTB / 64>(aj, tb, blockIdx.x - 1, gridDim.x - 1);
    return;
  }
  __shared__ uint64_t key[kSmallK];
  __shared__ __align__(16) unsigned char rb[32768];
  // 32 KB: the second buffer of the merge sort, later the next links and
  // the FP64 charges of small trees
  __shared__ uint16_t cnt[4][16][256];
  // during the sort
  int32_t* val = reinterpret_cast<int32_t*>(rb);                // [4096]
  // after the sort
  int8_t* cpl = reinterpret_cast<int8_t*>(rb);                  // [k + 1]
  int8_t* ell = reinterpret_cast<int8_t*>(rb + 4112);           // [k]
  int32_t* base = reinterpret_cast<int32_t*>(rb + 8224);        // [k + 1]
  int32_t* tsum = reinterpret_cast<int32_t*>(rb + 24640);       // [1024]
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

  // the bounding box of x (as k_box), kept in LDS and written to box; the
  // points stay in registers for their keys
  __shared__ uint32_t sbox[8];
  float4 xr[kSmallK / kSTB];
  {
    if (t < 8) sbox[t] = t < 4 ? 0xffffffffu : 0u;
    uint32_t mn[4], mx[4];
    for (int d = 0; d < 4; ++d) { mn[d] = 0xffffffffu; mx[d] = 0u; }
#pragma unroll
    for (int r = 0; r < kSmallK / kSTB; ++r) {
      const int v = r * kSTB + t;
      if (v >= k) break;
      xr[r] = x[v];
      const float c[4] = {xr[r].x, xr[r].y, xr[r].z, xr[r].w};
      for (int d = 0; d < 4; ++d) {
        const uint32_t f = fkey(c[d]);
        mn[d] = min(mn[d], f);
        mx[d] = max(mx[d], f);
      }
    }
    for (int off = 32; off > 0; off >>= 1)
      for (int d = 0; d < 4; ++d) {
        mn[d] = min(mn[d], (uint32_t)__shfl_xor((int)mn[d], off, 64));
        mx[d] = max(mx[d], (uint32_t)__shfl_xor((int)mx[d], off, 64));
      }
    __syncthreads();
    if (lane == 0)
      for (int d = 0; d < 4; ++d) {
        atomicMin(&sbox[d], mn[d]);
        atomicMax(&sbox[4 + d], mx[d]);
      }
    __syncthreads();
    if (t < 8) box[t] = sbox[t];
  }

  // (the four rounds unrolled: their loads are issued together)
#pragma unroll
  for (int r = 0; r < kSmallK / kSTB; ++r) {
    const int v = r * kSTB + t;
    if (v >= k) break;
    uint32_t kq[4];
    grid_coords_of(xr[r], sbox, kq);
    key[v] = morton4(kq);
    val[v] = v;
  }
  __syncthreads();

  if (k <= kSTB) {
    // At most one point per thread: a bitonic sort of the (key, index) pairs,
    // which are all distinct, so the result is the stable order by key.  N
    // (a power of two, at least 64) positions; those from k on hold (2^64 - 1,
    // INT_MAX), which sorts after every point.  Partners closer than 64
    // positions are in the same wavefront (shuffles); farther ones are
    // exchanged through LDS.  Every thread runs every step (the barriers).
    int N = 64;
    while (N < k) N <<= 1;
    uint64_t mk = t < k ? key[t] : ~0ull;
    int32_t mv = t < k ? t : 0x7fffffff;
    for (int kk = 2; kk <= N; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        uint64_t ok;
        int32_t ov;
        if (j >= 64) {
          key[t] = mk;
          val[t] = mv;
          __syncthreads();
          ok = key[t ^ j];
          ov = val[t ^ j];
          __syncthreads();
        } else {
          const uint32_t lo = __shfl_xor((uint32_t)mk, j, 64);
          const uint32_t hi = __shfl_xor((uint32_t)(mk >> 32), j, 64);
          ok = ((uint64_t)hi << 32) | lo;
          ov = __shfl_xor(mv, j, 64);
        }
        const bool other_less = ok < mk || (ok == mk && ov < mv);
        // the lower position of a pair keeps the smaller pair in ascending
        // runs ((t & kk) == 0) and the larger one in descending runs
        const bool keep_min = ((t & j) == 0) == ((t & kk) == 0);
        if (t < N && other_less == keep_min) {
          mk = ok;
          mv = ov;
        }
      }
    }
    if (t < k) {
      key[t] = mk;
      val[t] = mv;
    }
    __syncthreads();
  }

  if (k > kSTB) {
    // Runs of 256 positions sorted by one wavefront each in registers (a
    // bitonic network; lane l holds positions 4l..4l+3 of its run), then
    // merged pairwise in LDS until one run remains; each merge step gives a
    // thread four consecutive outputs, found by a merge-path search.  The
    // (key, index) pairs are all distinct, so the result is the stable order
    // by key.  N = 2048 or 4096 positions; those from k on hold
    // (2^64 - 1, INT_MAX), which sorts after every point.
    int N = 2 * kSTB;
    while (N < k) N <<= 1;
    const int merges = N == 2 * kSTB ? 3 : 4;  // log2(N / 256)
    uint64_t* kX = key;
    int32_t* vX = val;
    uint64_t* kY = reinterpret_cast<uint64_t*>(&cnt[0][0][0]);  // [4096]
    int32_t* vY = reinterpret_cast<int32_t*>(rb + 16384);       // [4096]
    auto less = [](uint64_t ka, int32_t va, uint64_t kb, int32_t vb) {
      return ka < kb || (ka == kb && va < vb);
    };
    if (wv < N / 256) {
      uint64_t mk[4];
      int32_t mv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = 256 * wv + 4 * lane + q;
        mk[q] = p < k ? key[p] : ~0ull;
        mv[q] = p < k ? val[p] : 0x7fffffff;
      }
      for (int kk = 2; kk <= 256; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
          if (j >= 4) {
            // partner position p ^ j is lane l ^ (j / 4), same slot
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int p = 4 * lane + q;
              const uint32_t lo = __shfl_xor((uint32_t)mk[q], j >> 2, 64);
              const uint32_t hi = __shfl_xor((uint32_t)(mk[q] >> 32), j >> 2, 64);
              const uint64_t ok = ((uint64_t)hi << 32) | lo;
              const int32_t ov = __shfl_xor(mv[q], j >> 2, 64);
              // the lower position of a pair keeps the smaller pair in
              // ascending runs ((p & kk) == 0), the larger in descending ones
              const bool keep_min = ((p & j) == 0) == ((p & kk) == 0);
              if (less(ok, ov, mk[q], mv[q]) == keep_min) {
                mk[q] = ok;
                mv[q] = ov;
              }
            }
          } else {
            // partners in the same lane: slots (q, q | j)
            auto cas = [&](int q, int q2) {
              const bool asc = ((4 * lane + q) & kk) == 0;
              const bool sw = asc ? less(mk[q2], mv[q2], mk[q], mv[q]) : less(mk[q], mv[q], mk[q2], mv[q2]);
              if (sw) {
                const uint64_t tk = mk[q];
                const int32_t tv = mv[q];
                mk[q] = mk[q2];
                mv[q] = mv[q2];
                mk[q2] = tk;
                mv[q2] = tv;
              }
            };
            if (j == 2) {
              cas(0, 2);
              cas(1, 3);
            } else {
              cas(0, 1);
              cas(2, 3);
            }
          }
        }
      }
      // an odd number of merges ends in the other buffer: start there
      uint64_t* kd = (merges & 1) ? kY : kX;
      int32_t* vd = (merges & 1) ? vY : vX;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = 256 * wv + 4 * lane + q;
        kd[p] = mk[q];
        vd[p] = mv[q];
      }
    }
    __syncthreads();
    uint64_t* ks = (merges & 1) ? kY : kX;
    int32_t* vs = (merges & 1) ? vY : vX;
    uint64_t* kt = (merges & 1) ? kX : kY;
    int32_t* vt = (merges & 1) ? vX : vY;
    for (int R = 256; R < N; R <<= 1) {
      const int o = 4 * t;  // N <= 4 * kSTB
      if (o < N) {
        const int a0 = o & ~(2 * R - 1), d = o - a0;
        const uint64_t* kA = ks + a0;
        const int32_t* vA = vs + a0;
        const uint64_t* kB = kA + R;
        const int32_t* vB = vA + R;
        // i = the number of the run A's pairs among the first d outputs
        int lo = d - R > 0 ? d - R : 0, hi = d < R ? d : R;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (less(kA[mid], vA[mid], kB[d - 1 - mid], vB[d - 1 - mid])) lo = mid + 1;
          else hi = mid;
        }
        int i = lo, j = d - lo;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool fromA = j >= R || (i < R && less(kA[i], vA[i], kB[j], vB[j]));
          if (fromA) {
            kt[o + u] = kA[i];
            vt[o + u] = vA[i];
            ++i;
          } else {
            kt[o + u] = kB[j];
            vt[o + u] = vB[j];
            ++j;
          }
        }
      }
      __syncthreads();
      uint64_t* k2 = ks; ks = kt; kt = k2;
      int32_t* v2 = vs; vs = vt; vt = v2;
    }
  }

  // points in tree order (the four rounds unrolled)
#pragma unroll
  for (int r = 0; r < kSmallK / kSTB; ++r) {
    const int j = r * kSTB + t;
    if (j >= k) break;
    const int32_t v = val[j];
    order[j] = v;
    uint32_t kq[4];
    grid_coords(x, v, sbox, kq);
    const float4 xv = x[v];
    const float c[4] = {xv.x, xv.y, xv.z, xv.w};
    for (int d = 0; d < 4; ++d) {
      xs[(int64_t)d * k + j] = c[d];
      p2[(int64_t)d * k + j] = 2 * (int32_t)kq[d] + 1;
    }
    P[j] = make_float4(c[0], c[1], c[2], c[3]);
    ws[j] = w ? w[v] : 1.0f;
  }
  __syncthreads();  // val is dead from here

  for (int i = t; i <= k; i += kSTB) {
    int c;
    if (i == 0 || i == k) c = -1;
    else {
      const uint64_t dd = key[i - 1] ^ key[i];
      c = dd == 0 ? 16 : (__clzll(dd) >> 2);
    }
    cpl[i] = (int8_t)c;
  }
  __syncthreads();
  // leaf depth and the number of nodes beginning at each position (as k_cpl_ell)
  for (int i = t; i <= k; i += kSTB) {
    if (i == k) { base[k] = 0; continue; }
    const int lo = i - cap + 1 < 0 ? 0 : i - cap + 1;
    const int hi = i + cap > k ? k : i + cap;
    int L = 0;
    if (cap <= 16) {
      L = leaf_depth16([&](int32_t p) { return cpl[p]; }, i, lo, hi, cap);
    } else {
      for (; L <= 16; ++L) {
        int b = -1, e = -1;
        for (int jj = i; jj >= lo; --jj)
          if (cpl[jj] < L) { b = jj; break; }
        for (int jj = i + 1; jj <= hi; ++jj)
          if (cpl[jj] < L) { e = jj; break; }
        if (b >= 0 && e >= 0 && e - b <= cap) break;
      }
    }
    if (L > 16) L = 16;
    ell[i] = (int8_t)L;
    const int ci = cpl[i];
    base[i] = L >= ci + 1 ? L - ci : 0;
  }
  __syncthreads();
  // exclusive scan of base[0..k]: five consecutive entries per thread
  {
    const int b0 = 5 * t;
    int loc = 0;
    for (int e = 0; e < 5; ++e)
      if (b0 + e <= k) loc += base[b0 + e];
    // inclusive scan within the wavefront, then the earlier wavefronts' totals
    int inc = loc;
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(inc, off, 64);
      if (lane >= off) inc += u;
    }
    if (lane == 63) tsum[wv] = inc;
    __syncthreads();
    int run2 = inc - loc;
    for (int w2 = 0; w2 < wv; ++w2) run2 += tsum[w2];
    for (int e = 0; e < 5; ++e)
      if (b0 + e <= k) {
        const int c = base[b0 + e];
        base[b0 + e] = run2;
        run2 += c;
      }
  }
  __syncthreads();
  const int32_t n = base[k];
  if (t == 0) nn[k] = n;
  // the next links, kept in LDS for the children lists when they fit (the
  // sort's count area is free from here)
  int32_t* nxt = reinterpret_cast<int32_t*>(&cnt[0][0][0]);
  constexpr int32_t kNxtCap = (int32_t)(sizeof(cnt) / sizeof(int32_t));
  const bool nxt_lds = n <= kNxtCap;
  // nodes in pre-order (as k_tree_nodes), one thread per node: node tn
  // begins at the last position i with base[i] <= tn, at depth
  // cpl[i] + 1 + (tn - base[i])
  for (int32_t tn = t; tn < n; tn += kSTB) {
    int32_t i = 0, hb = k;  // the last i in [0, k) with base[i] <= tn
    while (hb - i > 1) {
      const int32_t mid = (i + hb) >> 1;
      if (base[mid] <= tn) i = mid; else hb = mid;
    }
    const int ci = cpl[i], li = ell[i];
    const int L = ci + 1 + (tn - base[i]);
    const uint64_t ki = key[i];
    int32_t kq[4];
    for (int d = 0; d < 4; ++d) kq[d] = key_coord(ki, d);
    {
      int32_t end = k;
      if (L > 0) {
        const int shf = 64 - 4 * L;
        const uint64_t pre = ki >> shf;
        int32_t lo2 = i, hi2;
        int64_t step = 1;
        while (true) {
          const int64_t h = lo2 + step;
          if (h >= k) { hi2 = k; break; }
          if ((key[h] >> shf) != pre) { hi2 = (int32_t)h; break; }
          lo2 = (int32_t)h;
          step <<= 1;
        }
        while (hi2 - lo2 > 1) {
          const int32_t mid = lo2 + (hi2 - lo2) / 2;
          if ((key[mid] >> shf) == pre) lo2 = mid; else hi2 = mid;
        }
        end = hi2;
      }
      const int side = 1 << (16 - L);
      int4 cc;
      cc.x = 2 * ((kq[0] >> (16 - L)) << (16 - L)) + side;
      cc.y = 2 * ((kq[1] >> (16 - L)) << (16 - L)) + side;
      cc.z = 2 * ((kq[2] >> (16 - L)) << (16 - L)) + side;
      cc.w = 2 * ((kq[3] >> (16 - L)) << (16 - L)) + side;
      node_geom(nd.t[tn], cc, ft.T[L]);
      nd.t[tn].b = make_int4(base[end], i, end - i, L | ((L == li ? 1 : 0) << 8));
      if (nxt_lds) nxt[tn] = base[end] | (L == li ? (int32_t)0x80000000 : 0);
    }
  }
  __syncthreads();
  // children lists (as k_tree_links), the sibling chain followed in LDS
  for (int32_t tn = t; tn < n; tn += kSTB) {
    int cnt2 = 0;
    if (nxt_lds) {
      const int32_t bx = nxt[tn];
      if (bx >= 0) {
        int32_t ch = tn + 1;
        while (ch != bx) {
          if (cnt2 < 16) nd.cid[16 * (int64_t)tn + cnt2] = ch;
          ++cnt2;
          ch = nxt[ch] & 0x7fffffff;
        }
      }
    } else {
      const int4 b = nd.t[tn].b;
      if (!((b.w >> 8) & 1)) {
        int32_t ch = tn + 1;
        while (ch != b.x) {
          if (cnt2 < 16) nd.cid[16 * (int64_t)tn + cnt2] = ch;
          ++cnt2;
          ch = nd.t[ch].b.x;
        }
      }
    }
    nd.nch[tn] = cnt2;
  }
  __syncthreads();
  // nodes grouped by depth (any order within a depth): counts, offsets, lists
  int32_t* dcnt = tsum;        // [17] after the scan above, tsum is free
  int32_t* doff = tsum + 32;   // [18]
  int32_t* dpos = tsum + 64;   // [17]
  if (t < 17) dcnt[t] = 0;
  __syncthreads();
  for (int32_t tn = t; tn < n; tn += kSTB) {
    const int w = nd.t[tn].b.w;
    if (!((w >> 8) & 1)) atomicAdd(&dcnt[w & 255], 1);  // internal nodes only
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int L = 0; L <= 16; ++L) {
      doff[L] = acc;
      dpos[L] = acc;
      acc += dcnt[L];
    }
    doff[17] = acc;
  }
  __syncthreads();
  // Trees of up to kQLds nodes keep the depth lists and the FP64 charges in
  // LDS (the keys' and the sort counts' space is free from here), so a depth
  // of the bottom-up pass reads its children's charges from LDS
  constexpr int32_t kQLds = 1024;
  const bool qlds = n <= kQLds;
  int32_t* ctr = qlds ? base : nd.ctr;                        // the depth lists of internal nodes
  double* qW = reinterpret_cast<double*>(&cnt[0][0][0]);     // [n]
  double* qS = reinterpret_cast<double*>(key);                // [n][4]
  for (int32_t tn = t; tn < n; tn += kSTB) {
    const int w = nd.t[tn].b.w;
    if (!((w >> 8) & 1)) ctr[atomicAdd(&dpos[w & 255], 1)] = tn;
  }
  __syncthreads();
  // charges (same sums and order as k_tree_moments): every leaf first, then
  // the internal nodes depth by depth, deepest first, skipping empty depths
  for (int32_t tn = t; tn < n; tn += kSTB) {
    const int4 b = nd.t[tn].b;
    if (!((b.w >> 8) & 1)) continue;
    double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
    leaf_sums(b.y, b.z, k, xs, ws, Wd, Sd);
    node_finish(nd, tn, Wd, Sd);
    if (qlds) {
      qW[tn] = Wd;
      for (int d = 0; d < 4; ++d) qS[4 * tn + d] = Sd[d];
    }
  }
  __syncthreads();
  for (int L = 16; L >= 0; --L) {
    if (doff[L] == doff[L + 1]) continue;  // uniform: doff is in LDS
    for (int32_t e = doff[L] + t; e < doff[L + 1]; e += kSTB) {
      const int32_t tn = ctr[e];
      const int32_t nc = nd.nch[tn];
      double Wd = 0.0, Sd[4] = {0.0, 0.0, 0.0, 0.0};
      if (qlds) {
        // children in child order, as child_sums, from LDS
        const int4* cq = reinterpret_cast<const int4*>(nd.cid + 16 * (int64_t)tn);
        for (int32_t r0 = 0; r0 < nc; r0 += 4) {
          const int4 c4 = cq[r0 >> 2];
          const int32_t cc[4] = {c4.x, c4.y, c4.z, c4.w};
          for (int u = 0; u < 4 && r0 + u < nc; ++u) {
            Wd += qW[cc[u]];
            for (int d = 0; d < 4; ++d) Sd[d] += qS[4 * cc[u] + d];
          }
        }
        qW[tn] = Wd;
        for (int d = 0; d < 4; ++d) qS[4 * tn + d] = Sd[d];
      } else {
        child_sums(nd, tn, nc, Wd, Sd);
      }
      node_finish(nd, tn, Wd, Sd);
    }
    __syncthreads();
  }
  __shared__ int32_t sw_plan[704];
  walk_plan(nd, sw_plan, heavy_pts(k));
}

struct Tree {
  int32_t k = 0, n = 0;
  Buf<uint64_t> key;
  Buf<int32_t> order, p2, nn, nnp;
  Buf<float> xs, ws;
  Buf<int8_t> cpl, ell;
  Buf<TNode> nodes;
  Buf<float4> P;  // points in tree order
  Buf<double> Wd, Sd;
  Buf<int32_t> nch, ctr, cid, plan;
  NodeView view() {
    NodeView v;
    v.t = nodes.p; v.Wd = Wd.p; v.Sd = Sd.p;
    v.nch = nch.p; v.ctr = ctr.p; v.cid = cid.p; v.plan = plan.p;
    return v;
  }
};

// Build the tree of x (one record per point; weights w or 1) with the bounding box dbox: the
// one-block build (small_ok, k <= kSmallK) computes the box of x itself into
// dbox, the multi-kernel build reads it.  The node count is left on the device
// at T.nn[k] (no host round trip): node arrays are sized for the largest
// possible tree, 17 nodes per position.
static void build_tree(Ctx& C, Tree& T, const float4* x, const float* w, int32_t k, int32_t cap, uint32_t* dbox,
                       double th2, hipStream_t s, bool small_ok = true, const AttractJob* aj = nullptr) {
  T.k = k;
  T.n = -1;
  // at most 17 nodes begin at a position.  The buffers are kept from one
  // build to the next and only grow; during a layout they are sized for its
  // largest level at once, so every level and iteration uses the same blocks.
  const size_t kk = (size_t)std::max<int64_t>(k, C.layout_kmax);
  const size_t nmax = 17 * kk + 1;
  auto grow = [&](auto& b, size_t n) {
    if (!b.p || b.n < n) {
      b.release();
      b = std::remove_reference_t<decltype(b)>(C.pool, n);
    }
  };
  grow(T.order, kk);
  grow(T.xs, 4 * kk);
  grow(T.ws, kk);
  grow(T.p2, 4 * kk);
  grow(T.P, kk);
  grow(T.nn, kk + 1);
  grow(T.nodes, nmax);
  grow(T.Wd, nmax);
  grow(T.Sd, 4 * nmax);
  grow(T.nch, nmax);
  grow(T.cid, 16 * nmax);
  grow(T.plan, kPlan);
  if (small_ok && k > 0 && k <= kSmallK) {
    grow(T.ctr, nmax);
    AttractJob none{};
    const int64_t ab = aj && aj->k > 0 ? nblocks(aj->k, kSTB / 64) : 0;
    VMO_LAUNCH(k_tree_small, (unsigned)(1 + (ab < 256 ? ab : 256)), kSTB, 0, s, x, w, k, cap, dbox, far_table(th2),
               T.order.p, T.xs.p, T.ws.p, T.p2.p, T.P.p, T.view(), T.nn.p, aj ? *aj : none);
    return;
  }
  grow(T.key, kk);
  VMO_LAUNCH(k_tree_keys, gsz(k), kLT, 0, s, x, k, dbox, T.key.p, T.order.p);
  radix_sort<uint64_t>(C, T.key.p, T.order.p, k, 64, s);
  VMO_LAUNCH(k_tree_points, gsz(k), kLT, 0, s, x, w, k, dbox, T.order.p, T.xs.p, T.ws.p, T.p2.p, T.P.p);
  grow(T.cpl, (kk / kCplB + 1) * kCplB);
  grow(T.ell, kk + 1);
  grow(T.nnp, kk / kLT + 1);
  VMO_LAUNCH(k_cpl_ell, gsz((int64_t)k + 1), kLT, 0, s, T.key.p, k, cap, T.cpl.p, T.ell.p, T.nn.p, T.nnp.p);
  if ((int64_t)k + 1 <= kScanPartMax) scan_exclusive_parts(C, T.nn.p, T.nn.p, (int64_t)k + 1, T.nnp.p, s);
  else scan_exclusive<int32_t>(C, T.nn.p, T.nn.p, (int64_t)k + 1, nullptr, s);
  NodeView nd = T.view();
  VMO_LAUNCH(k_tree_nodes, gsz(k), kLT, 0, s, T.cpl.p, T.key.p, T.ell.p, T.nn.p, T.p2.p, k, far_table(th2), nd);
  // the node count stays on the device: grids sized for the usual count
  // (below 2 k), grid-stride loops up to the count
  const int32_t* n_dev = T.nn.p + k;
  VMO_LAUNCH(k_tree_links, gsz(2 * (int64_t)k), kLT, 0, s, n_dev, nd);
  VMO_LAUNCH(k_moments_sub, kParts * kParts * kParts + 1, kMomT, 0, s, k, T.xs.p, T.ws.p, nd);
  VMO_LAUNCH(k_moments_top, 1, kParts * kParts, 0, s, nd);
}

// ============================================================ gradient ====
// Net centres: pins summed in CSR order (each coordinate on its own), then
// divided by the net size.  z is AoS (one 16-byte record per net) so that the
// attraction gathers a centre with one load.
__global__ void k_centres(const int64_t* ptr, const int32_t* pins, int32_t l, const float4* x, float4* z) {
  GRID_STRIDE(e, l) {
    int64_t b = ptr[e], n = ptr[e + 1] - b;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    for (int64_t p = b; p < b + n; ++p) {
      const float4 xv = x[pins[p]];
      a0 = a0 + xv.x;
      a1 = a1 + xv.y;
      a2 = a2 + xv.z;
      a3 = a3 + xv.w;
    }
    float fn = (float)n;
    z[e] = n > 0 ? make_float4(a0 / fn, a1 / fn, a2 / fn, a3 / fn) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}
// Attraction of eq. (7): sum over the vertex's nets in ascending net order.
// Nets are taken eight at a time: their loads are issued together (vertices of
// coarse levels meet many nets), the sums stay in net order.
// Attraction with one thread per vertex; the first hb blocks give the listed
// heavy vertices a wavefront each (attract_waves), the others skip them.
__global__ __launch_bounds__(kLT) void k_attract(AttractJob aj, int32_t hb) {
  if ((int32_t)blockIdx.x < hb) {
    __shared__ __align__(16) AttractStage tb[kLT / 64];
    attract_waves<kLT / 64>(aj, tb, blockIdx.x, hb);
    return;
  }
  constexpr int B = 8;
  const int64_t stride = (int64_t)(gridDim.x - hb) * blockDim.x;
  for (int64_t v = (int64_t)(blockIdx.x - hb) * blockDim.x + threadIdx.x; v < aj.k; v += stride) {
    const int64_t b = aj.dptr[v], e = aj.dptr[v + 1];
    if (aj.heavy && e - b > kHeavyDeg) continue;
    const float4 xv = aj.x[v];
    const float x0 = xv.x, x1 = xv.y, x2 = xv.z, x3 = xv.w;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    for (int64_t t0 = b; t0 < e; t0 += B) {
      int32_t nb[B];
      float cb[B];
      float4 zb[B];
#pragma unroll
      for (int u = 0; u < B; ++u) nb[u] = t0 + u < e ? aj.dpins[t0 + u] : -1;
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (nb[u] >= 0) {
          cb[u] = aj.c ? aj.c[nb[u]] : 1.0f;
          zb[u] = aj.z[nb[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (nb[u] < 0) break;
        const float ce = cb[u];
        const float d0 = x0 - zb[u].x, d1 = x1 - zb[u].y, d2 = x2 - zb[u].z, d3 = x3 - zb[u].w;
        a0 = a0 + ce * d0;
        a1 = a1 + ce * d1;
        a2 = a2 + ce * d2;
        a3 = a3 + ce * d3;
      }
    }
    aj.y[v] = make_float4(a0, a1, a2, a3);
  }
}
// The same attraction with one wavefront per vertex (attract_waves), four
// vertices per block.
__global__ __launch_bounds__(256) void k_attract_wave(AttractJob aj) {
  __shared__ __align__(16) AttractStage tb[4];
  attract_waves<4>(aj, tb, blockIdx.x, gridDim.x);
}
__global__ void k_z_soa(const float4* z, int32_t l, float* out) {
  GRID_STRIDE(e, l) {
    const float4 a = z[e];
    out[e] = a.x;
    out[(int64_t)l + e] = a.y;
    out[2 * (int64_t)l + e] = a.z;
    out[3 * (int64_t)l + e] = a.w;
  }
}

// (d-2) W w_n |X - x|^-4 (X - x), d = 4, operation by operation; the squared
// distance and the accumulation are fused multiply-adds (one rounding each).
__device__ __forceinline__ void interact(float* y, const float* xn, float wn2, float X0, float X1, float X2, float X3,
                                         float W) {
  float dx0 = X0 - xn[0], dx1 = X1 - xn[1], dx2 = X2 - xn[2], dx3 = X3 - xn[3];
  float r2 = dx0 * dx0;
  r2 = __builtin_fmaf(dx1, dx1, r2);
  r2 = __builtin_fmaf(dx2, dx2, r2);
  r2 = __builtin_fmaf(dx3, dx3, r2);
  float num = W * wn2;  // (2 W) w_n = W (2 w_n) exactly
  float den = r2 * r2;
  // no branch at zero distance: f = 0 there, and fma(0, dx, y) = y, since
  // dx is finite and y, a sum that starts at +0, is never -0
  float f = num / den;
  asm volatile("" : "+v"(f));  // formed on every lane: a select below, not a branch
  f = r2 > 0.0f ? f : 0.0f;
  y[0] = __builtin_fmaf(f, dx0, y[0]);
  y[1] = __builtin_fmaf(f, dx1, y[1]);
  y[2] = __builtin_fmaf(f, dx2, y[2]);
  y[3] = __builtin_fmaf(f, dx3, y[3]);
}

// Minimum over the 64 lanes (all active), by DPP row shifts and row
// broadcasts; lane 63 ends with the minimum of the wavefront.
// Lanes without a source (and rows the mask leaves out) take INT_MAX, the
// identity of min, so that each step folds into one v_min_i32 with DPP.
__device__ __forceinline__ int32_t wave_min(int32_t v) {
  constexpr int32_t I = 0x7fffffff;
  v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Repulsion by the stackless walk of Algorithm 3: a far node acts as one charge
// and the walk jumps to its sibling link; a near internal node is entered; a
// near leaf acts point by point.  One lane per point, points in tree order.
//
// Parts.  The walk of a point is summed in two levels of parts (the same
// order as the oracle): a root that is a leaf or far from the point is one
// part; otherwise each child c1 of the root is a part, added in child order;
// the part of a c1 that is a leaf or far from the point ("single") is its walk
// from zero, and the part of any other c1 is the sum, from zero and in child
// order, of the walks over the children c2 of c1, each from zero.  Block row
// blockIdx.y = i1 * spread + i2 handles child i1 of the root and, with
// spread = 16, only child i2 of c1 (each such walk is then stored and
// k_combine adds them up); with spread = 1 the wavefront walks every c2 of c1
// in turn and stores the part of c1.  Spreading gives small levels 16 times
// more wavefronts; both layouts give the same sums.
//
// The 64 lanes of a wavefront step through the nodes of their range in
// pre-order together: node t is read once for the wave, and a lane takes
// part only if its own walk reaches t (t >= its skip mark).  Every jump of a
// single walk moves forward in pre-order, so each lane performs exactly the
// interactions of its own walk, in the same order.  The wave moves to t + 1
// while some lane is still descending, else to the smallest skip mark.
// Nodes are staged through a per-wavefront LDS window of kWin consecutive
// nodes (the five 16-byte chunks of an 80-byte node stored chunk-major, so
// that every lane reads one node's chunk with one broadcast read), and the
// points of near leaves through a second window of kWin consecutive points:
// the walk meets leaves in tree order, so one refill serves several leaves.
constexpr int kWin = 32;
constexpr int kWT = 64;     // threads per block of the walk: one wavefront (measured best of 64-512)
constexpr int kCntSlots = 256;  // interaction counters of the walk (16 words apart)

template <bool kCount>  // kCount: count the interactions into nint
// 64 registers (eight wavefronts per SIMD instead of seven at the compiler's 72:
// the finest levels' walks fill the chip and gain from the extra wavefront)
__global__ __launch_bounds__(kWT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_walk(
    int32_t k, const int32_t* __restrict__ n_dev, const float4* __restrict__ P, const float* __restrict__ ws,
    const int32_t* __restrict__ p2, const TNode* __restrict__ nodes, const int32_t* __restrict__ cid,
    const int32_t* __restrict__ nch, int spread, float* __restrict__ part, unsigned long long* nint,
    const int32_t* __restrict__ plan, int32_t hblocks) {
  constexpr int NW = kWT / 64;
  __shared__ int4 win[NW][5][kWin];  // the five 16-byte chunks of kWin nodes
  __shared__ float4 lp[NW][kWin];
  __shared__ float lw[NW][kWin];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // The row and the points of this block, from the launch plan (walk_plan):
  // blocks below hblocks take heavy_pts(k) points of a row's node, the others
  // 64 points of a row outside its node.
  const int R = kParts * spread, so = spread > 1 ? 0 : 256;
  const int64_t gb = blockIdx.x;
  int32_t yrow;
  int64_t j;
  bool valid;
  if (gb < hblocks) {
    const int32_t* hp = plan + kPlH + (spread > 1 ? 0 : 257);
    if (gb >= hp[R]) return;  // the whole block: past the heavy wavefronts
    int lo = 0, hi = R;       // the launch rank r with hp[r] <= gb < hp[r + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (hp[mid] <= gb) lo = mid; else hi = mid;
    }
    yrow = plan[kPlP + so + lo];
    const int64_t nf = plan[kPlF + so + yrow], nc = plan[kPlC + so + yrow];
    const int hpts = heavy_pts(k);
    j = nf + (gb - hp[lo]) * hpts + lane;
    valid = lane < hpts && j < nf + nc;
  } else {
    const int64_t gx = ((int64_t)k + 63) / 64, bn = gb - hblocks;
    const int r = (int)(bn / gx);
    yrow = plan[kPlP + so + r];
    int64_t x = bn % gx + plan[kPlX + so + yrow];
    if (x >= gx) x -= gx;
    const int64_t nf = plan[kPlF + so + yrow], nc = plan[kPlC + so + yrow];
    j = x * 64 + lane;
    valid = j < k && !(j >= nf && j < nf + nc);
  }
  const int i1 = yrow / spread, i2s = yrow % spread;
  const int32_t n = *n_dev;
  const bool rleaf = (nodes[0].b.w >> 8) & 1;
  const int n1 = rleaf ? 1 : min(nch[0], kParts);
  if (i1 >= n1) return;  // the whole block
  const int32_t c1 = rleaf ? 0 : cid[i1];
  const int4 b1 = nodes[c1].b;
  const bool c1leaf = (b1.w >> 8) & 1;
  const int n2 = c1leaf ? 0 : min(nch[c1], kParts);
  if (i2s > 0 && i2s >= n2) return;  // the whole block
  // interactions of the wavefront (uniform: counted from lane masks)
  unsigned long long cnt = 0;
  float xn[4] = {0.f, 0.f, 0.f, 0.f};
  double qd[4] = {0.0, 0.0, 0.0, 0.0};  // doubled grid coordinates
  float wn = 0.0f;
  if (valid) {
    float4 pj = P[j];
    xn[0] = pj.x; xn[1] = pj.y; xn[2] = pj.z; xn[3] = pj.w;
    for (int d = 0; d < 4; ++d) qd[d] = (double)p2[(int64_t)d * k + j];
    wn = ws[j];
  }
  const double q2 = norm2_q(qd);
  const float wn2 = 2.0f * wn;
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const bool rootfar = valid && far_q(qd, q2, nodes[0].A, nodes[0].Tq);
  const bool single = valid && (rootfar || c1leaf || far_q(qd, q2, nodes[c1].A, nodes[c1].Tq));

  int32_t wb = -2 * kWin;  // node window: nodes [wb, wb + kWin)
  int32_t pb = -2 * kWin;  // point window: points [pb, pb + kWin) in tree order
  // refill: lane l loads chunks 2 (l & 1) and 2 (l & 1) + 1 of node wb + l / 2,
  // lanes below kWin chunk 4 of node wb + l
  const int po = lane >> 1, pc = (lane & 1) * 2;
  const int4* nodes4 = reinterpret_cast<const int4*>(nodes);
  // the union walk of the lanes with skip marks < t1 over [.., t1), into y
  auto run = [&](int32_t skip, int32_t t1, float* y) {
    int32_t t = __builtin_amdgcn_readfirstlane(wave_min(skip));
    while (t < t1) {
      if (t < wb || t >= wb + kWin) {
        wb = t;
        // the three loads issued together (lanes past the tree's end, or
        // past the window for chunk 4, read node t again and write nothing)
        const bool oka = t + po < n, okb = lane < kWin && t + lane < n;
        const int64_t ia = oka ? t + po : t, ib = okb ? t + lane : t;
        const int4 c0 = nodes4[5 * ia + pc], c1 = nodes4[5 * ia + pc + 1], c4 = nodes4[5 * ib + 4];
        if (oka) {
          win[wv][pc][po] = c0;
          win[wv][pc + 1][po] = c1;
        }
        if (okb) win[wv][4][lane] = c4;
        wave_sync();
      }
      const int o = t - wb;
      const int4 a01 = win[wv][0][o];
      const int4 a23 = win[wv][1][o];
      const int4 b = win[wv][2][o];
      const int4 xi = win[wv][3][o];
      const int4 tw = win[wv][4][o];
      // all five reads in flight together, one wait for them
      asm volatile("" ::"v"(a01.x), "v"(a01.y), "v"(a01.z), "v"(a01.w), "v"(a23.x), "v"(a23.y), "v"(a23.z),
                   "v"(a23.w), "v"(xi.x), "v"(xi.y), "v"(xi.z), "v"(xi.w), "v"(tw.x), "v"(tw.y), "v"(tw.z));
      const double A[4] = {__hiloint2double(a01.y, a01.x), __hiloint2double(a01.w, a01.z),
                           __hiloint2double(a23.y, a23.x), __hiloint2double(a23.w, a23.z)};
      // the link fields are the same on every lane: the flags (and, at a
      // leaf, the point range) in scalar registers, so that the leaf loops
      // below are scalar loops
      const int32_t bnext = b.x;
      const int32_t bflags = __builtin_amdgcn_readfirstlane(b.w);
      const bool act = skip <= t;
      const bool far = act & far_q(qd, q2, A, __hiloint2double(tw.y, tw.x));
      if (far) {
        interact(y, xn, wn2, __int_as_float(xi.x), __int_as_float(xi.y), __int_as_float(xi.z), __int_as_float(xi.w),
                 __int_as_float(tw.z));
        skip = bnext;
      }
      if (kCount) cnt += (unsigned long long)__popcll(__ballot(far));
      const bool near = act && !far;
      if ((bflags >> 8) & 1) {
        if (__any(near)) {
          const int32_t bfirst = __builtin_amdgcn_readfirstlane(b.y);
          const int32_t f1 = bfirst + __builtin_amdgcn_readfirstlane(b.z);
          for (int32_t base = bfirst; base < f1; base += kWin) {
            const int32_t e = f1 - base < kWin ? f1 : base + kWin;
            if (base < pb || e > pb + kWin) {
              // slide the point window to start at this leaf
              wave_sync();
              pb = base;
              const int32_t ii = base + lane;
              if (lane < kWin && ii < k) {
                lp[wv][lane] = P[ii];
                lw[wv][lane] = ws[ii];
              }
              wave_sync();
            }
            const int32_t m = e - base, o2 = base - pb;
            if (near) {
              // the point itself is not skipped by index: its distance is
              // zero, and interact() leaves y unchanged at zero distance
              // two points per step, both read before the first interaction
              // (the interactions stay in point order)
              int32_t i = 0;
              for (; i + 1 < m; i += 2) {
                const float4 pa = lp[wv][o2 + i], pb = lp[wv][o2 + i + 1];
                const float wa = lw[wv][o2 + i], wb = lw[wv][o2 + i + 1];
                interact(y, xn, wn2, pa.x, pa.y, pa.z, pa.w, wa);
                interact(y, xn, wn2, pb.x, pb.y, pb.z, pb.w, wb);
              }
              if (i < m) {
                const float4 pi = lp[wv][o2 + i];
                interact(y, xn, wn2, pi.x, pi.y, pi.z, pi.w, lw[wv][o2 + i]);
              }
            }
            if (kCount)
              cnt += (unsigned long long)m * __popcll(__ballot(near)) -
                   __popcll(__ballot(near && j >= base && j < base + m));
          }
        }
        if (near) skip = bnext;
      } else if (near) {
        skip = t + 1;
      }
      int32_t nt = t + 1;
      if (!__any(skip <= nt)) {
        nt = wave_min(skip);
        if (nt <= t) nt = t + 1;  // every walk mark lies beyond t; keeps the loop advancing
      }
      t = __builtin_amdgcn_readfirstlane(nt);
    }
  };

  float acc1[4] = {0.f, 0.f, 0.f, 0.f};
  if (i2s == 0) {
    // single parts: the root's interaction (part 0 only), or the walk of c1
    if (rootfar && i1 == 0) {
      const float4 X = nodes[0].X;
      interact(acc1, xn, wn2, X.x, X.y, X.z, X.w, nodes[0].W);
    }
    if (kCount && i1 == 0) cnt += (unsigned long long)__popcll(__ballot(rootfar));
    run(single && !rootfar ? c1 : 0x7fffffff, c1 + 1, acc1);
  }
  // children of c1 walked here (none when c1 is a leaf: n2 = 0)
  const int i2b = spread > 1 ? i2s : 0, i2e = spread > 1 ? (i2s < n2 ? i2s + 1 : i2s) : n2;
  float acc2[4] = {0.f, 0.f, 0.f, 0.f};
  for (int i2 = i2b; i2 < i2e; ++i2) {
    const int32_t c2 = cid[16 * (int64_t)c1 + i2];
    for (int d = 0; d < 4; ++d) acc2[d] = 0.0f;
    run(valid && !single ? c2 : 0x7fffffff, nodes[c2].b.x, acc2);
    if (spread == 1 && !single)
      for (int d = 0; d < 4; ++d) acc1[d] = acc1[d] + acc2[d];
  }
  if (valid) {
    if (spread == 1) {
      for (int d = 0; d < 4; ++d) part[((int64_t)i1 * 4 + d) * k + j] = acc1[d];
    } else if (single) {
      if (i2s == 0)
        for (int d = 0; d < 4; ++d) part[(((int64_t)i1 * kParts) * 4 + d) * k + j] = acc1[d];
    } else {
      for (int d = 0; d < 4; ++d) part[(((int64_t)i1 * kParts + i2s) * 4 + d) * k + j] = acc2[d];
    }
  }
  if (kCount) {
    // kCntSlots counters, 128 bytes apart, so that the wavefronts' atomics
    // (finishing at about the same time) do not queue on one address
    const unsigned slot = ((unsigned)blockIdx.x * (kWT / 64) + wv) % kCntSlots;
    if (lane == 0 && cnt) atomicAdd(&nint[16 * slot], cnt);
  }
}

// *out = sum of the walk's interaction counters, which are cleared for the
// next walk (one block of kCntSlots threads).
__global__ __launch_bounds__(kCntSlots) void k_sum_slots(unsigned long long* slots, unsigned long long* out) {
  __shared__ unsigned long long sm[kCntSlots];
  const int t = threadIdx.x;
  sm[t] = slots[16 * t];
  slots[16 * t] = 0ull;
  __syncthreads();
  for (int off = kCntSlots / 2; off > 0; off >>= 1) {
    if (t < off) sm[t] += sm[t + off];
    __syncthreads();
  }
  if (t == 0) *out = sm[0];
}

// y_v = attraction + the parts of the walk in order (point j in tree order is
// vertex order[j]).  xmove == NULL: y receives the gradient; else the descent
// step of Algorithm 3 is applied to xmove: x_v <- x_v - (alpha / |y_v|) y_v.
// A block takes 64 points; wavefront i1 forms part i1 of each of them (its
// loads coalesced over the points, the sub-parts of a spread part loaded
// together and summed in child order), and wavefront 0 adds the parts to the
// attraction in part order.
constexpr int kCombT = 64 * kParts;
__global__ __launch_bounds__(kCombT) void k_combine(int32_t k, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ p2, const TNode* __restrict__ nodes,
                                                    const int32_t* __restrict__ cid, const int32_t* __restrict__ nch,
                                                    int spread, const float* __restrict__ part, float4* y,
                                                    float4* xmove, double alpha, const double* __restrict__ alpha_d,
                                                    int32_t it, double decay, uint32_t* box_next) {
  // the empty box for the next step's box of the moved points (every reader
  // of this step's box ran before this launch)
  if (box_next && blockIdx.x == 0 && threadIdx.x < 8) box_next[threadIdx.x] = threadIdx.x < 4 ? 0xffffffffu : 0u;
  __shared__ float4 sh[kParts][64];
  const int i1 = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  const bool valid = j < k;
  const bool rleaf = (nodes[0].b.w >> 8) & 1;
  const int n1 = rleaf ? 1 : min(nch[0], kParts);
  double qd[4] = {0.0, 0.0, 0.0, 0.0};
  if (valid)
    for (int d = 0; d < 4; ++d) qd[d] = (double)p2[(int64_t)d * k + j];
  const double q2 = norm2_q(qd);
  // a root that is a leaf or far from the point: one part, in slot 0
  const bool one = rleaf || (valid && far_q(qd, q2, nodes[0].A, nodes[0].Tq));
  const int np = one ? 1 : n1;
  float a1[4] = {0.f, 0.f, 0.f, 0.f};
  if (valid && i1 < np) {
    if (one || spread == 1) {
      const int64_t slot = one ? 0 : (spread == 1 ? i1 : (int64_t)i1 * kParts);
      for (int d = 0; d < 4; ++d) a1[d] = part[(slot * 4 + d) * k + j];
    } else {
      const int32_t c1 = cid[i1];
      const bool c1leaf = (nodes[c1].b.w >> 8) & 1;
      if (c1leaf || far_q(qd, q2, nodes[c1].A, nodes[c1].Tq)) {
        for (int d = 0; d < 4; ++d) a1[d] = part[(((int64_t)i1 * kParts) * 4 + d) * k + j];
      } else {
        const int n2 = min(nch[c1], kParts);
        float v[kParts][4];
#pragma unroll
        for (int i2 = 0; i2 < kParts; ++i2)
          if (i2 < n2)
            for (int d = 0; d < 4; ++d) v[i2][d] = part[(((int64_t)i1 * kParts + i2) * 4 + d) * k + j];
#pragma unroll
        for (int i2 = 0; i2 < kParts; ++i2)
          if (i2 < n2)
            for (int d = 0; d < 4; ++d) a1[d] = a1[d] + v[i2][d];
      }
    }
  }
  // the point's own records, loaded by wavefront 0 before the barrier so
  // that their latency overlaps the other wavefronts' part loads
  int32_t v = 0;
  float4 y0 = make_float4(0.f, 0.f, 0.f, 0.f), xo = y0;
  if (i1 == 0 && valid) {
    v = order[j];
    y0 = y[v];
    if (xmove) xo = xmove[v];
  }
  sh[i1][lane] = make_float4(a1[0], a1[1], a1[2], a1[3]);
  __syncthreads();
  if (i1 != 0 || !valid) return;
  float yv[4] = {y0.x, y0.y, y0.z, y0.w};
  for (int i = 0; i < np; ++i) {
    const float4 a = sh[i][lane];
    yv[0] = yv[0] + a.x;
    yv[1] = yv[1] + a.y;
    yv[2] = yv[2] + a.z;
    yv[3] = yv[3] + a.w;
  }
  if (!xmove) {
    y[v] = make_float4(yv[0], yv[1], yv[2], yv[3]);
    return;
  }
  float n2s = yv[0] * yv[0];
  n2s = n2s + yv[1] * yv[1];
  n2s = n2s + yv[2] * yv[2];
  n2s = n2s + yv[3] * yv[3];
  if (!(n2s > 0.0f)) return;
  double a = alpha;
  if (alpha_d) {
    // the step length of step it of the level: alpha_0, then times decay
    // after every step, as the host carries it
    a = *alpha_d;
    for (int32_t i = 0; i < it; ++i) a = a * decay;
  }
  float f = (float)(a / sqrt((double)n2s));
  const float xv[4] = {xo.x, xo.y, xo.z, xo.w};
  float xn[4];
  for (int d = 0; d < 4; ++d) {
    float td = f * yv[d];
    xn[d] = xv[d] - td;
  }
  xmove[v] = make_float4(xn[0], xn[1], xn[2], xn[3]);
}

struct GradWork {
  Buf<float4> z;  // net centres, one record per net
  Buf<uint32_t> box;
  Buf<float> part;  // partial repulsions, tree order: [16][4][k], or [16][16][4][k] when spread
  Tree T;
  Buf<double> alpha;  // alpha_0 of the level (device step length)
  bool box_reset = false;  // box holds the empty box (set by the last combine)
};

// Attraction into y, net centres, box of x (gw.box) and the tree of x.
static void gradient_prepare(Ctx& C, const Level& L, const float4* x, double th2, int32_t cap, float4* y, GradWork& gw,
                             hipStream_t s) {
  if (!gw.box.p) gw.box = Buf<uint32_t>(C.pool, 8);
  // else the one-block tree build forms it
  if (L.k > kSmallK) box_of(x, L.k, gw.box.p, s, gw.box_reset);
  gw.box_reset = false;
  gw.z = Buf<float4>(C.pool, (size_t)(L.l > 0 ? L.l : 1));
  if (L.l > 0) VMO_LAUNCH(k_centres, gsz(L.l), kLT, 0, s, L.ptr.p, L.pins.p, L.l, x, gw.z.p);
  const AttractJob aj{L.dptr.p, L.dpins.p, L.k, L.c.p, x, gw.z.p, y};
  if (L.k <= kSmallK) {
    // the one-block tree build runs the attraction in its other blocks
    build_tree(C, gw.T, x, L.w.p, L.k, cap, gw.box.p, th2, s, true, &aj);
    return;
  }
  if (L.k <= 16384)
    VMO_LAUNCH(k_attract_wave, nblocks(L.k, 4), 256, 0, s, aj);
  else {
    AttractJob ah = aj;
    ah.heavy = L.heavy.p;
    const int64_t hb = heavy_blocks(L);
    VMO_LAUNCH(k_attract, (unsigned)(hb + gsz(L.k)), kLT, 0, s, ah, (int32_t)hb);
  }
  build_tree(C, gw.T, x, L.w.p, L.k, cap, gw.box.p, th2, s);
}

// Repulsion by the tree walk, added to the attraction in y.  xmove == NULL:
// y receives the gradient of eq. (6); else the descent step of length alpha
// is applied to xmove (the layout being descended) and y is left as is.
// alpha_d (device, may be NULL): alpha_0 of the level, the step length of
// step it being alpha_0 times decay it times; else alpha is the step length.
static void gradient_walk(Ctx& C, const Level& L, float4* y, float4* xmove, double alpha, GradWork& gw,
                          unsigned long long* nint, hipStream_t s, const double* alpha_d = nullptr,
                          int32_t it = 0, double decay = 1.0) {
  // Levels of up to kSpreadMax points spread each part of the walk over the
  // children of its cell: 16 times the wavefronts, and up to 16 times the
  // parts to write and add up.  Above it the unspread walk already has more
  // than six wavefronts per resident slot of the chip (256 CUs x 32), and
  // spreading only adds traffic.
  constexpr int32_t kSpreadMax = 300000;
  if (L.k <= 0) return;
  const int spread = L.k <= kSpreadMax ? kParts : 1;
  const size_t np = (size_t)kParts * spread * 4 * L.k;
  // during a layout: the most any of its levels needs, so that every level
  // takes the same block
  const int64_t km = C.layout_kmax;
  const size_t np_all = km > 0 ? std::max((size_t)kParts * 4 * km, (size_t)kParts * kParts * 4 *
                                                                        std::min<int64_t>(km, kSpreadMax))
                               : 0;
  if (gw.part.n < np) gw.part = Buf<float>(C.pool, std::max(np, np_all));
  unsigned long long* pc = nullptr;
  int ph = prof_begin(C, "walk", 0.0, s, nint ? nullptr : &pc);
  unsigned long long* target = nint ? nint : pc;
  if (target && !C.wslots) {
    // the counters are zero before every counting walk: cleared here once,
    // then by k_sum_slots after each reading
    VMO_HIP(hipMalloc(&C.wslots, sizeof(unsigned long long) * 16 * kCntSlots));
    VMO_HIP(hipMemsetAsync(C.wslots, 0, sizeof(unsigned long long) * 16 * kCntSlots, s));
    if (ph >= 0) prof_restart(C, ph, s);
  }
  // heavy wavefronts: at most one per heavy_pts(k) points plus one per row
  // (the rows' nodes are disjoint), then 64-point blocks for every row
  const int64_t rows = (int64_t)kParts * spread;
  const int64_t hblocks = ((int64_t)L.k + heavy_pts(L.k) - 1) / heavy_pts(L.k) + rows;
  const unsigned wgrid = (unsigned)(hblocks + nblocks(L.k, kWT) * rows);
  if (target)
    VMO_LAUNCH((k_walk<true>), wgrid, kWT, 0, s, L.k, gw.T.nn.p + L.k, gw.T.P.p, gw.T.ws.p, gw.T.p2.p, gw.T.nodes.p,
               gw.T.cid.p, gw.T.nch.p, spread, gw.part.p, C.wslots, gw.T.plan.p, (int32_t)hblocks);
  else
    VMO_LAUNCH((k_walk<false>), wgrid, kWT, 0, s, L.k, gw.T.nn.p + L.k, gw.T.P.p, gw.T.ws.p, gw.T.p2.p, gw.T.nodes.p,
               gw.T.cid.p, gw.T.nch.p, spread, gw.part.p, nullptr, gw.T.plan.p, (int32_t)hblocks);
  prof_end(C, ph, s);
  if (target) VMO_LAUNCH(k_sum_slots, 1, kCntSlots, 0, s, C.wslots, target);
  VMO_LAUNCH(k_combine, nblocks(L.k, 64), kCombT, 0, s, L.k, gw.T.order.p, gw.T.p2.p, gw.T.nodes.p, gw.T.cid.p,
             gw.T.nch.p, spread, gw.part.p, y, xmove, alpha, alpha_d, it, decay, xmove ? gw.box.p : nullptr);
  gw.box_reset = xmove != nullptr && gw.box.p != nullptr;
}

// alpha_0 = step0 * V^(1/4) from the box (V = 0: its largest side), as the
// host forms it (one thread).
__global__ void k_alpha0(const uint32_t* box, double step0, double* alpha) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double V = 1.0, ext = 0.0;
  for (int d = 0; d < 4; ++d) {
    const double e = (double)fkey_inv(box[4 + d]) - (double)fkey_inv(box[d]);
    V = V * e;
    if (e > ext) ext = e;
  }
  const double side = V > 0.0 ? sqrt(sqrt(V)) : ext;
  *alpha = step0 * side;
}

// One descent step (Algorithm 3).  alpha: step length (host); at it == 0 it
// is set from the box, alpha = step0 * V^(1/4) (V = 0: largest side), then
// multiplied by decay after every step.  alpha == NULL: the same on the
// device (no read-back): alpha_0 formed at it == 0, the combine applying the
// decays.
static void descent_step(Ctx& C, const Level& L, float4* x, const vmo_layout_params* p, int32_t it, double* alpha,
                         float4* y, GradWork& gw, hipStream_t s) {
  double th2 = (double)p->theta * (double)p->theta;
  gradient_prepare(C, L, x, th2, p->leaf_cap, y, gw, s);
  if (!alpha) {
    if (!gw.alpha.p) gw.alpha = Buf<double>(C.pool, 1);
    if (it == 0) VMO_LAUNCH(k_alpha0, 1, 64, 0, s, gw.box.p, (double)p->step0_frac, gw.alpha.p);
    gradient_walk(C, L, y, x, 0.0, gw, nullptr, s, gw.alpha.p, it, (double)p->decay);
    return;
  }
  if (it == 0) {
    HostBox hb = read_box(gw.box.p, s);
    double V = 1.0, ext = 0.0;
    for (int d = 0; d < 4; ++d) {
      double e = (double)hb.hi[d] - (double)hb.lo[d];
      V = V * e;
      if (e > ext) ext = e;
    }
    double side = V > 0.0 ? sqrt(sqrt(V)) : ext;
    *alpha = (double)p->step0_frac * side;
  } else {
    *alpha = *alpha * (double)p->decay;
  }
  gradient_walk(C, L, y, x, *alpha, gw, nullptr, s);
}

// ================================================================ coarsen ===
struct Prio {
  double om;
  uint64_t hs;
  int32_t a, b;
};
__device__ __forceinline__ bool prio_gt(const Prio& x, const Prio& y) {
  if (x.om != y.om) return x.om > y.om;
  if (x.hs != y.hs) return x.hs > y.hs;
  if (x.a != y.a) return x.a < y.a;
  return x.b < y.b;
}

// Best unmatched candidate partner of every unmatched vertex: the pair of
// highest priority (cost/(|e|-1) over a shared net of 2..mm pins, then the
// keyed hash, then the smaller ids).  The priorities of distinct pairs differ,
// so the best partner is unique whatever order the candidates are met in.
// prev: the match count of the previous round of the group (NULL for its
// first round); after a round that matched nothing the rounds change nothing,
// so both kernels return at once.
// A vertex whose scan meets more than kMatchLight candidate pins, or that
// lies in more than kHeavyDeg nets, is listed once per coarsening step; its
// nets are scanned in chunks of kMatchChunk, one wavefront per chunk; a vertex
// of several chunks keeps each chunk's best candidate, and the wavefront that
// finishes the vertex's last chunk takes the best of them (counted by an
// agent-scope acquire-release add, so that the chunks' records are visible to
// it).  Every other vertex is scanned by one thread.
constexpr int32_t kMatchChunk = 256;
constexpr int32_t kMatchLight = 512;
struct ChunkBest {
  double om;
  uint64_t hs;
  int32_t v, pad;
};
struct MatchJob {
  const int64_t* ptr;
  const int32_t* pins;
  const int64_t* dptr;
  const int32_t* dpins;
  const float* c;
  int32_t k, mm;
  const int32_t* mate;
  uint64_t seed, mkey;
  const int32_t* heavy;   // [0]: count, then the listed vertices (in no particular order)
  const uint8_t* listed;  // [k]: 1 for the listed vertices
  const int32_t* cstart;  // [k + 1]: first chunk of each listed vertex (exclusive scan)
  ChunkBest* cres;        // per chunk: its best candidate
  int32_t* hdone;         // per listed vertex: chunks finished in this launch (left at zero)
};
// candidates of u over its nets tb, tb + step, ... below te into (bp, bv)
__device__ __forceinline__ void match_scan(const MatchJob& mj, int32_t u, int64_t tb, int64_t te, int64_t step,
                                           Prio& bp, int32_t& bv) {
  for (int64_t t = tb; t < te; t += step) {
    int32_t e = mj.dpins[t];
    int64_t b = mj.ptr[e], n = mj.ptr[e + 1] - b;
    if (n < 2 || n > mj.mm) continue;
    double om = (double)(mj.c ? mj.c[e] : 1.0f) / (double)(n - 1);
    for (int64_t p = b; p < b + n; ++p) {
      int32_t v = mj.pins[p];
      if (v == u || mj.mate[v] >= 0) continue;
      Prio q;
      q.om = om;
      q.a = u < v ? u : v;
      q.b = u < v ? v : u;
      q.hs = rng3(mj.seed, mj.mkey, (uint64_t)q.a, (uint64_t)q.b);
      if (bv < 0 || prio_gt(q, bp)) { bp = q; bv = v; }
    }
  }
}
// (bp, bv) <- the better of (bp, bv) and candidate (om, hs, v) of u
__device__ __forceinline__ void match_keep(int32_t u, double om, uint64_t hs, int32_t v, Prio& bp, int32_t& bv) {
  Prio q;
  q.om = om;
  q.hs = hs;
  q.a = u < v ? u : v;
  q.b = u < v ? v : u;
  if (v >= 0 && (bv < 0 || prio_gt(q, bp))) { bp = q; bv = v; }
}
// One thread per vertex; the first hb blocks give the chunks of the heavy
// vertices a wavefront each, whose lanes take every 64th net of the chunk and
// then keep the best of the lanes' candidates.
__global__ __launch_bounds__(kLT) void k_match_best(MatchJob mj, int32_t hb, const int32_t* prev, int32_t* best) {
  if (prev && *prev == 0) return;
  if ((int32_t)blockIdx.x < hb) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)hb * (kLT / 64);
    const int32_t nh = mj.heavy[0], nc = mj.cstart[nh];
    for (int64_t c = (int64_t)blockIdx.x * (kLT / 64) + (threadIdx.x >> 6); c < nc; c += nw) {
      // the listed vertex of chunk c: the last i with cstart[i] <= c
      int32_t lo = 0, hi = nh;
      while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (mj.cstart[mid] <= c) lo = mid; else hi = mid;
      }
      const int32_t i = lo, u = mj.heavy[1 + i];
      const int32_t c0 = mj.cstart[i], nch = mj.cstart[i + 1] - c0;
      if (mj.mate[u] >= 0) {
        if (lane == 0 && c == c0) best[u] = -1;
        continue;
      }
      const int64_t tb = mj.dptr[u] + (int64_t)(c - c0) * kMatchChunk;
      const int64_t te = min(mj.dptr[u + 1], tb + kMatchChunk);
      Prio bp;
      bp.om = -1.0; bp.hs = 0; bp.a = 0x7fffffff; bp.b = 0x7fffffff;
      int32_t bv = -1;
      match_scan(mj, u, tb + lane, te, 64, bp, bv);
      for (int off = 32; off > 0; off >>= 1) {
        const double om = __shfl_xor(bp.om, off);
        const uint64_t hs = __shfl_xor(bp.hs, off);
        const int32_t v = __shfl_xor(bv, off);
        match_keep(u, om, hs, v, bp, bv);
      }
      if (lane != 0) continue;
      if (nch == 1) {
        best[u] = bv;
        continue;
      }
      ChunkBest r;
      r.om = bp.om; r.hs = bp.hs; r.v = bv; r.pad = 0;
      mj.cres[c] = r;
      const int32_t done =
          __hip_atomic_fetch_add(&mj.hdone[i], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (done != nch - 1) continue;
      // the last chunk of u: every chunk's record is visible here
      Prio b2;
      b2.om = -1.0; b2.hs = 0; b2.a = 0x7fffffff; b2.b = 0x7fffffff;
      int32_t v2 = -1;
      for (int32_t q = 0; q < nch; ++q) {
        const ChunkBest cb = mj.cres[c0 + q];
        match_keep(u, cb.om, cb.hs, cb.v, b2, v2);
      }
      best[u] = v2;
      mj.hdone[i] = 0;  // every chunk of u has counted: zero again for the next launch
    }
    return;
  }
  const int64_t stride = (int64_t)(gridDim.x - hb) * blockDim.x;
  for (int64_t u64 = (int64_t)(blockIdx.x - hb) * blockDim.x + threadIdx.x; u64 < mj.k; u64 += stride) {
    int32_t u = (int32_t)u64;
    if (mj.listed[u]) continue;
    if (mj.mate[u] >= 0) { best[u] = -1; continue; }
    Prio bp;
    bp.om = -1.0; bp.hs = 0; bp.a = 0x7fffffff; bp.b = 0x7fffffff;
    int32_t bv = -1;
    match_scan(mj, u, mj.dptr[u], mj.dptr[u + 1], 1, bp, bv);
    best[u] = bv;
  }
}
// The vertices the matching scans by chunks: more than kHeavyDeg nets, or
// more than kMatchLight pins over their nets of 2..mm pins.
__global__ void k_match_list(const int64_t* ptr, const int64_t* dptr, const int32_t* dpins, int32_t k, int32_t mm,
                             int32_t* list, uint8_t* listed) {
  GRID_STRIDE(u, k) {
    const int64_t b = dptr[u], e = dptr[u + 1];
    bool heavy = e - b > kHeavyDeg;
    if (!heavy) {
      int64_t w = 0;
      for (int64_t t = b; t < e; ++t) {
        const int32_t n = dpins[t];
        const int64_t m = ptr[n + 1] - ptr[n];
        if (m >= 2 && m <= mm) w += m;
      }
      heavy = w > kMatchLight;
    }
    listed[u] = heavy ? 1 : 0;
    if (heavy) list[1 + atomicAdd(list, 1)] = (int32_t)u;
  }
}
// chunks of each listed vertex (the entries past the list's count get none)
__global__ void k_match_chunks(const int32_t* heavy, const int64_t* dptr, int64_t cap, int32_t* cnt) {
  const int32_t nh = heavy[0];
  GRID_STRIDE(i, cap) {
    int32_t n = 0;
    if (i < nh) {
      const int32_t u = heavy[1 + i];
      n = (int32_t)((dptr[u + 1] - dptr[u] + kMatchChunk - 1) / kMatchChunk);
    }
    cnt[i] = n;
  }
}
__global__ void k_match_pair(const int32_t* best, int32_t k, const int32_t* prev, int32_t* mate, int32_t* changed) {
  if (prev && *prev == 0) return;
  GRID_STRIDE(u64, k) {
    int32_t u = (int32_t)u64;
    int32_t v = best[u];
    if (mate[u] < 0 && v >= 0 && best[v] == u) {
      mate[u] = v;
      atomicAdd(changed, 1);
    }
  }
}
// Group root: the smaller vertex of a matched pair; an unmatched vertex with
// exactly one candidate neighbour joins that neighbour's group.
__global__ void k_group_root(const int64_t* ptr, const int32_t* pins, const int64_t* dptr, const int32_t* dpins,
                             int32_t k, int32_t mm, const int32_t* mate, int32_t* root, int32_t* gmin) {
  GRID_STRIDE(u64, k) {
    int32_t u = (int32_t)u64;
    int32_t m = mate[u];
    int32_t r = u;
    if (m >= 0) r = u < m ? u : m;
    else {
      int32_t v0 = -1;
      bool multi = false;
      for (int64_t t = dptr[u]; t < dptr[u + 1] && !multi; ++t) {
        int32_t e = dpins[t];
        int64_t b = ptr[e], n = ptr[e + 1] - b;
        if (n < 2 || n > mm) continue;
        for (int64_t p = b; p < b + n; ++p) {
          int32_t v = pins[p];
          if (v == u) continue;
          if (v0 < 0) v0 = v;
          else if (v != v0) { multi = true; break; }
        }
      }
      if (v0 >= 0 && !multi) {
        int32_t mv = mate[v0];
        r = mv >= 0 ? (v0 < mv ? v0 : mv) : v0;
      }
    }
    root[u] = r;
  }
}
__global__ void k_group_min(const int32_t* root, int32_t k, int32_t* gmin) {
  GRID_STRIDE(u, k) atomicMin(&gmin[root[u]], (int32_t)u);
}
__global__ void k_group_flag(const int32_t* root, const int32_t* gmin, int32_t k, int32_t* flag) {
  GRID_STRIDE(u, k) flag[u] = gmin[root[u]] == (int32_t)u ? 1 : 0;
}
__global__ void k_group_pi(const int32_t* root, const int32_t* gmin, const int32_t* rank, int32_t k, int32_t* pi,
                           uint32_t* key) {
  GRID_STRIDE(u, k) {
    int32_t g = rank[gmin[root[u]]];
    pi[u] = g;
    key[u] = (uint32_t)g;
  }
}
__global__ void k_count_i32(const int32_t* idx, int64_t n, int64_t* cnt) {
  GRID_STRIDE(i, n) atomicAdd((unsigned long long*)&cnt[idx[i]], 1ull);
}
// Coarse weight = member weights summed in ascending member id.
__global__ void k_coarse_w(const int64_t* gstart, const int32_t* members, const float* w, const int32_t* kc_dev,
                           float* cw) {
  const int32_t kc = *kc_dev;
  GRID_STRIDE(g, kc) {
    float a = 0.0f;
    for (int64_t t = gstart[g]; t < gstart[g + 1]; ++t) a = a + (w ? w[members[t]] : 1.0f);
    cw[g] = a;
  }
}
// Net images: key (net, coarse pin) per pin.
__global__ void k_img_keys(const int64_t* ptr, const int32_t* pins, int32_t l, const int32_t* pi, uint64_t* key) {
  GRID_STRIDE(e, l) {
    for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) key[p] = ((uint64_t)e << 32) | (uint32_t)pi[pins[p]];
  }
}
__global__ void k_img_uniq(const uint64_t* key, int64_t np, int32_t* ufl, int64_t* ilen) {
  GRID_STRIDE(p, np) {
    bool u = p == 0 || key[p] != key[p - 1];
    ufl[p] = u ? 1 : 0;
    if (u) atomicAdd((unsigned long long*)&ilen[key[p] >> 32], 1ull);
  }
}
__global__ void k_img_keep(const int64_t* ilen, int32_t l, int32_t* kf) {
  GRID_STRIDE(e, l) kf[e] = ilen[e] >= 2 ? 1 : 0;
}
__global__ void k_img_len(const int64_t* ilen, const int32_t* kf, const int32_t* kidx, int32_t l, int64_t* klen) {
  GRID_STRIDE(e, l) if (kf[e]) klen[kidx[e]] = ilen[e];
}
__global__ void k_img_pins(const uint64_t* key, const int32_t* ufl, const int32_t* uscan, const int64_t* ptr,
                           const int32_t* kf, const int32_t* kidx, const int64_t* iptr, int64_t np, int32_t* ipins) {
  GRID_STRIDE(p, np) {
    if (!ufl[p]) continue;
    int32_t e = (int32_t)(key[p] >> 32);
    if (!kf[e]) continue;
    int64_t r = uscan[p] - uscan[ptr[e]];
    ipins[iptr[kidx[e]] + r] = (int32_t)(key[p] & 0xffffffffu);
  }
}
// (entries nk..cap-1 get the largest key, which a stable sort leaves after
// every image)
__global__ void k_img_hash(const int64_t* iptr, const int32_t* ipins, const int32_t* nk_dev, int32_t cap, uint64_t* hs,
                           int32_t* val) {
  const int32_t nk = *nk_dev;
  GRID_STRIDE(i, cap) {
    if (i >= nk) {
      hs[i] = ~0ull;
      val[i] = (int32_t)i;
      continue;
    }
    uint64_t h = 0x5851F42D4C957F2DULL;
    for (int64_t p = iptr[i]; p < iptr[i + 1]; ++p) h = sm_mix(h + kGamma * ((uint64_t)(uint32_t)ipins[p] + 1));
    hs[i] = sm_mix(h + (uint64_t)(iptr[i + 1] - iptr[i]));
    val[i] = (int32_t)i;
  }
}
__device__ bool img_equal(const int64_t* iptr, const int32_t* ipins, int32_t a, int32_t b) {
  int64_t la = iptr[a + 1] - iptr[a], lb = iptr[b + 1] - iptr[b];
  if (la != lb) return false;
  for (int64_t t = 0; t < la; ++t)
    if (ipins[iptr[a] + t] != ipins[iptr[b] + t]) return false;
  return true;
}
// Representative of each kept net: the first net (in net order) of its run of
// equal hashes with the same image.
__global__ void k_img_rep(const uint64_t* hs, const int32_t* val, const int64_t* iptr, const int32_t* ipins,
                          const int32_t* nk_dev, int32_t* repflag, int32_t* reppos) {
  const int32_t nk = *nk_dev;
  GRID_STRIDE(i, nk) {
    int32_t me = val[i];
    int64_t r = i;
    for (int64_t j = i - 1; j >= 0 && hs[j] == hs[i]; --j)
      if (img_equal(iptr, ipins, val[j], me)) r = j;
    reppos[i] = (int32_t)r;
    repflag[me] = r == i ? 1 : 0;
  }
}
// Merged cost (members in ascending net order) and length of each coarse net.
__global__ void k_img_cost(const uint64_t* hs, const int32_t* val, const int32_t* reppos, const int32_t* kept_net,
                           const float* c, const int64_t* iptr, const int32_t* cidx, const int32_t* nk_dev, float* cc,
                           int64_t* clen) {
  const int32_t nk = *nk_dev;
  GRID_STRIDE(i, nk) {
    if (reppos[i] != i) continue;
    int32_t me = val[i];
    float a = c ? c[kept_net[me]] : 1.0f;
    for (int64_t j = i + 1; j < nk && hs[j] == hs[i]; ++j)
      if (reppos[j] == i) a = a + (c ? c[kept_net[val[j]]] : 1.0f);
    cc[cidx[me]] = a;
    clen[cidx[me]] = iptr[me + 1] - iptr[me];
  }
}
__global__ void k_kept_net(const int32_t* kf, const int32_t* kidx, int32_t l, int32_t* kept_net) {
  GRID_STRIDE(e, l) if (kf[e]) kept_net[kidx[e]] = (int32_t)e;
}
__global__ void k_coarse_pins(const int32_t* repflag, const int32_t* cidx, const int64_t* iptr, const int32_t* ipins,
                              const int64_t* cptr, const int32_t* nk_dev, int32_t* cpins) {
  const int32_t nk = *nk_dev;
  GRID_STRIDE(i, nk) {
    if (!repflag[i]) continue;
    int64_t o = cptr[cidx[i]];
    for (int64_t p = iptr[i]; p < iptr[i + 1]; ++p) cpins[o + (p - iptr[i])] = ipins[p];
  }
}

// The sizes of a coarse level, read back once at its end.
__global__ void k_coarse_sizes(const int32_t* kc, const int32_t* lc, const int64_t* cnp, int64_t* out) {
  out[0] = *kc;
  out[1] = lc ? *lc : 0;
  out[2] = cnp ? *cnp : 0;
}

// One coarsening step of level F into C (pi written to F.pi).  The counts of
// the coarse level (vertices, kept nets, image pins, coarse nets and pins)
// stay on the device until the end: buffers take their upper bounds (the fine
// level's sizes) and the kernels read the counts from device memory, so the
// step waits for the device once after the matching.
static void coarsen_level(Ctx& Cx, Level& F, Level& Cl, uint64_t seed, uint64_t comp, int32_t level, int32_t mm,
                          hipStream_t s) {
  int32_t k = F.k, l = F.l;
  int64_t np = F.np;
  uint64_t mkey = kTagMatch | ((uint64_t)level << 8) | (comp << 32);
  // Rounds run in groups of kRounds with one host check per group: a round
  // after the one that matched nothing changes nothing, so the extra rounds
  // of the last group leave the matching as it is (and return at once).
  constexpr int kRounds = 8;
  Buf<int32_t> mate(Cx.pool, k), best(Cx.pool, k), chg(Cx.pool, kRounds);
  fill_i32(mate.p, -1, k, s);
  // the vertices scanned by chunks, and their chunks: at most one per
  // kMatchChunk pins of the dual plus one per listed vertex
  Buf<int32_t> mlist(Cx.pool, (size_t)k + 1), cstart(Cx.pool, (size_t)k + 1), hdone(Cx.pool, (size_t)k);
  Buf<uint8_t> listed(Cx.pool, (size_t)k);
  const int64_t ccap = (int64_t)k + np / kMatchChunk + 1;
  Buf<ChunkBest> cres(Cx.pool, (size_t)ccap);
  fill_i32(mlist.p, 0, 1, s);
  VMO_LAUNCH(k_match_list, gsz(k), kLT, 0, s, F.ptr.p, F.dptr.p, F.dpins.p, k, mm, mlist.p, listed.p);
  VMO_LAUNCH(k_match_chunks, gsz(k), kLT, 0, s, mlist.p, F.dptr.p, (int64_t)k, cstart.p);
  scan_exclusive<int32_t>(Cx, cstart.p, cstart.p, k, cstart.p + k, s);
  fill_i32(hdone.p, 0, k, s);
  const MatchJob mj{F.ptr.p, F.pins.p, F.dptr.p, F.dpins.p, F.c.p, k, mm, mate.p, seed, mkey, mlist.p,
                    listed.p, cstart.p, cres.p, hdone.p};
  const int64_t hb = std::min<int64_t>(kHeavyBlocks, (ccap + kLT / 64 - 1) / (kLT / 64));
  // every round matches at least the best remaining pair, so at most k/2 + 1
  for (int64_t round = 0;; round += kRounds) {
    VMO_REQUIRE(round <= (int64_t)k / 2 + 1, "matching did not settle");
    VMO_HIP(hipMemsetAsync(chg.p, 0, 4 * kRounds, s));
    for (int r = 0; r < kRounds; ++r) {
      const int32_t* prev = r > 0 ? chg.p + r - 1 : nullptr;
      VMO_LAUNCH(k_match_best, (unsigned)(hb + gsz(k)), kLT, 0, s, mj, (int32_t)hb, prev, best.p);
      VMO_LAUNCH(k_match_pair, gsz(k), kLT, 0, s, best.p, k, prev, mate.p, chg.p + r);
    }
    if (read1(chg.p + kRounds - 1, s) == 0) break;
  }
  Buf<int32_t> root(Cx.pool, k), gmin(Cx.pool, k), flag(Cx.pool, (size_t)k + 1), rank(Cx.pool, (size_t)k + 1);
  VMO_LAUNCH(k_group_root, gsz(k), kLT, 0, s, F.ptr.p, F.pins.p, F.dptr.p, F.dpins.p, k, mm, mate.p, root.p, gmin.p);
  fill_i32(gmin.p, k, k, s);
  VMO_LAUNCH(k_group_min, gsz(k), kLT, 0, s, root.p, k, gmin.p);
  VMO_LAUNCH(k_group_flag, gsz(k), kLT, 0, s, root.p, gmin.p, k, flag.p);
  scan_exclusive<int32_t>(Cx, flag.p, rank.p, k, rank.p + k, s);
  const int32_t* kc_dev = rank.p + k;  // coarse vertices (groups)
  F.pi = Buf<int32_t>(Cx.pool, k);
  Buf<uint32_t> gkey(Cx.pool, k);
  Buf<int32_t> members(Cx.pool, k);
  VMO_LAUNCH(k_group_pi, gsz(k), kLT, 0, s, root.p, gmin.p, rank.p, k, F.pi.p, gkey.p);
  iota_i32(members.p, k, s);
  radix_sort<uint32_t>(Cx, gkey.p, members.p, k, bits_for((uint64_t)(k - 1)), s);
  Buf<int64_t> gstart(Cx.pool, (size_t)k + 1);
  fill_i64(gstart.p, 0, (int64_t)k + 1, s);
  VMO_LAUNCH(k_count_i32, gsz(k), kLT, 0, s, F.pi.p, (int64_t)k, gstart.p);
  scan_exclusive<int64_t>(Cx, gstart.p, gstart.p, k, gstart.p + k, s);
  Cl.w = Buf<float>(Cx.pool, k);
  VMO_LAUNCH(k_coarse_w, gsz(k), kLT, 0, s, gstart.p, members.p, F.w.p, kc_dev, Cl.w.p);
  // net images
  Cl.ptr = Buf<int64_t>(Cx.pool, (size_t)(l > 0 ? l : 0) + 1);
  const int32_t* lc_dev = nullptr;
  const int64_t* cnp_dev = nullptr;
  Buf<int32_t> cidx;
  if (l > 0 && np > 0) {
    Buf<uint64_t> key(Cx.pool, np);
    VMO_LAUNCH(k_img_keys, gsz(l), kLT, 0, s, F.ptr.p, F.pins.p, l, F.pi.p, key.p);
    radix_sort<uint64_t>(Cx, key.p, nullptr, np, 32 + bits_for((uint64_t)l), s);
    Buf<int32_t> ufl(Cx.pool, np + 1), uscan(Cx.pool, np + 1);
    Buf<int64_t> ilen(Cx.pool, l);
    fill_i64(ilen.p, 0, l, s);
    VMO_LAUNCH(k_img_uniq, gsz(np), kLT, 0, s, key.p, np, ufl.p, ilen.p);
    scan_exclusive<int32_t>(Cx, ufl.p, uscan.p, np, uscan.p + np, s);
    Buf<int32_t> kf(Cx.pool, (size_t)l + 1), kidx(Cx.pool, (size_t)l + 1);
    VMO_LAUNCH(k_img_keep, gsz(l), kLT, 0, s, ilen.p, l, kf.p);
    scan_exclusive<int32_t>(Cx, kf.p, kidx.p, l, kidx.p + l, s);
    const int32_t* nk_dev = kidx.p + l;  // kept nets (images of at least two coarse vertices)
    Buf<int64_t> iptr(Cx.pool, (size_t)l + 1);
    fill_i64(iptr.p, 0, (int64_t)l + 1, s);
    VMO_LAUNCH(k_img_len, gsz(l), kLT, 0, s, ilen.p, kf.p, kidx.p, l, iptr.p);
    scan_exclusive<int64_t>(Cx, iptr.p, iptr.p, l, iptr.p + l, s);
    Buf<int32_t> ipins(Cx.pool, np);
    VMO_LAUNCH(k_img_pins, gsz(np), kLT, 0, s, key.p, ufl.p, uscan.p, F.ptr.p, kf.p, kidx.p, iptr.p, np, ipins.p);
    Buf<uint64_t> hs(Cx.pool, l);
    Buf<int32_t> val(Cx.pool, l), repflag(Cx.pool, (size_t)l + 1), reppos(Cx.pool, l);
    cidx = Buf<int32_t>(Cx.pool, (size_t)l + 1);
    Buf<int32_t> kept_net(Cx.pool, l);
    VMO_LAUNCH(k_kept_net, gsz(l), kLT, 0, s, kf.p, kidx.p, l, kept_net.p);
    VMO_LAUNCH(k_img_hash, gsz(l), kLT, 0, s, iptr.p, ipins.p, nk_dev, l, hs.p, val.p);
    radix_sort<uint64_t>(Cx, hs.p, val.p, l, 64, s);
    fill_i32(repflag.p, 0, (int64_t)l + 1, s);
    VMO_LAUNCH(k_img_rep, gsz(l), kLT, 0, s, hs.p, val.p, iptr.p, ipins.p, nk_dev, repflag.p, reppos.p);
    scan_exclusive<int32_t>(Cx, repflag.p, cidx.p, l, cidx.p + l, s);
    lc_dev = cidx.p + l;  // coarse nets
    Cl.c = Buf<float>(Cx.pool, l);
    Buf<int64_t> clen(Cx.pool, (size_t)l + 1);
    fill_i64(clen.p, 0, (int64_t)l + 1, s);
    VMO_LAUNCH(k_img_cost, gsz(l), kLT, 0, s, hs.p, val.p, reppos.p, kept_net.p, F.c.p, iptr.p, cidx.p, nk_dev, Cl.c.p,
               clen.p);
    scan_exclusive<int64_t>(Cx, clen.p, Cl.ptr.p, l, Cl.ptr.p + l, s);
    cnp_dev = Cl.ptr.p + l;  // coarse pins
    Cl.pins = Buf<int32_t>(Cx.pool, np);
    VMO_LAUNCH(k_coarse_pins, gsz(l), kLT, 0, s, repflag.p, cidx.p, iptr.p, ipins.p, Cl.ptr.p, nk_dev, Cl.pins.p);
  }
  Buf<int64_t> sizes(Cx.pool, 3);
  VMO_LAUNCH(k_coarse_sizes, 1, 1, 0, s, kc_dev, lc_dev, cnp_dev, sizes.p);
  int64_t hsz[3];
  read_bytes(hsz, sizes.p, sizeof hsz, s);
  Cl.k = (int32_t)hsz[0];
  Cl.l = (int32_t)hsz[1];
  Cl.np = hsz[2];
  if (Cl.l == 0) {
    fill_i64(Cl.ptr.p, 0, 1, s);
    Cl.c = Buf<float>(Cx.pool, 1);
    Cl.pins = Buf<int32_t>(Cx.pool, 1);
    Cl.np = 0;
  }
  VMO_HIP(hipStreamSynchronize(s));
}

// ======================================================= init / prolong ====
__global__ void k_init_x(int32_t k, uint64_t seed, uint64_t key, float a, float4* x) {
  GRID_STRIDE(v, k) {
    float c[4];
    for (int d = 0; d < 4; ++d) {
      uint64_t r = rng3(seed, key, (uint64_t)v, (uint64_t)d);
      float u = (float)(uint32_t)(r >> 40) * 0x1p-24f;
      c[d] = (u - 0.5f) * a;
    }
    x[v] = make_float4(c[0], c[1], c[2], c[3]);
  }
}
// eps = jitter * ext / kc^(1/4) from the coarse layout's box (ext its largest
// side), formed by every thread as the host would.
__global__ void k_prolong(int32_t kf, const int32_t* pi, const float4* xc, uint64_t seed, uint64_t key, float sigma,
                          const uint32_t* box, double jitter, int32_t kc, float4* xf) {
  double ext = 0.0;
  for (int d = 0; d < 4; ++d) {
    const double a = (double)fkey_inv(box[4 + d]) - (double)fkey_inv(box[d]);
    if (a > ext) ext = a;
  }
  const double epsd = jitter * ext;
  const float eps = (float)(epsd / sqrt(sqrt((double)kc)));
  GRID_STRIDE(v, kf) {
    const float4 cv = xc[pi[v]];
    const float cc[4] = {cv.x, cv.y, cv.z, cv.w};
    float o[4];
    for (int d = 0; d < 4; ++d) {
      uint64_t r = rng3(seed, key, (uint64_t)v, (uint64_t)d);
      float u = (float)(uint32_t)(r >> 40) * 0x1p-23f;
      u = u - 1.0f;
      float a = sigma * cc[d];
      float b = eps * u;
      o[d] = a + b;
    }
    xf[v] = make_float4(o[0], o[1], o[2], o[3]);
  }
}
// Coordinates between the caller's layout ([4][k], one array per dimension)
// and the descent's (one 16-byte record per vertex).
__global__ void k_to_rec(const float* x, int32_t k, float4* r) {
  GRID_STRIDE(v, k) r[v] = make_float4(x[v], x[(int64_t)k + v], x[2 * (int64_t)k + v], x[3 * (int64_t)k + v]);
}
__global__ void k_from_rec(const float4* r, int32_t k, float* x) {
  GRID_STRIDE(v, k) {
    const float4 a = r[v];
    x[v] = a.x;
    x[(int64_t)k + v] = a.y;
    x[2 * (int64_t)k + v] = a.z;
    x[3 * (int64_t)k + v] = a.w;
  }
}

// Multilevel layout of one connected hypergraph (Algorithm 2).  L[0] is the
// finest level (with its dual); x [4][k0] output.
static void layout_component(Ctx& C, std::vector<Level>& L, const vmo_layout_params* p, uint64_t comp, float* xout,
                             hipStream_t s) {
  int32_t J = 0;
  while (L[J].k > p->min_coarse && J < p->max_levels) {
    Level Cl;
    coarsen_level(C, L[J], Cl, p->seed, comp, J, p->match_max_net, s);
    if ((double)Cl.k > (double)p->stall * (double)L[J].k) {
      L[J].pi = Buf<int32_t>();
      break;
    }
    make_dual(C, Cl, s);
    L.push_back(std::move(Cl));
    ++J;
  }
  Buf<float4> x(C.pool, (size_t)L[J].k);
  {
    float a = (float)sqrt(sqrt((double)L[J].k));
    uint64_t key = kTagInit | ((uint64_t)J << 8) | (comp << 32);
    VMO_LAUNCH(k_init_x, gsz(L[J].k), kLT, 0, s, L[J].k, p->seed, key, a, x.p);
  }
  GradWork gw;
  for (int32_t j = J; j >= 0; --j) {
    int32_t iters = j == J ? p->coarsest_iters : p->level_iters;
    Buf<float4> y(C.pool, (size_t)L[j].k);
    // the step lengths stay on the device: no read-back inside the descent
    for (int32_t it = 0; it < iters; ++it) descent_step(C, L[j], x.p, p, it, nullptr, y.p, gw, s);
    if (j > 0) {
      if (!gw.box.p) gw.box = Buf<uint32_t>(C.pool, 8);
      box_of(x.p, L[j].k, gw.box.p, s);
      gw.box_reset = false;  // it holds this box now
      int32_t kf = L[j - 1].k, kc = L[j].k;
      float sigma = (float)sqrt(sqrt((double)kf / (double)kc));
      uint64_t key = kTagProlong | ((uint64_t)(j - 1) << 8) | (comp << 32);
      Buf<float4> xf(C.pool, (size_t)kf);
      VMO_LAUNCH(k_prolong, gsz(kf), kLT, 0, s, kf, L[j - 1].pi.p, x.p, p->seed, key, sigma, gw.box.p,
                 (double)p->jitter, kc, xf.p);
      x = std::move(xf);
    }
  }
  VMO_LAUNCH(k_from_rec, gsz(L[0].k), kLT, 0, s, x.p, L[0].k, xout);
  VMO_HIP(hipStreamSynchronize(s));
}

// ============================================================ components ===
__global__ void k_comp_flag(const uint32_t* lab_sorted, int32_t k, int32_t* flag) {
  GRID_STRIDE(i, k) flag[i] = (i == 0 || lab_sorted[i] != lab_sorted[i - 1]) ? 1 : 0;
}
__global__ void k_comp_index(const int32_t* vorder, const int32_t* cscan, const int32_t* flag, int32_t k,
                             int32_t* comp_of, int32_t* cstart) {
  GRID_STRIDE(i, k) {
    int32_t c = cscan[i] + flag[i] - 1;  // inclusive count - 1
    comp_of[vorder[i]] = c;
    if (flag[i]) cstart[c] = (int32_t)i;
  }
}
__global__ void k_local_id(const int32_t* vorder, const int32_t* comp_of, const int32_t* cstart, int32_t k,
                           int32_t* loc) {
  GRID_STRIDE(i, k) loc[vorder[i]] = (int32_t)i - cstart[comp_of[vorder[i]]];
}
__global__ void k_net_comp(const int64_t* ptr, const int32_t* pins, int32_t l, const int32_t* comp_of, int32_t ncomp,
                           uint32_t* key, int32_t* val) {
  GRID_STRIDE(e, l) {
    key[e] = ptr[e + 1] > ptr[e] ? (uint32_t)comp_of[pins[ptr[e]]] : (uint32_t)ncomp;
    val[e] = (int32_t)e;
  }
}
// start[g] = the first position of the ascending keys with key >= g, for
// g = 0..G (keys below G; start[G] = n).
__global__ void k_sorted_starts(const uint32_t* key, int64_t n, uint32_t G, int64_t* start) {
  GRID_STRIDE(i, n + 1) {
    const uint32_t cur = i < n ? key[i] : G;
    const uint32_t from = i > 0 ? key[i - 1] + 1 : 0u;
    for (uint32_t g = from; g <= cur; ++g) start[g] = i;
  }
}
// The label of component c: its smallest vertex id (the first in id order).
__global__ void k_comp_label(const int32_t* vorder, const int32_t* cstart, int32_t ncomp, int32_t* lab) {
  GRID_STRIDE(c, ncomp) lab[c] = vorder[cstart[c]];
}
__global__ void k_net_len(const int64_t* ptr, const int32_t* order, int32_t l, int64_t* len) {
  GRID_STRIDE(t, l) len[t] = ptr[order[t] + 1] - ptr[order[t]];
}
__global__ void k_net_fill(const int64_t* ptr, const int32_t* pins, const int32_t* order, const int64_t* optr,
                           const int32_t* loc, const float* c, int32_t l, int32_t* opins, float* oc) {
  GRID_STRIDE(t, l) {
    int32_t e = order[t];
    int64_t o = optr[t];
    for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) opins[o + (p - ptr[e])] = loc[pins[p]];
    oc[t] = c ? c[e] : 1.0f;
  }
}
__global__ void k_gather_w(const int32_t* vorder, const float* w, int32_t k, float* ow) {
  GRID_STRIDE(i, k) ow[i] = w ? w[vorder[i]] : 1.0f;
}
__global__ void k_sub_ptr(const int64_t* in, int64_t n, int64_t sub, int64_t* out) {
  GRID_STRIDE(i, n) out[i] = in[i] - sub;
}
__global__ void k_comp_box(const float* xl, int32_t k, const int32_t* comp_of_pos, uint32_t* boxes) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1;
  uint32_t mn[4], mx[4];
  for (int d = 0; d < 4; ++d) { mn[d] = 0xffffffffu; mx[d] = 0u; }
  if (i < k) {
    key = comp_of_pos[i];
    for (int d = 0; d < 4; ++d) mn[d] = mx[d] = fkey(xl[(int64_t)d * k + i]);
  }
  int lane = threadIdx.x & 63;
  for (int off = 1; off < 64; off <<= 1) {
    int ok = __shfl_down(key, off, 64);
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
      atomicMin(&boxes[8 * (int64_t)key + d], mn[d]);
      atomicMax(&boxes[8 * (int64_t)key + 4 + d], mx[d]);
    }
}
__global__ void k_comp_pos(const int32_t* vorder, const int32_t* comp_of, int32_t k, int32_t* cpos) {
  GRID_STRIDE(i, k) cpos[i] = comp_of[vorder[i]];
}
__global__ void k_boxes_init(uint32_t* b, int64_t n) {
  GRID_STRIDE(i, n) b[i] = (i & 7) < 4 ? 0xffffffffu : 0u;
}
// Packing: component c is shifted so its box minimum sits at (off_c, 0, 0, 0).
__global__ void k_pack(const float* xl, const int32_t* vorder, const int32_t* cpos, const float* clo,
                       const double* coff, int32_t k, float* x) {
  GRID_STRIDE(i, k) {
    int32_t v = vorder[i], c = cpos[i];
    double t0 = (double)xl[i] - (double)clo[4 * (int64_t)c];
    x[v] = (float)(t0 + coff[c]);
    for (int d = 1; d < 4; ++d)
      x[(int64_t)d * k + v] = (float)((double)xl[(int64_t)d * k + i] - (double)clo[4 * (int64_t)c + d]);
  }
}
// Copy component c's SoA block (k_c points at offset o of xl) from x_c.
__global__ void k_put_comp(const float* xc, int32_t kc, int32_t o, int32_t k, float* xl) {
  GRID_STRIDE(i, kc) for (int d = 0; d < 4; ++d) xl[(int64_t)d * k + o + i] = xc[(int64_t)d * kc + i];
}

static void check_params(const vmo_layout_params* p) {
  VMO_REQUIRE(p != nullptr, "layout parameters are NULL");
  VMO_REQUIRE(p->coarsest_iters >= 0 && p->level_iters >= 0, "iteration counts must be >= 0");
  VMO_REQUIRE(p->min_coarse >= 1 && p->max_levels >= 0, "min_coarse >= 1 and max_levels >= 0");
  VMO_REQUIRE(p->leaf_cap >= 1 && p->leaf_cap <= 64, "leaf_cap must be in [1, 64]");
  VMO_REQUIRE(p->match_max_net >= 2, "match_max_net must be >= 2");
  VMO_REQUIRE(p->theta >= 0.0f && p->step0_frac > 0.0f && p->decay > 0.0f, "theta >= 0, step0_frac > 0, decay > 0");
  VMO_REQUIRE(p->jitter >= 0.0f && p->stall > 0.0f && p->pack_gap >= 0.0f, "jitter, stall, pack_gap out of range");
}

// Host copy of one level from device arrays (the finest level of a component).
static Level level_from(Ctx& C, int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, const float* w,
                        const float* c, hipStream_t s) {
  Level L;
  L.k = k;
  L.l = l;
  L.np = read1(ptr + l, s) - read1(ptr, s);
  int64_t base = read1(ptr, s);
  L.ptr = Buf<int64_t>(C.pool, (size_t)l + 1);
  VMO_LAUNCH(k_sub_ptr, gsz((int64_t)l + 1), kLT, 0, s, ptr, (int64_t)l + 1, base, L.ptr.p);
  L.pins = Buf<int32_t>(C.pool, L.np > 0 ? L.np : 1);
  if (L.np > 0) VMO_HIP(hipMemcpyAsync(L.pins.p, pins + base, 4 * L.np, hipMemcpyDeviceToDevice, s));
  L.w = Buf<float>(C.pool, k);
  if (w) VMO_HIP(hipMemcpyAsync(L.w.p, w, 4 * (size_t)k, hipMemcpyDeviceToDevice, s));
  else VMO_LAUNCH(k_gather_w, gsz(k), kLT, 0, s, (const int32_t*)nullptr, (const float*)nullptr, k, L.w.p);
  L.c = Buf<float>(C.pool, l > 0 ? l : 1);
  if (l > 0) {
    if (c) VMO_HIP(hipMemcpyAsync(L.c.p, c, 4 * (size_t)l, hipMemcpyDeviceToDevice, s));
    else fill_i32(reinterpret_cast<int32_t*>(L.c.p), 0x3f800000, l, s);
  }
  make_dual(C, L, s);
  return L;
}

// =========================================================== entry points ==
void layout(Ctx& C, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, hipStream_t s) {
  check_params(p);
  validate_hypergraph(C, h, true, s);
  VMO_REQUIRE(x != nullptr, "x is NULL");
  int32_t k = h->k, l = h->l;
  struct KmaxScope {
    Ctx& c;
    ~KmaxScope() { c.layout_kmax = 0; }
  } kmax_scope{C};
  C.layout_kmax = k;
  Buf<int32_t> label(C.pool, k);
  components(C, k, l, h->net_ptr, h->pins, label.p, s);
  // vertices grouped by component (ascending label, ascending id)
  Buf<uint32_t> lkey(C.pool, k);
  Buf<int32_t> vorder(C.pool, k);
  VMO_HIP(hipMemcpyAsync(lkey.p, label.p, 4 * (size_t)k, hipMemcpyDeviceToDevice, s));
  iota_i32(vorder.p, k, s);
  radix_sort<uint32_t>(C, lkey.p, vorder.p, k, bits_for((uint64_t)(k - 1)), s);
  Buf<int32_t> cflag(C.pool, (size_t)k + 1), cscan(C.pool, (size_t)k + 1);
  VMO_LAUNCH(k_comp_flag, gsz(k), kLT, 0, s, lkey.p, k, cflag.p);
  scan_exclusive<int32_t>(C, cflag.p, cscan.p, k, cscan.p + k, s);
  int32_t ncomp = read1(cscan.p + k, s);
  Buf<int32_t> comp_of(C.pool, k), cstart(C.pool, (size_t)ncomp + 1), loc(C.pool, k);
  VMO_LAUNCH(k_comp_index, gsz(k), kLT, 0, s, vorder.p, cscan.p, cflag.p, k, comp_of.p, cstart.p);
  VMO_LAUNCH(k_local_id, gsz(k), kLT, 0, s, vorder.p, comp_of.p, cstart.p, k, loc.p);
  std::vector<int32_t> hstart(ncomp + 1), hlabel(ncomp);
  {
    Buf<int32_t> lab(C.pool, ncomp);
    VMO_LAUNCH(k_comp_label, gsz(ncomp), kLT, 0, s, vorder.p, cstart.p, ncomp, lab.p);
    read_bytes(hstart.data(), cstart.p, 4 * (size_t)ncomp, s);
    read_bytes(hlabel.data(), lab.p, 4 * (size_t)ncomp, s);
  }
  hstart[ncomp] = k;
  // nets grouped by component, local pins
  Buf<uint32_t> nkey(C.pool, l > 0 ? l : 1);
  Buf<int32_t> norder(C.pool, l > 0 ? l : 1);
  Buf<int64_t> optr(C.pool, (size_t)l + 1);
  Buf<int32_t> opins;
  Buf<float> oc(C.pool, l > 0 ? l : 1), ow(C.pool, k);
  std::vector<int64_t> hnstart(ncomp + 2, 0);
  if (l > 0) {
    VMO_LAUNCH(k_net_comp, gsz(l), kLT, 0, s, h->net_ptr, h->pins, l, comp_of.p, ncomp, nkey.p, norder.p);
    radix_sort<uint32_t>(C, nkey.p, norder.p, l, bits_for((uint64_t)ncomp), s);
    Buf<int64_t> len(C.pool, (size_t)l + 1);
    VMO_LAUNCH(k_net_len, gsz(l), kLT, 0, s, h->net_ptr, norder.p, l, len.p);
    scan_exclusive<int64_t>(C, len.p, optr.p, l, optr.p + l, s);
    int64_t np = read1(optr.p + l, s);
    opins = Buf<int32_t>(C.pool, np > 0 ? np : 1);
    VMO_LAUNCH(k_net_fill, gsz(l), kLT, 0, s, h->net_ptr, h->pins, norder.p, optr.p, loc.p, h->c, l, opins.p, oc.p);
    // nets of component c: [hnstart[c], hnstart[c + 1]) of the sorted keys
    // (key ncomp: the empty nets, last)
    Buf<int64_t> nst(C.pool, (size_t)ncomp + 2);
    VMO_LAUNCH(k_sorted_starts, gsz((int64_t)l + 1), kLT, 0, s, nkey.p, (int64_t)l, (uint32_t)ncomp + 1, nst.p);
    read_bytes(hnstart.data(), nst.p, 8 * ((size_t)ncomp + 2), s);
  } else {
    opins = Buf<int32_t>(C.pool, 1);
    fill_i64(optr.p, 0, 1, s);
  }
  VMO_LAUNCH(k_gather_w, gsz(k), kLT, 0, s, vorder.p, h->w, k, ow.p);
  // per component layout into xl (component-grouped positions)
  Buf<float> xl(C.pool, 4 * (size_t)k);
  VMO_HIP(hipMemsetAsync(xl.p, 0, 4 * 4 * (size_t)k, s));
  for (int32_t c = 0; c < ncomp; ++c) {
    int32_t kc = hstart[c + 1] - hstart[c];
    if (kc < 2) continue;
    int32_t lc = (int32_t)(hnstart[c + 1] - hnstart[c]);
    std::vector<Level> L;
    L.push_back(level_from(C, kc, lc, optr.p + hnstart[c], opins.p, ow.p + hstart[c], oc.p + hnstart[c], s));
    Buf<float> xc(C.pool, 4 * (size_t)kc);
    layout_component(C, L, p, (uint64_t)hlabel[c], xc.p, s);
    VMO_LAUNCH(k_put_comp, gsz(kc), kLT, 0, s, xc.p, kc, hstart[c], k, xl.p);
  }
  // packing along the first axis, components in label order
  Buf<int32_t> cpos(C.pool, k);
  VMO_LAUNCH(k_comp_pos, gsz(k), kLT, 0, s, vorder.p, comp_of.p, k, cpos.p);
  Buf<uint32_t> boxes(C.pool, 8 * (size_t)ncomp);
  VMO_LAUNCH(k_boxes_init, gsz(8 * (int64_t)ncomp), kLT, 0, s, boxes.p, 8 * (int64_t)ncomp);
  VMO_LAUNCH(k_comp_box, nblocks(k, kLT), kLT, 0, s, xl.p, k, cpos.p, boxes.p);
  std::vector<uint32_t> hb(8 * (size_t)ncomp);
  VMO_HIP(hipMemcpyAsync(hb.data(), boxes.p, 4 * hb.size(), hipMemcpyDeviceToHost, s));
  VMO_HIP(hipStreamSynchronize(s));
  std::vector<float> clo(4 * (size_t)ncomp);
  std::vector<double> cext(ncomp), coff(ncomp);
  double maxext = 0.0;
  for (int32_t c = 0; c < ncomp; ++c) {
    double e = 0.0;
    for (int d = 0; d < 4; ++d) {
      float lo = fkey_inv(hb[8 * c + d]), hi = fkey_inv(hb[8 * c + 4 + d]);
      clo[4 * c + d] = lo;
      double a = (double)hi - (double)lo;
      if (a > e) e = a;
    }
    cext[c] = e;
    if (e > maxext) maxext = e;
  }
  double gap = (double)p->pack_gap * maxext;
  double off = 0.0;
  for (int32_t c = 0; c < ncomp; ++c) {
    coff[c] = off;
    off = off + cext[c];
    off = off + gap;
  }
  Buf<float> dlo(C.pool, clo.size());
  Buf<double> doff(C.pool, coff.size());
  VMO_HIP(hipMemcpyAsync(dlo.p, clo.data(), 4 * clo.size(), hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(doff.p, coff.data(), 8 * coff.size(), hipMemcpyHostToDevice, s));
  VMO_LAUNCH(k_pack, gsz(k), kLT, 0, s, xl.p, vorder.p, cpos.p, dlo.p, doff.p, k, x);
}

void coarsen(Ctx& C, const vmo_hypergraph* h, uint64_t seed, uint64_t comp, int32_t level, int32_t mm, int32_t* pi,
             int64_t* cptr, int32_t* cpins, float* cw, float* cc, int32_t* kc, int32_t* lc, hipStream_t s) {
  validate_hypergraph(C, h, false, s);
  VMO_REQUIRE(pi && cptr && cpins && cw && cc && kc && lc, "NULL output");
  VMO_REQUIRE(mm >= 2, "match_max_net must be >= 2");
  Level F = level_from(C, h->k, h->l, h->net_ptr, h->pins, h->w, h->c, s);
  Level Cl;
  coarsen_level(C, F, Cl, seed, comp, level, mm, s);
  VMO_HIP(hipMemcpyAsync(pi, F.pi.p, 4 * (size_t)h->k, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipMemcpyAsync(cptr, Cl.ptr.p, 8 * ((size_t)Cl.l + 1), hipMemcpyDeviceToDevice, s));
  if (Cl.np > 0) VMO_HIP(hipMemcpyAsync(cpins, Cl.pins.p, 4 * (size_t)Cl.np, hipMemcpyDeviceToDevice, s));
  if (Cl.k > 0) VMO_HIP(hipMemcpyAsync(cw, Cl.w.p, 4 * (size_t)Cl.k, hipMemcpyDeviceToDevice, s));
  if (Cl.l > 0) VMO_HIP(hipMemcpyAsync(cc, Cl.c.p, 4 * (size_t)Cl.l, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipStreamSynchronize(s));
  *kc = Cl.k;
  *lc = Cl.l;
}

__global__ void k_tree_out(int32_t n, NodeView nd, int32_t* ints, int32_t* cell2, float* flt) {
  GRID_STRIDE(t, n) {
    int4 b = nd.t[t].b;
    int4 a;  // the cell centre back from A = -2 c (exact)
    a.x = (int)(-0.5 * nd.t[t].A[0]); a.y = (int)(-0.5 * nd.t[t].A[1]);
    a.z = (int)(-0.5 * nd.t[t].A[2]); a.w = (int)(-0.5 * nd.t[t].A[3]);
    float4 X = nd.t[t].X;
    int32_t* r = ints + 8 * t;
    r[0] = b.y; r[1] = b.z; r[2] = b.w & 255; r[3] = (b.w >> 8) & 1; r[4] = b.x; r[5] = r[6] = r[7] = 0;
    cell2[4 * t] = a.x; cell2[4 * t + 1] = a.y; cell2[4 * t + 2] = a.z; cell2[4 * t + 3] = a.w;
    flt[5 * t] = nd.t[t].W;
    flt[5 * t + 1] = X.x; flt[5 * t + 2] = X.y; flt[5 * t + 3] = X.z; flt[5 * t + 4] = X.w;
  }
}

void tree(Ctx& C, const float* x, const float* w, int32_t k, int32_t cap, int32_t* ints, int32_t* cell2, float* flt,
          int32_t* order, int32_t max_nodes, int32_t* n_nodes, hipStream_t s) {
  VMO_REQUIRE(k >= 1, "k must be >= 1");
  VMO_REQUIRE(cap >= 1 && cap <= 64, "leaf_cap must be in [1, 64]");
  VMO_REQUIRE(ints && cell2 && flt && order && n_nodes, "NULL output");
  validate_finite(C, x, 4 * (int64_t)k, "x", s);
  Buf<uint32_t> box(C.pool, 8);
  Buf<float4> xr(C.pool, (size_t)k);
  VMO_LAUNCH(k_to_rec, gsz(k), kLT, 0, s, x, k, xr.p);
  box_of(xr.p, k, box.p, s);
  Tree T;
  // the same builds as the layout's: one workgroup up to kSmallK points
  build_tree(C, T, xr.p, w, k, cap, box.p, 0.25, s);
  const int32_t n = read1(T.nn.p + k, s);
  VMO_REQUIRE(n <= max_nodes, "max_nodes is too small");
  VMO_LAUNCH(k_tree_out, gsz(n), kLT, 0, s, n, T.view(), ints, cell2, flt);
  VMO_HIP(hipMemcpyAsync(order, T.order.p, 4 * (size_t)k, hipMemcpyDeviceToDevice, s));
  *n_nodes = n;
}

void gradient(Ctx& C, const vmo_hypergraph* h, const float* x, float theta, int32_t cap, float* y, float* z,
              int64_t* nint, hipStream_t s) {
  validate_hypergraph(C, h, false, s);
  VMO_REQUIRE(cap >= 1 && cap <= 64, "leaf_cap must be in [1, 64]");
  VMO_REQUIRE(y != nullptr, "y is NULL");
  validate_finite(C, x, 4 * (int64_t)h->k, "x", s);
  Level L = level_from(C, h->k, h->l, h->net_ptr, h->pins, h->w, h->c, s);
  GradWork gw;
  Buf<unsigned long long> cnt(C.pool, 1);  // written by the walk's counter sum
  Buf<float4> xr(C.pool, (size_t)L.k), yr(C.pool, (size_t)L.k);
  VMO_LAUNCH(k_to_rec, gsz(L.k), kLT, 0, s, x, L.k, xr.p);
  gradient_prepare(C, L, xr.p, (double)theta * (double)theta, cap, yr.p, gw, s);
  gradient_walk(C, L, yr.p, nullptr, 0.0, gw, cnt.p, s);
  VMO_LAUNCH(k_from_rec, gsz(L.k), kLT, 0, s, yr.p, L.k, y);
  if (z && L.l > 0) VMO_LAUNCH(k_z_soa, gsz(L.l), kLT, 0, s, gw.z.p, L.l, z);
  const unsigned long long c = L.k > 0 ? read1(cnt.p, s) : 0ull;
  if (nint) *nint = (int64_t)c;
}

void layout_steps(Ctx& C, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, int32_t it0, int32_t iters,
                  double* alpha, hipStream_t s) {
  check_params(p);
  validate_hypergraph(C, h, false, s);
  VMO_REQUIRE(x && alpha && it0 >= 0 && iters >= 0, "bad arguments");
  Level L = level_from(C, h->k, h->l, h->net_ptr, h->pins, h->w, h->c, s);
  GradWork gw;
  Buf<float4> xr(C.pool, (size_t)h->k), y(C.pool, (size_t)h->k);
  VMO_LAUNCH(k_to_rec, gsz(h->k), kLT, 0, s, x, h->k, xr.p);
  double a = *alpha;
  for (int32_t t = 0; t < iters; ++t) descent_step(C, L, xr.p, p, it0 + t, &a, y.p, gw, s);
  VMO_LAUNCH(k_from_rec, gsz(h->k), kLT, 0, s, xr.p, h->k, x);
  *alpha = a;
}

}  // namespace vmo
