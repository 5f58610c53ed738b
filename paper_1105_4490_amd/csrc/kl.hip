// Kernighan-Lin refinement of bisections of a graph (Sec. 3: partitionings
// made by Algorithm 4 improve under a few Kernighan-Lin iterations; Kernighan
// and Lin 1970).  Every net is an edge of weight 1 (parallel edges add up).
// label[v] = 2 g + s puts v on side s of bisection g (-1: left out); each
// bisection is refined on its own, by one workgroup, with only the edges
// inside it counting.
//
// A pass keeps D(v) = (edges to the other side) - (edges to its own side) in
// device memory and runs min(|A|, |B|) steps.  A step takes the unlocked pair
// (a in A, b in B) of largest gain D(a) + D(b) - 2 m(a, b) (m = edges joining
// them), ties to the smallest a, then the smallest b; it locks both and moves
// the D of their unlocked neighbours as if they had swapped.  The best pair is
// found without visiting all pairs: every unlocked a of A forms its best gain
// from its unlocked neighbours in B (with their multiplicities) and from the
// largest D among the B vertices it does not touch, read off a histogram of the
// unlocked B vertices' D (a value d is free for a when more B vertices have
// D = d than a has distinct neighbours there); one packed 64-bit maximum gives
// the best gain with the smallest a, one minimum the smallest b reaching it.
// After the steps, the smallest j of largest prefix gain G(j) is found by a
// block scan; if G(j) > 0 the first j pairs change sides, else the bisection
// is done.
#include "vmo_internal.h"

namespace vmo {

constexpr int kKT = 512;
constexpr int kKlMaxDeg = 1024;  // histogram of D in [-maxdeg, maxdeg] in LDS

__device__ __forceinline__ int32_t kl_other(const int32_t* pins, int32_t e, int32_t v) {
  return pins[2 * e] + pins[2 * e + 1] - v;
}
// D is changed by atomic adds, which the L1 cache of the CU does not see:
// its reads go to L2.
__device__ __forceinline__ int32_t ldD(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kKT) void k_kl(const int64_t* __restrict__ dptr, const int32_t* __restrict__ dnets,
                                            const int32_t* __restrict__ pins, const int32_t* __restrict__ gbeg,
                                            const int32_t* __restrict__ mem, int32_t* __restrict__ label,
                                            int32_t* __restrict__ D, int32_t* __restrict__ lk,
                                            int32_t* __restrict__ pa, int32_t* __restrict__ pb,
                                            int32_t* __restrict__ pg, int32_t passes, int32_t maxdeg,
                                            long long* __restrict__ gain) {
  const int32_t g = blockIdx.x, t = threadIdx.x;
  const int32_t m0 = gbeg[g], n = gbeg[g + 1] - m0;
  const int32_t lA = 2 * g, lB = 2 * g + 1;
  __shared__ int32_t hist[2 * kKlMaxDeg + 1];
  __shared__ int32_t sh_n[2], sh_dmax, sh_b;
  __shared__ unsigned long long sh_best;
  __shared__ long long sh_scan[kKT];
  __shared__ unsigned long long sh_pre;
  __shared__ int32_t sh_stop;
  const int H = 2 * maxdeg + 1;

  if (t < 2) sh_n[t] = 0;
  __syncthreads();
  {
    int na = 0, nb = 0;
    for (int32_t i = t; i < n; i += kKT) (label[mem[m0 + i]] == lA ? na : nb)++;
    if (na) atomicAdd(&sh_n[0], na);
    if (nb) atomicAdd(&sh_n[1], nb);
  }
  __syncthreads();
  const int32_t steps = min(sh_n[0], sh_n[1]);
  long long total = 0;
  for (int32_t pass = 0; pass < passes && steps > 0; ++pass) {
    // D from the current sides; everything unlocked
    for (int32_t i = t; i < n; i += kKT) {
      const int32_t v = mem[m0 + i];
      const int32_t sv = label[v];
      int32_t d = 0;
      for (int64_t p = dptr[v]; p < dptr[v + 1]; ++p) {
        const int32_t w = kl_other(pins, dnets[p], v);
        const int32_t lw = label[w];
        if (lw == lA || lw == lB) d += lw != sv ? 1 : -1;
      }
      D[v] = d;
      lk[v] = 0;
    }
    __syncthreads();
    int32_t nst = steps;
    for (int32_t st = 0; st < steps; ++st) {
      // histogram of D over the unlocked B vertices, and its largest value
      for (int i = t; i < H; i += kKT) hist[i] = 0;
      if (t == 0) {
        sh_dmax = -kKlMaxDeg - 1;
        sh_best = 0ull;
        sh_b = INT32_MAX;
      }
      __syncthreads();
      {
        int dm = -kKlMaxDeg - 1;
        for (int32_t i = t; i < n; i += kKT) {
          const int32_t v = mem[m0 + i];
          if (label[v] != lB || lk[v]) continue;
          const int32_t d = ldD(&D[v]);
          atomicAdd(&hist[d + maxdeg], 1);
          dm = max(dm, d);
        }
        for (int off = 32; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off, 64));
        if ((t & 63) == 0) atomicMax(&sh_dmax, dm);
      }
      __syncthreads();
      const int32_t dmax = sh_dmax;
      // every unlocked a of A: its best gain
      for (int32_t i = t; i < n; i += kKT) {
        const int32_t a = mem[m0 + i];
        if (label[a] != lA || lk[a]) continue;
        const int32_t Da = ldD(&D[a]);
        const int64_t p0 = dptr[a], p1 = dptr[a + 1];
        int32_t best = INT32_MIN;
        // neighbours in B: gain with the multiplicity, once per distinct b
        for (int64_t p = p0; p < p1; ++p) {
          const int32_t b = kl_other(pins, dnets[p], a);
          if (label[b] != lB || lk[b]) continue;
          bool first = true;
          int32_t mult = 1;
          for (int64_t q = p0; q < p1; ++q) {
            if (q == p) continue;
            if (kl_other(pins, dnets[q], a) == b) {
              if (q < p) { first = false; break; }
              ++mult;
            }
          }
          if (!first) continue;
          best = max(best, Da + ldD(&D[b]) - 2 * mult);
        }
        // the largest D among the B vertices a does not touch
        for (int32_t d = dmax; d >= -maxdeg; --d) {
          const int32_t c = hist[d + maxdeg];
          if (c == 0) continue;
          int32_t nb = 0;  // distinct unlocked neighbours in B with D = d
          for (int64_t p = p0; p < p1; ++p) {
            const int32_t b = kl_other(pins, dnets[p], a);
            if (label[b] != lB || lk[b] || ldD(&D[b]) != d) continue;
            bool first = true;
            for (int64_t q = p0; q < p; ++q)
              if (kl_other(pins, dnets[q], a) == b) { first = false; break; }
            nb += first;
          }
          if (c > nb) {
            best = max(best, Da + d);
            break;
          }
        }
        if (best == INT32_MIN) continue;
        // larger gain first, then the smaller a
        const unsigned long long key = ((unsigned long long)(uint32_t)(best + (1 << 30)) << 32) |
                                       (unsigned long long)(uint32_t)(0x7fffffff - a);
        atomicMax(&sh_best, key);
      }
      __syncthreads();
      const unsigned long long bk = sh_best;
      if (bk == 0ull) {  // unreachable while both sides have unlocked vertices
        nst = st;
        break;
      }
      const int32_t gstar = (int32_t)(bk >> 32) - (1 << 30);
      const int32_t astar = 0x7fffffff - (int32_t)(bk & 0xffffffffull);
      const int32_t Das = ldD(&D[astar]);
      const int64_t q0 = dptr[astar], q1 = dptr[astar + 1];
      // the smallest b reaching the gain: among the neighbours of a* ...
      for (int64_t p = q0 + t; p < q1; p += kKT) {
        const int32_t b = kl_other(pins, dnets[p], astar);
        if (label[b] != lB || lk[b]) continue;
        int32_t mult = 0;
        for (int64_t q = q0; q < q1; ++q) mult += kl_other(pins, dnets[q], astar) == b;
        if (Das + ldD(&D[b]) - 2 * mult == gstar) atomicMin(&sh_b, b);
      }
      // ... and among the B vertices a* does not touch
      const int32_t want = gstar - Das;
      for (int32_t i = t; i < n; i += kKT) {
        const int32_t b = mem[m0 + i];
        if (label[b] != lB || lk[b] || ldD(&D[b]) != want) continue;
        bool adj = false;
        for (int64_t q = q0; q < q1; ++q)
          if (kl_other(pins, dnets[q], astar) == b) { adj = true; break; }
        if (!adj) atomicMin(&sh_b, b);
      }
      __syncthreads();
      const int32_t bstar = sh_b;
      if (bstar == INT32_MAX) {  // unreachable: the best gain has a partner
        nst = st;
        break;
      }
      if (t == 0) {
        lk[astar] = 1;
        lk[bstar] = 1;
        pa[m0 + st] = astar;
        pb[m0 + st] = bstar;
        pg[m0 + st] = gstar;
      }
      __syncthreads();
      // D of the unlocked vertices of the bisection as if a* and b* swapped
      {
        const int64_t na = q1 - q0, nbb = dptr[bstar + 1] - dptr[bstar];
        for (int64_t p = t; p < na + nbb; p += kKT) {
          const int32_t x = p < na ? astar : bstar;
          const int32_t w = kl_other(pins, dnets[p < na ? q0 + p : dptr[bstar] + (p - na)], x);
          const int32_t lw = label[w];
          if ((lw != lA && lw != lB) || lk[w]) continue;
          atomicAdd(&D[w], lw == label[x] ? 2 : -2);
        }
      }
      __syncthreads();
    }
    // the smallest j of largest prefix gain (block scan over the steps)
    const int32_t per = (nst + kKT - 1) / kKT;
    const int32_t s0 = t * per, s1 = min(nst, s0 + per);
    long long loc = 0;
    for (int32_t s = s0; s < s1; ++s) loc += pg[m0 + s];
    sh_scan[t] = loc;
    if (t == 0) sh_pre = 0ull;
    __syncthreads();
    for (int off = 1; off < kKT; off <<= 1) {
      const long long v = t >= off ? sh_scan[t - off] : 0;
      __syncthreads();
      sh_scan[t] += v;
      __syncthreads();
    }
    {
      long long run = sh_scan[t] - loc;
      long long bv = LLONG_MIN;
      int32_t bi = -1;
      for (int32_t s = s0; s < s1; ++s) {
        run += pg[m0 + s];
        if (run > bv) { bv = run; bi = s; }
      }
      if (bi >= 0) {
        // larger prefix first, then the smaller index (|prefix| < 2^37, steps < 2^25)
        const unsigned long long key = ((unsigned long long)(bv + (1ll << 37)) << 25) |
                                       (unsigned long long)((1 << 25) - 1 - bi);
        atomicMax(&sh_pre, key);
      }
    }
    __syncthreads();
    const unsigned long long pk = sh_pre;
    const long long bestG = (long long)(pk >> 25) - (1ll << 37);
    const int32_t jstar = (1 << 25) - 1 - (int32_t)(pk & ((1ull << 25) - 1)) + 1;
    if (t == 0) sh_stop = pk == 0ull || bestG <= 0;
    __syncthreads();
    if (sh_stop) break;
    for (int32_t s = t; s < jstar; s += kKT) {
      label[pa[m0 + s]] = lB;
      label[pb[m0 + s]] = lA;
    }
    total += bestG;
    __syncthreads();
  }
  if (t == 0 && gain) gain[g] = total;
}

// label checks: bad |= 1 for a label below -1; the largest bisection index
__global__ void k_kl_labels(const int32_t* label, int32_t k, int* bad, int32_t* gmax) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t l = label[v];
    if (l < -1) atomicOr(bad, 1);
    if (l >= 0) atomicMax(gmax, l >> 1);
  }
}
__global__ void k_kl_keys(const int32_t* label, int32_t k, int32_t G, uint32_t* key, int32_t* val) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t l = label[v];
    key[v] = l >= 0 ? (uint32_t)(l >> 1) : (uint32_t)G;
    val[v] = (int32_t)v;
  }
}
// gbeg[g] = first position of bisection g in the sorted order (gbeg[G] = end)
__global__ void k_kl_bounds(const uint32_t* key, int32_t k, int32_t G, int32_t* gbeg) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= k; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cur = i < k ? key[i] : (uint32_t)G;
    const uint32_t prev = i > 0 ? key[i - 1] : 0u;
    const uint32_t from = i > 0 ? prev + 1 : 0u;
    for (uint32_t g = from; g <= cur && g <= (uint32_t)G; ++g) gbeg[g] = (int32_t)i;
  }
}
__global__ void k_maxdeg(const int64_t* dptr, int32_t k, int32_t* md) {
  int m = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x)
    m = max(m, (int)(dptr[v + 1] - dptr[v]));
  for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(md, m);
}

static unsigned ksz(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

void refine_kl(Ctx& c, const vmo_hypergraph* h, int32_t* label, int32_t passes, int64_t* gain, int32_t* ngroups,
               hipStream_t s) {
  VMO_REQUIRE(label != nullptr, "label is NULL");
  VMO_REQUIRE(passes >= 0, "passes must be >= 0");
  std::vector<int64_t> npins;
  validate_jobs(c, {JobCheck{h, nullptr, false, true}}, npins, s);
  const int32_t k = h->k, l = h->l;
  Buf<int> bad(c.pool, 1);
  Buf<int32_t> gm(c.pool, 2);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  fill_i32(gm.p, -1, 1, s);
  fill_i32(gm.p + 1, 0, 1, s);
  VMO_LAUNCH(k_kl_labels, ksz(k), 256, 0, s, label, k, bad.p, gm.p);
  VMO_REQUIRE(read1(bad.p, s) == 0, "labels must be -1 or 2 * bisection + side");
  const int32_t G = read1(gm.p, s) + 1;
  if (ngroups) *ngroups = G;
  if (G == 0 || passes == 0) {
    if (gain && G > 0) fill_i64(gain, 0, G, s);
    VMO_HIP(hipStreamSynchronize(s));
    return;
  }
  // adjacency: the edges at every vertex, ascending
  Buf<int64_t> dptr(c.pool, (int64_t)k + 1);
  Buf<int32_t> dnets(c.pool, 2 * (int64_t)l + 1);
  csr_transpose(c, l, k, h->net_ptr, h->pins, dptr.p, dnets.p, s);
  VMO_LAUNCH(k_maxdeg, ksz(k), 256, 0, s, dptr.p, k, gm.p + 1);
  const int32_t maxdeg = read1(gm.p + 1, s);
  VMO_REQUIRE(maxdeg <= kKlMaxDeg, "Kernighan-Lin refinement supports vertex degrees up to 1024");
  VMO_REQUIRE(k < (1 << 25), "Kernighan-Lin refinement supports up to 2^25 vertices");
  // members of every bisection, ascending ids
  Buf<uint32_t> key(c.pool, k);
  Buf<int32_t> mem(c.pool, k), gbeg(c.pool, (int64_t)G + 1);
  VMO_LAUNCH(k_kl_keys, ksz(k), 256, 0, s, label, k, G, key.p, mem.p);
  radix_sort<uint32_t>(c, key.p, mem.p, k, bits_for((uint64_t)G), s);
  VMO_LAUNCH(k_kl_bounds, ksz((int64_t)k + 1), 256, 0, s, key.p, k, G, gbeg.p);
  Buf<int32_t> D(c.pool, k), pa(c.pool, k), pb(c.pool, k), pg(c.pool, k);
  Buf<int32_t> lk(c.pool, k);
  Buf<long long> gl(c.pool, G);
  VMO_LAUNCH(k_kl, (unsigned)G, kKT, 0, s, dptr.p, dnets.p, h->pins, gbeg.p, mem.p, label, D.p, lk.p, pa.p, pb.p,
             pg.p, passes, maxdeg, gl.p);
  if (gain) VMO_HIP(hipMemcpyAsync(gain, gl.p, sizeof(int64_t) * G, hipMemcpyDeviceToDevice, s));
  VMO_HIP(hipStreamSynchronize(s));
}

}  // namespace vmo
