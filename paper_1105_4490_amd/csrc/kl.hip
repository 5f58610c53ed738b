// Kernighan-Lin refinement of bisections of a graph (Sec. 3: partitionings
// made by Algorithm 4 improve under a few Kernighan-Lin iterations; Kernighan
// and Lin 1970).  Every net is an edge of weight 1 (parallel edges add up).
// label[v] = 2 g + s puts v on side s of bisection g (-1: left out); each
// bisection is refined on its own, by one workgroup, with only the edges
// inside it counting.
//
// The members of every bisection get indices in ascending vertex id and a
// local adjacency (their neighbours inside the bisection, by member index).
// A pass keeps D(v) = (edges to the other side) - (edges to its own side) in
// LDS (device memory for bisections above 9,216 vertices) and runs
// min(|A|, |B|) steps.  A step takes the unlocked pair
// (a in A, b in B) of largest gain D(a) + D(b) - 2 m(a, b) (m = edges joining
// them), ties to the smallest a, then the smallest b; it locks both and moves
// the D of their unlocked neighbours as if they had swapped.  The best pair is
// found without visiting all pairs: every unlocked a of A forms its best gain
// from its unlocked neighbours in B (with their multiplicities) and from the
// largest D among the B vertices it does not touch, read off a histogram of the
// unlocked B vertices' D (a value d is free for a when more B vertices have
// D = d than a has neighbours there); one packed 64-bit maximum gives
// the best gain with the smallest a, one minimum the smallest b reaching it.
// After the steps, the smallest j of largest prefix gain G(j) is found by a
// block scan; if G(j) > 0 the first j pairs change sides, else the bisection
// is done.
#include "vmo_internal.h"

namespace vmo {

constexpr int kKT = 1024;
constexpr int kKlMaxDeg = 1024;    // histogram of D in [-maxdeg, maxdeg] in LDS
constexpr int kKlLdsMax = 9216;    // bisections up to this size keep D and the flags in LDS

__device__ __forceinline__ int32_t kl_other(const int32_t* pins, int32_t e, int32_t v) {
  return pins[2 * e] + pins[2 * e + 1] - v;
}

// D and the flags (bit 0: side B, bit 1: locked) of the members of one
// bisection, by member index (ascending vertex id).  Kept in LDS, or for
// larger bisections in device memory, where D changes by atomic adds that the
// CU's L1 cache does not see, so its reads go to L2.
template <bool kLds>
__device__ __forceinline__ int32_t rdD(const int32_t* p) {
  if constexpr (kLds) return *p;
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool kLds>
__global__ __launch_bounds__(kKT) void k_kl(const int64_t* __restrict__ lptr, const int32_t* __restrict__ ladj,
                                            const int32_t* __restrict__ lmul, const int32_t* __restrict__ gbeg, const int32_t* __restrict__ mem,
                                            int32_t* __restrict__ label, int32_t* __restrict__ Dg,
                                            uint8_t* __restrict__ Fg, int32_t* __restrict__ pa,
                                            int32_t* __restrict__ pb, int32_t* __restrict__ pg, int32_t passes,
                                            int32_t maxdeg, long long* __restrict__ gain) {
  const int32_t g = blockIdx.x, t = threadIdx.x;
  const int32_t m0 = gbeg[g], n = gbeg[g + 1] - m0;
  extern __shared__ __align__(16) unsigned char dyn[];
  int32_t* D = kLds ? reinterpret_cast<int32_t*>(dyn) : Dg + m0;
  uint8_t* F = kLds ? dyn + 4 * (size_t)n : Fg + m0;
  const int64_t* lp = lptr + m0;
  __shared__ int32_t hist[2 * kKlMaxDeg + 1];
  __shared__ int32_t sh_n, sh_dmax, sh_b;
  __shared__ unsigned long long sh_best;
  __shared__ long long sh_scan[kKT];
  __shared__ unsigned long long sh_pre;
  __shared__ int32_t sh_stop;
  const int H = 2 * maxdeg + 1;

  if (t == 0) sh_n = 0;
  __syncthreads();
  {
    int nb = 0;
    for (int32_t j = t; j < n; j += kKT) {
      const uint8_t side = (uint8_t)(label[mem[m0 + j]] & 1);
      F[j] = side;
      nb += side;
    }
    if (nb) atomicAdd(&sh_n, nb);
  }
  __syncthreads();
  const int32_t steps = min(sh_n, n - sh_n);
  long long total = 0;
  for (int32_t pass = 0; pass < passes && steps > 0; ++pass) {
    // D from the current sides; everything unlocked
    for (int32_t j = t; j < n; j += kKT) {
      const int32_t sj = F[j] & 1;
      int32_t d = 0;
      for (int64_t p = lp[j]; p < lp[j + 1]; ++p) d += (F[ladj[p]] & 1) != sj ? lmul[p] : -lmul[p];
      D[j] = d;
      F[j] = (uint8_t)sj;
    }
    __syncthreads();
    int32_t nst = steps;
    for (int32_t st = 0; st < steps; ++st) {
      // histogram of D over the unlocked B members, and its largest value
      for (int i = t; i < H; i += kKT) hist[i] = 0;
      if (t == 0) {
        sh_dmax = -kKlMaxDeg - 1;
        sh_best = 0ull;
        sh_b = INT32_MAX;
      }
      __syncthreads();
      {
        int dm = -kKlMaxDeg - 1;
        for (int32_t j = t; j < n; j += kKT) {
          if (F[j] != 1) continue;  // side B, unlocked
          const int32_t d = rdD<kLds>(&D[j]);
          atomicAdd(&hist[d + maxdeg], 1);
          dm = max(dm, d);
        }
        for (int off = 32; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off, 64));
        if ((t & 63) == 0) atomicMax(&sh_dmax, dm);
      }
      __syncthreads();
      const int32_t dmax = sh_dmax;
      // every unlocked a of A: its best gain
      for (int32_t a = t; a < n; a += kKT) {
        if (F[a] != 0) continue;  // side A, unlocked
        const int32_t Da = rdD<kLds>(&D[a]);
        const int64_t p0 = lp[a], p1 = lp[a + 1];
        int32_t best = INT32_MIN;
        // neighbours in B (distinct, with their multiplicities)
        for (int64_t p = p0; p < p1; ++p) {
          const int32_t b = ladj[p];
          if (F[b] != 1) continue;
          best = max(best, Da + rdD<kLds>(&D[b]) - 2 * lmul[p]);
        }
        // the largest D among the B members a does not touch
        for (int32_t d = dmax; d >= -maxdeg; --d) {
          const int32_t c = hist[d + maxdeg];
          if (c == 0) continue;
          int32_t nb = 0;  // unlocked neighbours in B with D = d
          for (int64_t p = p0; p < p1; ++p) {
            const int32_t b = ladj[p];
            nb += F[b] == 1 && rdD<kLds>(&D[b]) == d;
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
      if (bk == 0ull) {  // unreachable while both sides have unlocked members
        nst = st;
        break;
      }
      const int32_t gstar = (int32_t)(bk >> 32) - (1 << 30);
      const int32_t astar = 0x7fffffff - (int32_t)(bk & 0xffffffffull);
      const int32_t Das = rdD<kLds>(&D[astar]);
      const int64_t q0 = lp[astar], q1 = lp[astar + 1];
      // the smallest b reaching the gain: among the neighbours of a* ...
      for (int64_t p = q0 + t; p < q1; p += kKT) {
        const int32_t b = ladj[p];
        if (F[b] == 1 && Das + rdD<kLds>(&D[b]) - 2 * lmul[p] == gstar) atomicMin(&sh_b, b);
      }
      // ... and among the B members a* does not touch
      const int32_t want = gstar - Das;
      for (int32_t b = t; b < n; b += kKT) {
        if (F[b] != 1 || rdD<kLds>(&D[b]) != want) continue;
        bool adj = false;
        for (int64_t q = q0; q < q1; ++q)
          if (ladj[q] == b) { adj = true; break; }
        if (!adj) atomicMin(&sh_b, b);
      }
      __syncthreads();
      const int32_t bstar = sh_b;
      if (bstar == INT32_MAX) {  // unreachable: the best gain has a partner
        nst = st;
        break;
      }
      if (t == 0) {
        F[astar] |= 2;
        F[bstar] |= 2;
        pa[m0 + st] = astar;
        pb[m0 + st] = bstar;
        pg[m0 + st] = gstar;
      }
      __syncthreads();
      // D of the unlocked members as if a* and b* swapped
      {
        const int64_t na = q1 - q0, r0 = lp[bstar], nbb = lp[bstar + 1] - r0;
        for (int64_t p = t; p < na + nbb; p += kKT) {
          const int32_t x = p < na ? astar : bstar;
          const int64_t pp = p < na ? q0 + p : r0 + (p - na);
          const int32_t w = ladj[pp];
          const uint8_t fw = F[w];
          if (fw & 2) continue;
          atomicAdd(&D[w], (fw & 1) == (F[x] & 1) ? 2 * lmul[pp] : -2 * lmul[pp]);
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
      F[pa[m0 + s]] ^= 1;
      F[pb[m0 + s]] ^= 1;
    }
    total += bestG;
    __syncthreads();
  }
  __syncthreads();
  for (int32_t j = t; j < n; j += kKT) label[mem[m0 + j]] = 2 * g + (F[j] & 1);
  if (t == 0 && gain) gain[g] = total;
}

// Local adjacency of the members: for member position i (vertex mem[i] of
// bisection g), the member indices within g of its distinct neighbours in g
// (in the order of their first edge) with the number of edges to each.
__global__ void k_kl_midx(const int32_t* mem, const int32_t* label, const int32_t* gbeg, int32_t K, int32_t* midx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = mem[i];
    midx[v] = (int32_t)i - gbeg[label[v] >> 1];
  }
}
// true if edge p of v is the first edge of v to its other end w
__device__ __forceinline__ bool kl_first(const int64_t* dptr, const int32_t* dnets, const int32_t* pins, int32_t v,
                                         int64_t p, int32_t w) {
  for (int64_t q = dptr[v]; q < p; ++q)
    if (kl_other(pins, dnets[q], v) == w) return false;
  return true;
}
__global__ void k_kl_lcount(const int64_t* dptr, const int32_t* dnets, const int32_t* pins, const int32_t* mem,
                            const int32_t* label, int32_t K, int64_t* lcnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = mem[i], lv = label[v] >> 1;
    int64_t c = 0;
    for (int64_t p = dptr[v]; p < dptr[v + 1]; ++p) {
      const int32_t w = kl_other(pins, dnets[p], v);
      if (label[w] >= 0 && (label[w] >> 1) == lv) c += kl_first(dptr, dnets, pins, v, p, w);
    }
    lcnt[i] = c;
  }
}
__global__ void k_kl_lfill(const int64_t* dptr, const int32_t* dnets, const int32_t* pins, const int32_t* mem,
                           const int32_t* label, const int32_t* midx, const int64_t* lptr, int32_t K,
                           int32_t* ladj, int32_t* lmul) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = mem[i], lv = label[v] >> 1;
    int64_t o = lptr[i];
    for (int64_t p = dptr[v]; p < dptr[v + 1]; ++p) {
      const int32_t w = kl_other(pins, dnets[p], v);
      if (label[w] < 0 || (label[w] >> 1) != lv || !kl_first(dptr, dnets, pins, v, p, w)) continue;
      int32_t mult = 0;
      for (int64_t q = p; q < dptr[v + 1]; ++q) mult += kl_other(pins, dnets[q], v) == w;
      ladj[o] = midx[w];
      lmul[o] = mult;
      ++o;
    }
  }
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
  VMO_REQUIRE(G <= k, "bisection indices must be below k (labels below 2k)");
  if (ngroups) *ngroups = G;
  if (G == 0 || passes == 0) {
    if (gain && G > 0) fill_i64(gain, 0, G, s);
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
  const int32_t K = read1(gbeg.p + G, s);  // labelled vertices (members of some bisection)
  std::vector<int32_t> hb(G + 1);
  VMO_HIP(hipMemcpyAsync(hb.data(), gbeg.p, sizeof(int32_t) * (G + 1), hipMemcpyDeviceToHost, s));
  Buf<int32_t> midx(c.pool, k);
  Buf<int64_t> lptr(c.pool, (int64_t)K + 1);
  VMO_LAUNCH(k_kl_midx, ksz(K), 256, 0, s, mem.p, label, gbeg.p, K, midx.p);
  VMO_LAUNCH(k_kl_lcount, ksz(K), 256, 0, s, dptr.p, dnets.p, h->pins, mem.p, label, K, lptr.p);
  scan_exclusive<int64_t>(c, lptr.p, lptr.p, K, lptr.p + K, s);
  const int64_t nadj = read1(lptr.p + K, s);
  Buf<int32_t> ladj(c.pool, nadj > 0 ? nadj : 1), lmul(c.pool, nadj > 0 ? nadj : 1);
  VMO_LAUNCH(k_kl_lfill, ksz(K), 256, 0, s, dptr.p, dnets.p, h->pins, mem.p, label, midx.p, lptr.p, K, ladj.p,
             lmul.p);
  int32_t nmax = 0;
  for (int32_t g = 0; g < G; ++g) nmax = std::max(nmax, hb[g + 1] - hb[g]);
  Buf<int32_t> D(c.pool, K > 0 ? K : 1), pa(c.pool, K > 0 ? K : 1), pb(c.pool, K > 0 ? K : 1),
      pg(c.pool, K > 0 ? K : 1);
  Buf<uint8_t> F(c.pool, K > 0 ? K : 1);
  Buf<long long> gl(c.pool, G);
  if (nmax <= kKlLdsMax) {
    const size_t lds = ((5 * (size_t)nmax + 15) / 16) * 16;
    VMO_LAUNCH((k_kl<true>), (unsigned)G, kKT, lds, s, lptr.p, ladj.p, lmul.p, gbeg.p, mem.p, label, D.p, F.p, pa.p, pb.p,
               pg.p, passes, maxdeg, gl.p);
  } else {
    VMO_LAUNCH((k_kl<false>), (unsigned)G, kKT, 0, s, lptr.p, ladj.p, lmul.p, gbeg.p, mem.p, label, D.p, F.p, pa.p, pb.p,
               pg.p, passes, maxdeg, gl.p);
  }
  if (gain) VMO_HIP(hipMemcpyAsync(gain, gl.p, sizeof(int64_t) * G, hipMemcpyDeviceToDevice, s));
}

}  // namespace vmo
