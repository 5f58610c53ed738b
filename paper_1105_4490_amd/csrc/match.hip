// Strengthened diagonal (Sec. 4.2: a perfect matching of the bipartite graph
// kept intact by Algorithm 7; Sec. 5: a heavy edge matching augmented to a
// perfect matching), the row and column permutations it gives, and finegrain
// coordinates (Sec. 4.2: every nonzero at the average of the points of its
// row and its column).
//
// Heavy edge matching.  Nonzero e = (i, j) has the priority
// key(e) = bits(|a_e|) << 32 | fmix32(e + seed), fmix32 being the 32-bit
// finalizer of MurmurHash3 (a bijection), so no two nonzeros tie and the
// greedy matching of this order (visit by decreasing key, take an edge whose
// ends are free) is unique.  It is computed by locally dominant rounds: every
// free row and every free column marks its heaviest edge to a free partner
// (64-bit atomic max), and an edge marked by both ends is taken.  The heaviest
// edge among free vertices is always taken, and an edge taken in a round is
// the heaviest of both its ends among the edges still free, which is exactly
// when the sequential greedy takes it: the result is the greedy matching.
//
// Augmentation to a maximum matching.  Each phase grows a breadth-first forest
// of alternating paths from all free rows at once, level by level: a column
// reached from several rows of the frontier goes to the smallest row id, the
// matched row of a reached column joins the next frontier in the same tree,
// and a tree that reaches a free column stops growing (its claim is the
// smallest free column found at the first level it found one).  Every claimed
// tree then flips the path from its claimed column to its root; trees are
// vertex-disjoint, so the flips do not interfere.  Phases repeat until one
// claims nothing: then no augmenting path exists and the matching is maximum.
// All choices are minima over sets, so the result does not depend on thread
// timing.
#include "order_engine.h"

namespace vmo {

constexpr int kHT = 256;

static unsigned hsz(int64_t n) {
  int64_t b = (n + kHT - 1) / kHT;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}
#define HM_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}
__device__ __forceinline__ uint64_t match_key(const float* a, int64_t e, uint32_t seed) {
  const float w = a ? fabsf(a[e]) : 1.0f;
  return ((uint64_t)__float_as_uint(w) << 32) | fmix32((uint32_t)e + seed);
}

// Row of every nonzero (binary search over rowptr).
__global__ void k_rowid(const int64_t* rowptr, int32_t m, int64_t nnz, int32_t* rowid) {
  HM_STRIDE(e, nnz) {
    int32_t lo = 0, hi = m;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (rowptr[mid] <= e) lo = mid; else hi = mid;
    }
    rowid[e] = lo;
  }
}

__global__ void k_hm_propose(const int32_t* rowid, const int32_t* col, const float* a, uint32_t seed, int64_t nnz,
                             const int32_t* mrow, const int32_t* mcol, unsigned long long* rbest,
                             unsigned long long* cbest) {
  HM_STRIDE(e, nnz) {
    const int32_t i = rowid[e], j = col[e];
    if (mrow[i] >= 0 || mcol[j] >= 0) continue;
    const unsigned long long key = match_key(a, e, seed);
    atomicMax(&rbest[i], key);
    atomicMax(&cbest[j], key);
  }
}
// An edge marked by both ends is taken; only that edge can match its row and
// its column in this round (keys are unique).
__global__ void k_hm_accept(const int32_t* rowid, const int32_t* col, const float* a, uint32_t seed, int64_t nnz,
                            int32_t* mrow, int32_t* mcol, const unsigned long long* rbest,
                            const unsigned long long* cbest, int32_t* taken) {
  HM_STRIDE(e, nnz) {
    const int32_t i = rowid[e], j = col[e];
    if (mrow[i] >= 0 || mcol[j] >= 0) continue;
    const unsigned long long key = match_key(a, e, seed);
    if (rbest[i] == key && cbest[j] == key) {
      mrow[i] = j;
      mcol[j] = i;
      atomicAdd(taken, 1);
    }
  }
}

// Phase start: roots are the free rows, which form the first frontier.
__global__ void k_aug_init(const int32_t* mrow, int32_t m, int32_t* root, unsigned long long* claim, int32_t* front,
                           int32_t* fcount) {
  HM_STRIDE(i, m) {
    claim[i] = ~0ull;
    if (mrow[i] < 0) {
      root[i] = (int32_t)i;
      front[atomicAdd(fcount, 1)] = (int32_t)i;
    } else {
      root[i] = -1;
    }
  }
}
// A frontier row is skipped once its tree claimed a free column at an earlier
// level (claims of this level carry this level in their upper word).
__device__ __forceinline__ bool aug_skip(const unsigned long long* claim, int32_t r, int32_t level) {
  return (int64_t)(claim[r] >> 32) < (int64_t)level;
}
__global__ void k_aug_cand(const int32_t* front, int32_t F, int32_t level, const int32_t* root,
                           const unsigned long long* claim, const int64_t* rowptr, const int32_t* col,
                           const int32_t* cvis, int32_t* cand) {
  HM_STRIDE(t, F) {
    const int32_t u = front[t];
    if (aug_skip(claim, root[u], level)) continue;
    for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) {
      const int32_t j = col[p];
      if (cvis[j] < 0) atomicMin(&cand[j], u);
    }
  }
}
__global__ void k_aug_visit(const int32_t* front, int32_t F, int32_t level, int32_t* root, unsigned long long* claim,
                            const int64_t* rowptr, const int32_t* col, int32_t* cvis, const int32_t* cand,
                            const int32_t* mcol, int32_t* next, int32_t* ncount) {
  HM_STRIDE(t, F) {
    const int32_t u = front[t];
    const int32_t r = root[u];
    if (aug_skip(claim, r, level)) continue;
    for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) {
      const int32_t j = col[p];
      if (cvis[j] >= 0 || cand[j] != u) continue;
      cvis[j] = u;
      const int32_t r2 = mcol[j];
      if (r2 < 0) {
        atomicMin(&claim[r], ((unsigned long long)(uint32_t)level << 32) | (uint32_t)j);
      } else {
        root[r2] = r;
        next[atomicAdd(ncount, 1)] = r2;
      }
    }
  }
}
// Flip the augmenting path of every claimed tree (one thread per root).
__global__ void k_aug_flip(int32_t m, const unsigned long long* claim, const int32_t* cvis, int32_t levels,
                           int32_t* mrow, int32_t* mcol, int32_t* flipped) {
  HM_STRIDE(i, m) {
    if (mrow[i] >= 0 || claim[i] == ~0ull) continue;
    int32_t j = (int32_t)(claim[i] & 0xffffffffull);
    for (int32_t step = 0; step <= levels; ++step) {
      const int32_t u = cvis[j];
      if (u < 0) break;  // unreachable: every column on a tree path was visited
      const int32_t nj = mrow[u];
      mrow[u] = j;
      mcol[j] = u;
      if (u == (int32_t)i) break;
      j = nj;
    }
    atomicAdd(flipped, 1);
  }
}

__global__ void k_match_out(const int32_t* mrow, const int32_t* mcol, int32_t m, int32_t n, int32_t* mu,
                            int32_t* count) {
  HM_STRIDE(v, (int64_t)m + n) {
    int32_t w;
    if (v < m) {
      w = mrow[v] >= 0 ? m + mrow[v] : -1;
      if (mrow[v] >= 0) atomicAdd(count, 1);
    } else {
      w = mcol[v - m];
    }
    if (mu) mu[v] = w;
  }
}

void match(Ctx& c, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* a, uint32_t seed,
           int augment, int32_t* mrow, int32_t* mcol, int32_t* mu, int64_t* size_out, hipStream_t s) {
  VMO_REQUIRE(m >= 1 && n >= 1, "matrix needs m, n >= 1");
  VMO_REQUIRE((int64_t)m + n < (int64_t(1) << 31), "m + n must be below 2^31");
  VMO_REQUIRE(rowptr && mrow && mcol && size_out, "NULL argument");
  vmo_hypergraph rows{n, m, rowptr, col, nullptr, nullptr};  // rows as nets over columns
  validate_hypergraph(c, &rows, false, s);
  const int64_t nnz = read1(rowptr + m, s);
  VMO_REQUIRE(nnz < (int64_t(1) << 32), "too many nonzeros");
  if (a && nnz > 0) validate_finite(c, a, nnz, "a", s);
  fill_i32(mrow, -1, m, s);
  fill_i32(mcol, -1, n, s);
  if (nnz > 0) {
    Buf<int32_t> rowid(c.pool, nnz), taken(c.pool, 1);
    Buf<unsigned long long> rbest(c.pool, m), cbest(c.pool, n);
    VMO_LAUNCH(k_rowid, hsz(nnz), kHT, 0, s, rowptr, m, nnz, rowid.p);
    for (int64_t round = 0; round <= (int64_t)m; ++round) {  // every round takes an edge or ends
      VMO_HIP(hipMemsetAsync(rbest.p, 0, sizeof(unsigned long long) * m, s));
      VMO_HIP(hipMemsetAsync(cbest.p, 0, sizeof(unsigned long long) * n, s));
      VMO_HIP(hipMemsetAsync(taken.p, 0, sizeof(int32_t), s));
      VMO_LAUNCH(k_hm_propose, hsz(nnz), kHT, 0, s, rowid.p, col, a, seed, nnz, mrow, mcol, rbest.p, cbest.p);
      VMO_LAUNCH(k_hm_accept, hsz(nnz), kHT, 0, s, rowid.p, col, a, seed, nnz, mrow, mcol, rbest.p, cbest.p,
                 taken.p);
      if (read1(taken.p, s) == 0) break;
    }
  }
  if (augment && nnz > 0) {
    Buf<int32_t> root(c.pool, m), fa(c.pool, m), fb(c.pool, m), cvis(c.pool, n), cand(c.pool, n), cnt(c.pool, 2);
    Buf<unsigned long long> claim(c.pool, m);
    for (int64_t phase = 0; phase <= (int64_t)m; ++phase) {  // every phase augments or ends
      VMO_HIP(hipMemsetAsync(cnt.p, 0, 2 * sizeof(int32_t), s));
      VMO_LAUNCH(k_aug_init, hsz(m), kHT, 0, s, mrow, m, root.p, claim.p, fa.p, cnt.p);
      int32_t F = read1(cnt.p, s);
      if (F == 0) break;
      fill_i32(cvis.p, -1, n, s);
      fill_i32(cand.p, INT32_MAX, n, s);
      int32_t* cur = fa.p;
      int32_t* nxt = fb.p;
      int32_t level = 0;
      while (F > 0) {
        VMO_HIP(hipMemsetAsync(cnt.p + 1, 0, sizeof(int32_t), s));
        VMO_LAUNCH(k_aug_cand, hsz(F), kHT, 0, s, cur, F, level, root.p, claim.p, rowptr, col, cvis.p, cand.p);
        VMO_LAUNCH(k_aug_visit, hsz(F), kHT, 0, s, cur, F, level, root.p, claim.p, rowptr, col, cvis.p, cand.p,
                   mcol, nxt, cnt.p + 1);
        F = read1(cnt.p + 1, s);
        std::swap(cur, nxt);
        ++level;
      }
      VMO_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t), s));
      VMO_LAUNCH(k_aug_flip, hsz(m), kHT, 0, s, m, claim.p, cvis.p, level, mrow, mcol, cnt.p);
      if (read1(cnt.p, s) == 0) break;
    }
  }
  Buf<int32_t> count(c.pool, 1);
  VMO_HIP(hipMemsetAsync(count.p, 0, sizeof(int32_t), s));
  VMO_LAUNCH(k_match_out, hsz((int64_t)m + n), kHT, 0, s, mrow, mcol, m, n, mu, count.p);
  *size_out = read1(count.p, s);
}

// ------------------------------------------------- strengthened diagonal ----
// bad |= 1: mu[v] outside [-1, k), mu[v] = v, or mu[mu[v]] != v.
__global__ void k_mu_check(const int32_t* mu, int32_t k, int* bad) {
  HM_STRIDE(v, k) {
    const int32_t w = mu[v];
    if (w < -1 || w >= k || w == v) atomicOr(bad, 1);
    else if (w >= 0 && mu[w] != v) atomicOr(bad, 1);
  }
}
__global__ void k_mu_edges(const int32_t* pins, int32_t l, const int32_t* mu, int32_t* ok) {
  HM_STRIDE(e, l) {
    const int32_t a = pins[2 * e], b = pins[2 * e + 1];
    if (mu[a] == b) {
      ok[a] = 1;
      ok[b] = 1;
    }
  }
}
__global__ void k_mu_paired(const int32_t* mu, const int32_t* ok, int32_t k, int* bad) {
  HM_STRIDE(v, k) {
    if (mu[v] >= 0 && !ok[v]) atomicOr(bad, 2);
  }
}

// mu must be an involution without fixed points whose pairs are edges of the
// graph h (every net an edge, as graph mode requires).
void validate_mu(Ctx& c, const vmo_hypergraph* h, const int32_t* mu, hipStream_t s) {
  VMO_REQUIRE(mu != nullptr, "mu is NULL");
  const int32_t k = h->k, l = h->l;
  Buf<int> bad(c.pool, 1);
  Buf<int32_t> ok(c.pool, k);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  VMO_HIP(hipMemsetAsync(ok.p, 0, sizeof(int32_t) * k, s));
  VMO_LAUNCH(k_mu_check, hsz(k), kHT, 0, s, mu, k, bad.p);
  int b = read1(bad.p, s);
  VMO_REQUIRE(!(b & 1), "mu must map every vertex to -1 or to a partner w != v with mu[w] = v");
  if (l > 0) VMO_LAUNCH(k_mu_edges, hsz(l), kHT, 0, s, h->pins, l, mu, ok.p);
  VMO_LAUNCH(k_mu_paired, hsz(k), kHT, 0, s, mu, ok.p, k, bad.p);
  b = read1(bad.p, s);
  VMO_REQUIRE(!(b & 2), "every pair {v, mu[v]} must be an edge of the graph");
}

// ------------------------------------------------------------ permutations ----
__global__ void k_mp_check(const int32_t* vperm, const int32_t* mu, int32_t m, int32_t* mark, int32_t* isrow,
                           int* bad) {
  HM_STRIDE(p, 2 * (int64_t)m) {
    const int32_t v = vperm[p];
    if (v < 0 || v >= 2 * m) {
      atomicOr(bad, 1);
      isrow[p] = 0;
      continue;
    }
    atomicAdd(&mark[v], 1);
    isrow[p] = v < m;
    if (v < m && (mu[v] < m || mu[v] >= 2 * m)) atomicOr(bad, 2);
  }
}
__global__ void k_mp_marks(const int32_t* mark, int32_t m, int* bad) {
  HM_STRIDE(v, 2 * (int64_t)m) {
    if (mark[v] != 1) atomicOr(bad, 1);
  }
}
// writes nothing once the checks above failed (at[] may then exceed m)
__global__ void k_mp_write(const int32_t* vperm, const int32_t* mu, const int32_t* isrow, const int32_t* at, int32_t m,
                           int32_t* rperm, int32_t* cperm, const int* bad) {
  if (*bad) return;
  HM_STRIDE(p, 2 * (int64_t)m) {
    if (!isrow[p]) continue;
    const int32_t v = vperm[p];
    rperm[at[p]] = v;
    cperm[at[p]] = mu[v] - m;
  }
}

void matched_perms(Ctx& c, int32_t m, const int32_t* vperm, const int32_t* mu, int32_t* rperm, int32_t* cperm,
                   hipStream_t s) {
  VMO_REQUIRE(m >= 1 && m < (1 << 30), "m must be in [1, 2^30)");
  VMO_REQUIRE(vperm && mu && rperm && cperm, "NULL argument");
  const int64_t k = 2 * (int64_t)m;
  Buf<int> bad(c.pool, 1);
  Buf<int32_t> mark(c.pool, k), isrow(c.pool, k + 1), at(c.pool, k + 1);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  VMO_HIP(hipMemsetAsync(mark.p, 0, sizeof(int32_t) * k, s));
  VMO_LAUNCH(k_mp_check, hsz(k), kHT, 0, s, vperm, mu, m, mark.p, isrow.p, bad.p);
  VMO_LAUNCH(k_mp_marks, hsz(k), kHT, 0, s, mark.p, m, bad.p);
  // checked on the device: bit 1 (kAsyncPermutation) vperm is not a
  // permutation, bit 2 (kAsyncPartner) a row without a partner column; the
  // writes are then skipped and vmo_sync reports the failure
  scan_exclusive<int32_t>(c, isrow.p, at.p, k, at.p + k, s);
  VMO_LAUNCH(k_mp_write, hsz(k), kHT, 0, s, vperm, mu, isrow.p, at.p, m, rperm, cperm, bad.p);
  post_async_check(c, bad.p, s);
}

// -------------------------------------------------------------- finegrain ----
// The pattern's rows checked on the device: rowptr[0] = 0 and non-decreasing,
// columns in [0, n) and ascending within a row (else kAsyncCsr).
__global__ void k_fg_check(const int64_t* rowptr, const int32_t* col, int32_t m, int32_t n, int* bad) {
  HM_STRIDE(i, m) {
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    if ((i == 0 && b != 0) || e < b) {
      atomicOr(bad, kAsyncCsr);
      continue;
    }
    for (int64_t t = b; t < e; ++t) {
      const int32_t j = col[t];
      if (j < 0 || j >= n || (t > b && j <= col[t - 1])) {
        atomicOr(bad, kAsyncCsr);
        break;
      }
    }
  }
}
// One thread per row; nnz = rowptr[m] read on the device (no host round
// trip).  Writes nothing once the check failed.
__global__ void k_finegrain(const int64_t* rowptr, const int32_t* col, int32_t m, int32_t n, const float* x,
                            float* xnz, const int* bad) {
  if (*bad) return;
  const int64_t nnz = rowptr[m], k = (int64_t)m + n;
  HM_STRIDE(i, m) {
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int64_t jc = (int64_t)m + col[e];
      for (int d = 0; d < 4; ++d) xnz[d * nnz + e] = (x[d * k + i] + x[d * k + jc]) * 0.5f;
    }
  }
}

void finegrain(Ctx& c, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* x, float* xnz,
               hipStream_t s) {
  VMO_REQUIRE(m >= 1 && n >= 1, "matrix needs m, n >= 1");
  VMO_REQUIRE((int64_t)m + n < (int64_t(1) << 31), "m + n must be below 2^31");
  VMO_REQUIRE(rowptr && x && xnz, "NULL argument");
  Buf<int> bad(c.pool, 1);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  VMO_LAUNCH(k_fg_check, hsz(m), kHT, 0, s, rowptr, col, m, n, bad.p);
  VMO_LAUNCH(k_finegrain, hsz(m), kHT, 0, s, rowptr, col, m, n, x, xnz, bad.p);
  post_async_check(c, bad.p, s);
}

}  // namespace vmo
