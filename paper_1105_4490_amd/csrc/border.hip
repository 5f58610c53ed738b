// Recursive ordering of the border (Sec. 4.2: the freedom left in the cut
// rows and columns of a recursive BBD ordering, used to bring them into
// recursive BBD form as in the rightmost partitioning of the figure on matrix
// partitionings).  Every vertex w of the separator of a node h (heap id, depth
// d) gets b two-bit words, the first the most significant: word i collects,
// over the edges {v, w} with v below h, bit 1 when v lies in the first part
// (heap 2g) and bit 2 when it lies in the second part (2g + 1) of the split
// of its ancestor g at depth d + i.  Each separator block is then sorted by
// the words, stably.  The words are ORs of per-edge bits (atomic OR, any
// order), and the blocks are sorted by one stable radix sort over (block
// rank, words).
#include "vmo_internal.h"

namespace vmo {

constexpr int kBT = 256;

static unsigned bsz(int64_t n) {
  int64_t b = (n + kBT - 1) / kBT;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}
#define BD_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ int heap_depth(int32_t h) { return 31 - __clz(h); }

// Consistency of an ordering result (bad = 1 on any violation): heap ids in
// [1, 4P), block boundaries non-decreasing from 0 to k, part ids leaf parts
// [0, P) or P + a heap id, vperm a permutation (mark counts each vertex).
__global__ void k_bd_check_nodes(const int32_t* node_heap, const int32_t* node_vptr, int32_t nn, int32_t k,
                                 int32_t P, int* bad) {
  BD_STRIDE(r, nn) {
    const int32_t h = node_heap[r];
    if (h < 1 || h >= 4 * P) atomicExch(bad, 1);
    if (node_vptr[r] > node_vptr[r + 1]) atomicExch(bad, 1);
    if (r == 0 && node_vptr[0] != 0) atomicExch(bad, 1);
    if (r == nn - 1 && node_vptr[nn] != k) atomicExch(bad, 1);
  }
}
__global__ void k_bd_check_verts(const int32_t* vperm, const int32_t* part, int32_t k, int32_t P, int32_t* mark,
                                 int* bad) {
  BD_STRIDE(i, k) {
    const int32_t p = part[i];
    if (p < 0 || (p >= P && (p - P < 1 || p - P >= 4 * P))) atomicExch(bad, 1);
    const int32_t v = vperm[i];
    if (v < 0 || v >= k) atomicExch(bad, 1);
    else atomicAdd(&mark[v], 1);
  }
}
__global__ void k_bd_check_marks(const int32_t* mark, int32_t k, int* bad) {
  BD_STRIDE(v, k) {
    if (mark[v] != 1) atomicExch(bad, 1);
  }
}

// leaf_heap[p] = heap id of the leaf block holding part p (its first vertex
// names the part); parts that own no vertex keep the root.
__global__ void k_bd_leaf(const int32_t* vperm, const int32_t* part, const int32_t* node_heap,
                          const int32_t* node_vptr, int32_t nn, int32_t P, int32_t* leaf_heap) {
  BD_STRIDE(r, nn) {
    if (node_vptr[r] == node_vptr[r + 1]) continue;
    const int32_t p = part[vperm[node_vptr[r]]];
    if (p < P) leaf_heap[p] = node_heap[r];
  }
}

// The node each vertex ends in: a separator's heap id, or its leaf's.
__global__ void k_bd_vheap(const int32_t* part, int32_t k, int32_t P, const int32_t* leaf_heap, int32_t* vh) {
  BD_STRIDE(v, k) {
    const int32_t p = part[v];
    vh[v] = p >= P ? p - P : leaf_heap[p];
  }
}

// The words: edge {v, w} as seen from each end that is a separator vertex.
__global__ void k_bd_words(const int64_t* ptr, const int32_t* pins, int32_t l, const int32_t* part,
                           const int32_t* vh, int32_t P, int32_t b, uint32_t* word) {
  BD_STRIDE(e, l) {
    const int64_t p0 = ptr[e];
    for (int s = 0; s < 2; ++s) {
      const int32_t w = pins[p0 + s], v = pins[p0 + 1 - s];
      if (part[w] < P) continue;
      const int32_t h = vh[w], hv = vh[v];
      const int d = heap_depth(h), D = heap_depth(hv);
      if (D <= d || (hv >> (D - d)) != h) continue;  // v is not below h
      uint32_t bits = 0;
      for (int i = 1; i <= b && D >= d + i + 1; ++i) {
        const int second = (hv >> (D - d - i - 1)) & 1;
        bits |= (uint32_t)(second ? 2 : 1) << (2 * (b - i));
      }
      if (bits) atomicOr(&word[w], bits);
    }
  }
}

// Sort keys: (rank of the block holding position i) << 2b | words of its vertex.
__global__ void k_bd_keys(const int32_t* vperm, const int32_t* node_vptr, int32_t nn, int32_t k,
                          const uint32_t* word, int32_t b, uint64_t* key, int32_t* val) {
  BD_STRIDE(i, k) {
    int32_t lo = 0, hi = nn;  // the last r with node_vptr[r] <= i
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (node_vptr[mid] <= i) lo = mid; else hi = mid;
    }
    const int32_t v = vperm[i];
    key[i] = ((uint64_t)lo << (2 * b)) | (uint64_t)word[v];
    val[i] = v;
  }
}

int32_t check_ordering(Ctx& c, int32_t k, int32_t P, const vmo_order_out* in, hipStream_t s) {
  VMO_REQUIRE(in != nullptr, "in is NULL");
  VMO_REQUIRE(in->vperm && in->part && in->node_heap && in->node_vptr && in->n_nodes, "NULL ordering array");
  VMO_REQUIRE(P >= 1, "P must be >= 1");
  VMO_REQUIRE(k >= 1, "k must be >= 1");
  const int32_t nn = read1(in->n_nodes, s);
  VMO_REQUIRE(nn >= 1 && nn <= 4 * P, "n_nodes must be in [1, 4P]");
  Buf<int> bad(c.pool, 1);
  Buf<int32_t> mark(c.pool, k);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  VMO_HIP(hipMemsetAsync(mark.p, 0, sizeof(int32_t) * k, s));
  VMO_LAUNCH(k_bd_check_nodes, bsz(nn), kBT, 0, s, in->node_heap, in->node_vptr, nn, k, P, bad.p);
  VMO_LAUNCH(k_bd_check_verts, bsz(k), kBT, 0, s, in->vperm, in->part, k, P, mark.p, bad.p);
  VMO_LAUNCH(k_bd_check_marks, bsz(k), kBT, 0, s, mark.p, k, bad.p);
  VMO_REQUIRE(read1(bad.p, s) == 0, "the ordering arrays are inconsistent (vperm, part, node_heap, node_vptr)");
  return nn;
}

void order_border(Ctx& c, const vmo_hypergraph* h, const vmo_order_out* in, int32_t P, int32_t b, int32_t* vperm_out,
                  hipStream_t s) {
  VMO_REQUIRE(vperm_out != nullptr, "vperm_out is NULL");
  VMO_REQUIRE(b >= 0 && b <= 15, "b must be in [0, 15]");
  std::vector<int64_t> npins;
  validate_jobs(c, {JobCheck{h, nullptr, false, true}}, npins, s);
  const int32_t k = h->k, l = h->l;
  const int32_t nn = check_ordering(c, k, P, in, s);
  if (b == 0) {
    VMO_HIP(hipMemcpyAsync(vperm_out, in->vperm, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, s));
    return;
  }
  Buf<int32_t> leaf_heap(c.pool, P), vh(c.pool, k);
  Buf<uint32_t> word(c.pool, k);
  fill_i32(leaf_heap.p, 1, P, s);
  VMO_HIP(hipMemsetAsync(word.p, 0, sizeof(uint32_t) * k, s));
  VMO_LAUNCH(k_bd_leaf, bsz(nn), kBT, 0, s, in->vperm, in->part, in->node_heap, in->node_vptr, nn, P, leaf_heap.p);
  VMO_LAUNCH(k_bd_vheap, bsz(k), kBT, 0, s, in->part, k, P, leaf_heap.p, vh.p);
  if (l > 0) VMO_LAUNCH(k_bd_words, bsz(l), kBT, 0, s, h->net_ptr, h->pins, l, in->part, vh.p, P, b, word.p);
  Buf<uint64_t> key(c.pool, k);
  Buf<int32_t> val(c.pool, k);
  VMO_LAUNCH(k_bd_keys, bsz(k), kBT, 0, s, in->vperm, in->node_vptr, nn, k, word.p, b, key.p, val.p);
  radix_sort<uint64_t>(c, key.p, val.p, k, 2 * b + bits_for((uint64_t)(nn - 1)), s);
  VMO_HIP(hipMemcpyAsync(vperm_out, val.p, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, s));
}

}  // namespace vmo
