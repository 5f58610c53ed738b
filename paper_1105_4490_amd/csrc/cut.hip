// Cut metrics of a partition (Sec. 4.1 cut rows/columns; the cut-net metric of
// its footnote; Table 4's maximum cut per split): per-net counts of distinct
// part ids, deterministic FP64 sums, part weights; and the allocation-free
// variant of the call, whose workspace is a static device arena.
#include "vmo_internal.h"

namespace vmo {

constexpr int kCT = 256;
constexpr int kSmallNet = 64;

// first position in the ascending a[0..n) holding a value >= x
__device__ __forceinline__ int32_t lower_bound_u32(const uint32_t* a, int32_t n, uint32_t x) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// lambda(e) for nets of at most 64 pins: a pin counts if its part id does not
// occur at an earlier pin of the net.  Larger nets are flagged for the sort path.
__global__ void k_lambda_small(const int64_t* ptr, const int32_t* pins, int32_t l, const int32_t* part,
                               int32_t* lam, int32_t* big) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = ptr[e], n = ptr[e + 1] - b;
    if (n > kSmallNet) { lam[e] = 0; big[e] = 1; continue; }
    big[e] = 0;
    int32_t pv[kSmallNet];
    int32_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
      int32_t p = part[pins[b + i]];
      bool seen = false;
      for (int64_t j = 0; j < i; ++j) seen |= (pv[j] == p);
      pv[i] = p;
      cnt += seen ? 0 : 1;
    }
    lam[e] = cnt;
  }
}

// Large nets: one key (net rank, part id) per pin.
__global__ void k_big_keys(const int64_t* ptr, const int32_t* pins, const int32_t* big, const int32_t* bigrank,
                           const int64_t* bigpin, int32_t l, const int32_t* part, uint64_t* keys) {
  for (int64_t e = blockIdx.x; e < l; e += gridDim.x) {
    if (!big[e]) continue;
    int64_t b = ptr[e], n = ptr[e + 1] - b, o = bigpin[bigrank[e]];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
      keys[o + i] = ((uint64_t)(uint32_t)bigrank[e] << 32) | (uint32_t)part[pins[b + i]];
  }
}
__global__ void k_big_count(const uint64_t* keys, int64_t n, const int32_t* bignet, int32_t* lam) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (i == 0 || keys[i] != keys[i - 1]) atomicAdd(&lam[bignet[keys[i] >> 32]], 1);
}
__global__ void k_big_list(const int32_t* big, const int32_t* bigrank, int32_t l, const int64_t* ptr,
                           int32_t* bignet, int64_t* biglen) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x)
    if (big[e]) { bignet[bigrank[e]] = (int32_t)e; biglen[bigrank[e]] = ptr[e + 1] - ptr[e]; }
}

// Per-block partial sums in a fixed order (deterministic), three metrics.
__global__ __launch_bounds__(kCT) void k_cut_partial(const int32_t* lam, const float* c, int32_t l, double* part3) {
  __shared__ double sh[3][kCT];
  int t = threadIdx.x;
  double a = 0, b = 0, n = 0;
  for (int64_t e = (int64_t)blockIdx.x * kCT + t; e < l; e += (int64_t)gridDim.x * kCT) {
    int32_t L = lam[e];
    double ce = c ? (double)c[e] : 1.0;
    if (L > 1) { a += ce * (double)(L - 1); b += ce; n += 1.0; }
  }
  sh[0][t] = a; sh[1][t] = b; sh[2][t] = n;
  __syncthreads();
  for (int off = kCT / 2; off > 0; off >>= 1) {
    if (t < off) for (int f = 0; f < 3; ++f) sh[f][t] += sh[f][t + off];
    __syncthreads();
  }
  if (t == 0) for (int f = 0; f < 3; ++f) part3[blockIdx.x * 3 + f] = sh[f][0];
}
__global__ void k_cut_final(const double* part3, int nb, double* out3) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0, b = 0, n = 0;
  for (int i = 0; i < nb; ++i) { a += part3[3 * i]; b += part3[3 * i + 1]; n += part3[3 * i + 2]; }
  out3[0] = a; out3[1] = b; out3[2] = n;
}
// Unit weights: part sizes (integer counts, exact in FP64 in any order).
__global__ void k_part_count(const int32_t* part, int32_t k, int32_t nparts, double* pw) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t p = part[v];
    if (p >= 0 && p < nparts) atomicAdd(&pw[p], 1.0);
  }
}
// Weighted parts, summed in a fixed order: the vertices grouped by part with
// a stable sort of their part ids (so each group ascends by vertex id; ids
// outside [0, nparts) sort last), then each part's weights added one by one
// in FP64.
__global__ void k_pw_keys(const int32_t* part, int32_t k, int32_t nparts, uint32_t* key, int32_t* val) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = part[v];
    key[v] = (p >= 0 && p < nparts) ? (uint32_t)p : (uint32_t)nparts;
    val[v] = (int32_t)v;
  }
}
__global__ void k_pw_sum(const uint32_t* key, const int32_t* val, int32_t k, int32_t nparts, const float* w,
                         double* pw) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nparts; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = lower_bound_u32(key, k, (uint32_t)p), e = lower_bound_u32(key, k, (uint32_t)p + 1u);
    double a = 0.0;
    for (int32_t i = b; i < e; ++i) a = a + (double)w[val[i]];
    pw[p] = a;
  }
}

// bit 1: an id outside [0, 2^30); bit 2: an id >= nparts (separator ids)
__global__ void k_check_part(const int32_t* part, int32_t k, int32_t nparts, int* bad) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    if (part[v] < 0 || part[v] >= (1 << 30)) atomicOr(bad, 1);
    else if (part[v] >= nparts) atomicOr(bad, 2);
  }
}

// ------------------------------------------------------ per-split cut ----
// Node h (heap numbering, root 1) of a recursive bisection into P parts holds
// a contiguous part range: the root [0, P), child 2h the first ceil(K/2) of
// its K parts, child 2h + 1 the rest.  A cut net whose parts all lie below P
// is cut at the deepest node holding its smallest and its largest part.
__device__ __forceinline__ int32_t node_of_range(int32_t P, int32_t lo, int32_t hi) {
  int32_t h = 1, p0 = 0, K = P;
  while (K > 1) {
    const int32_t K1 = (K + 1) >> 1;
    if (hi < p0 + K1) { h = 2 * h; K = K1; }
    else if (lo >= p0 + K1) { h = 2 * h + 1; p0 += K1; K -= K1; }
    else break;
  }
  return h;
}
// key[e] = the node cutting net e, or 4P if it is not cut (or meets an id >= P)
__global__ void k_net_split(const int64_t* ptr, const int32_t* pins, int32_t l, const int32_t* part, const int32_t* lam,
                            int32_t P, uint32_t* key, int32_t* val) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
    uint32_t node = 4u * (uint32_t)P;
    if (lam[e] > 1) {
      int32_t lo = 0x7fffffff, hi = -1;
      for (int64_t p = ptr[e]; p < ptr[e + 1]; ++p) {
        const int32_t q = part[pins[p]];
        lo = min(lo, q);
        hi = max(hi, q);
      }
      if (hi < P) node = (uint32_t)node_of_range(P, lo, hi);
    }
    key[e] = node;
    val[e] = (int32_t)e;
  }
}
// split[h] = costs of the nets cut at h, one by one in ascending net id
__global__ __launch_bounds__(kCT) void k_split_sum(const uint32_t* key, const int32_t* val, int32_t l, int32_t P,
                                                   const float* c, double* split) {
  // one wavefront per node h: its nets are [lower_bound(h), lower_bound(h + 1))
  __shared__ __align__(16) float stage[kCT / 64][64];
  const int wv = threadIdx.x >> 6;
  for (int64_t h = (int64_t)blockIdx.x * (kCT / 64) + wv; h < 4 * (int64_t)P; h += (int64_t)gridDim.x * (kCT / 64)) {
    const int32_t b = lower_bound_u32(key, l, (uint32_t)h), e = lower_bound_u32(key, l, (uint32_t)h + 1u);
    const double a = wave_ordered_cost_sum(c, val, b, e, stage[wv]);
    if ((threadIdx.x & 63) == 0) split[h] = a;
  }
}
// graph mode: split[h] = |S_h|, the vertices with part id P + h
__global__ void k_sep_count(const int32_t* part, int32_t k, int32_t P, double* split) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t h = (int64_t)part[v] - P;
    if (h >= 1 && h < 4 * (int64_t)P) atomicAdd(&split[h], 1.0);
  }
}
// out[0] = max_h split[h], out[1] = the smallest such h (0: all zero); one block
__global__ __launch_bounds__(kCT) void k_split_max(const double* split, int32_t n, double* out) {
  __shared__ double sv[kCT];
  __shared__ int32_t sh[kCT];
  double bv = 0.0;
  int32_t bh = 0x7fffffff;
  for (int32_t h = threadIdx.x; h < n; h += kCT)
    if (split[h] > bv || (split[h] == bv && bv > 0.0 && h < bh)) { bv = split[h]; bh = h; }
  sv[threadIdx.x] = bv;
  sh[threadIdx.x] = bh;
  __syncthreads();
  for (int off = kCT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double ov = sv[threadIdx.x + off];
      const int32_t oh = sh[threadIdx.x + off];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oh < sh[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        sh[threadIdx.x] = oh;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sv[0];
    out[1] = sv[0] > 0.0 ? (double)sh[0] : 0.0;
  }
}

static unsigned gsz(int64_t n) {
  int64_t b = (n + kCT - 1) / kCT;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

void cut(Ctx& c, const vmo_hypergraph* h, const int32_t* part, int32_t nparts, double* part_weight,
         vmo_cut_result* out, hipStream_t s) {
  validate_hypergraph(c, h, false, s);
  VMO_REQUIRE(part != nullptr, "part is NULL");
  VMO_REQUIRE(out != nullptr, "out is NULL");
  VMO_REQUIRE(nparts >= 0, "nparts must be >= 0");
  bool separators = false;
  {
    Buf<int> bad(c.pool, 1);
    VMO_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    VMO_LAUNCH(k_check_part, gsz(h->k), kCT, 0, s, part, h->k, nparts, bad.p);
    const int b = read1(bad.p, s);
    VMO_REQUIRE(!(b & 1), "part ids must be in [0, 2^30)");
    separators = (b & 2) != 0;
  }
  int32_t l = h->l;
  Buf<int32_t> lam(c.pool, l > 0 ? l : 1), big(c.pool, l + 1), bigrank(c.pool, l + 1);
  if (l > 0) {
    VMO_LAUNCH(k_lambda_small, gsz(l), kCT, 0, s, h->net_ptr, h->pins, l, part, lam.p, big.p);
    scan_exclusive<int32_t>(c, big.p, bigrank.p, l, bigrank.p + l, s);
    int32_t nb = read1(bigrank.p + l, s);
    if (nb > 0) {
      Buf<int32_t> bignet(c.pool, nb);
      Buf<int64_t> biglen(c.pool, nb + 1);
      VMO_LAUNCH(k_big_list, gsz(l), kCT, 0, s, big.p, bigrank.p, l, h->net_ptr, bignet.p, biglen.p);
      scan_exclusive<int64_t>(c, biglen.p, biglen.p, nb, biglen.p + nb, s);
      int64_t nk = read1(biglen.p + nb, s);
      Buf<uint64_t> keys(c.pool, nk);
      VMO_LAUNCH(k_big_keys, (unsigned)(l < 65536 ? l : 65536), kCT, 0, s, h->net_ptr, h->pins, big.p, bigrank.p,
                 biglen.p, l, part, keys.p);
      radix_sort<uint64_t>(c, keys.p, nullptr, nk, 32 + bits_for((uint64_t)nb), s);
      VMO_LAUNCH(k_big_count, gsz(nk), kCT, 0, s, keys.p, nk, bignet.p, lam.p);
    }
  }
  int nb = 256;
  Buf<double> p3(c.pool, 3 * nb), o3(c.pool, 3);
  VMO_LAUNCH(k_cut_partial, nb, kCT, 0, s, lam.p, h->c, l, p3.p);
  VMO_LAUNCH(k_cut_final, 1, 64, 0, s, p3.p, nb, o3.p);
  if (part_weight && nparts > 0) {
    if (!h->w) {
      VMO_HIP(hipMemsetAsync(part_weight, 0, sizeof(double) * nparts, s));
      VMO_LAUNCH(k_part_count, gsz(h->k), kCT, 0, s, part, h->k, nparts, part_weight);
    } else {
      Buf<uint32_t> key(c.pool, h->k);
      Buf<int32_t> val(c.pool, h->k);
      VMO_LAUNCH(k_pw_keys, gsz(h->k), kCT, 0, s, part, h->k, nparts, key.p, val.p);
      radix_sort<uint32_t>(c, key.p, val.p, h->k, bits_for((uint64_t)nparts), s);
      VMO_LAUNCH(k_pw_sum, gsz(nparts), kCT, 0, s, key.p, val.p, h->k, nparts, h->w, part_weight);
    }
  }
  // per-split cut of the recursive bisection into nparts parts
  Buf<double> res(c.pool, 5);
  if (nparts >= 1) {
    const int64_t nh = 4 * (int64_t)nparts;
    Buf<double> split(c.pool, nh);
    if (separators) {
      VMO_HIP(hipMemsetAsync(split.p, 0, sizeof(double) * nh, s));
      VMO_LAUNCH(k_sep_count, gsz(h->k), kCT, 0, s, part, h->k, nparts, split.p);
    } else if (l > 0) {
      Buf<uint32_t> key(c.pool, l);
      Buf<int32_t> val(c.pool, l);
      VMO_LAUNCH(k_net_split, gsz(l), kCT, 0, s, h->net_ptr, h->pins, l, part, lam.p, nparts, key.p, val.p);
      radix_sort<uint32_t>(c, key.p, val.p, l, bits_for((uint64_t)nh), s);
      VMO_LAUNCH(k_split_sum, gsz(nh * 64), kCT, 0, s, key.p, val.p, l, nparts, h->c, split.p);
    } else {
      VMO_HIP(hipMemsetAsync(split.p, 0, sizeof(double) * nh, s));
    }
    VMO_LAUNCH(k_split_max, 1, kCT, 0, s, split.p, (int32_t)nh, res.p + 3);
  } else {
    VMO_HIP(hipMemsetAsync(res.p + 3, 0, sizeof(double) * 2, s));
  }
  VMO_HIP(hipMemcpyAsync(res.p, o3.p, sizeof(double) * 3, hipMemcpyDeviceToDevice, s));
  double r[5];
  read_bytes(r, res.p, sizeof r, s);
  out->lambda_minus_one = r[0];
  out->cut_net = r[1];
  out->nets_cut = (int64_t)r[2];
  out->max_split = r[3];
  out->max_split_node = (int32_t)r[4];
  out->separators = separators ? 1 : 0;
}

// ------------------------------------------------- allocation-free cut ----
// The workspace of vmo_cut_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes its name to a
// kernel or a copy (on the host it is only a stand-in, not a device address):
// its device address is looked up once per device with hipGetSymbolAddress
// (noalloc_init, called by vmo_create with the device current) and kept in
// g_arena, and only that address is used.
constexpr size_t kArenaBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kArenaBytes];

namespace {
std::mutex g_arena_mu;
std::map<int, uint8_t*> g_arena;       // device -> address of its copy of scratch
std::map<int, std::string> g_arena_err;
}  // namespace

void noalloc_init(int device) {
  std::lock_guard<std::mutex> g(g_arena_mu);
  if (g_arena.count(device) || g_arena_err.count(device)) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_arena_err[device] = std::string("hipGetSymbolAddress of the static arena failed: ") + hipGetErrorString(e);
    return;
  }
  g_arena[device] = static_cast<uint8_t*>(p);
}

void cut_noalloc(Ctx& c, const vmo_hypergraph* h, const int32_t* part, int32_t nparts, double* part_weight,
                 vmo_cut_result* out, hipStream_t s) {
  VMO_REQUIRE(h != nullptr, "h is NULL");
  if (h->k > kNoAllocMaxVerts || h->l > kNoAllocMaxNets)
    throw Error(VMO_E_UNSUPPORTED, "vmo_cut_noalloc takes at most 2^20 vertices and 2^20 nets");
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_arena_mu);
    auto it = g_arena.find(c.device);
    if (it == g_arena.end()) {
      auto er = g_arena_err.find(c.device);
      throw Error(VMO_E_DEVICE, er != g_arena_err.end() ? er->second : "static arena not set up on this device");
    }
    base = it->second;
  }
  // arena layout: [0, 256) the error flag of bounded device-side waits, then
  // the call's blocks by bump allocation
  Arena a{base, kArenaBytes, 256};
  struct Mode {
    Ctx& c;
    ~Mode() {
      c.pool.set_arena(nullptr);
      c.noalloc = false;
      c.arena_flag = nullptr;
      thread_noalloc() = false;
    }
  } mode{c};
  c.noalloc = true;
  c.arena_flag = reinterpret_cast<int*>(base);
  thread_noalloc() = true;
  c.pool.set_arena(&a);
  VMO_HIP(hipMemsetAsync(c.arena_flag, 0, sizeof(int), s));
  cut(c, h, part, nparts, part_weight, out, s);
  check_device_flag(c, s);
}

}  // namespace vmo
