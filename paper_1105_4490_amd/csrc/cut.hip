// Cut metrics of a partition (Sec. 4.1 cut rows/columns; the cut-net metric of
// its footnote; Table 4's maximum cut per split): per-net counts of distinct
// part ids, deterministic FP64 sums, part weights.
#include "vmo_internal.h"

namespace vmo {

constexpr int kCT = 256;
constexpr int kSmallNet = 64;

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
__global__ void k_part_weight(const int32_t* part, const float* w, int32_t k, int32_t nparts, double* pw) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t p = part[v];
    if (p >= 0 && p < nparts) atomicAdd(&pw[p], w ? (double)w[v] : 1.0);
  }
}
__global__ void k_check_part(const int32_t* part, int32_t k, int* bad) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x)
    if (part[v] < 0 || part[v] >= (1 << 30)) atomicOr(bad, 1);
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
  {
    Buf<int> bad(c.pool, 1);
    VMO_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    VMO_LAUNCH(k_check_part, gsz(h->k), kCT, 0, s, part, h->k, bad.p);
    VMO_REQUIRE(read1(bad.p, s) == 0, "part ids must be in [0, 2^30)");
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
    VMO_HIP(hipMemsetAsync(part_weight, 0, sizeof(double) * nparts, s));
    VMO_LAUNCH(k_part_weight, gsz(h->k), kCT, 0, s, part, h->w, h->k, nparts, part_weight);
  }
  double r[3];
  read_bytes(r, o3.p, sizeof r, s);
  out->lambda_minus_one = r[0];
  out->cut_net = r[1];
  out->nets_cut = (int64_t)r[2];
}

}  // namespace vmo
