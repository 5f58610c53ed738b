// Matrix-to-hypergraph models of Table 1 (row-net, column-net, symmetric,
// bipartite) and
// the dual hypergraph (Definition of the dual, Sec. 1.1).
#include "vmo_internal.h"

namespace vmo {

constexpr int kMT = 256;
static unsigned gsz(int64_t n) {
  int64_t b = (n + kMT - 1) / kMT;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Off-diagonal entries as keys min(i,j) * n + max(i,j).
__global__ void k_sym_flag(const int64_t* rowptr, const int32_t* col, int32_t m, int64_t nnz, int32_t* flag) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = m;
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (rowptr[mid] <= p) lo = mid; else hi = mid;
    }
    flag[p] = col[p] != lo;
  }
}
__global__ void k_sym_keys(const int64_t* rowptr, const int32_t* col, int32_t m, int32_t n, int64_t nnz,
                           const int32_t* flag, const int32_t* pos, uint64_t* keys) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[p]) continue;
    int32_t lo = 0, hi = m;
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (rowptr[mid] <= p) lo = mid; else hi = mid;
    }
    uint64_t a = (uint64_t)(lo < col[p] ? lo : col[p]), b = (uint64_t)(lo < col[p] ? col[p] : lo);
    keys[pos[p]] = a * (uint64_t)n + b;
  }
}
__global__ void k_uniq_flag(const uint64_t* keys, int64_t n, int32_t* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}
__global__ void k_sym_write(const uint64_t* keys, const int32_t* flag, const int32_t* pos, int64_t n, int32_t nv,
                            int64_t* net_ptr, int32_t* pins) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    int32_t e = pos[i];
    pins[2 * (int64_t)e] = (int32_t)(keys[i] / (uint64_t)nv);
    pins[2 * (int64_t)e + 1] = (int32_t)(keys[i] % (uint64_t)nv);
    net_ptr[e] = 2 * (int64_t)e;
  }
}
__global__ void k_set_last(int64_t* p, int64_t v) { *p = v; }

// Bipartite model: nonzero p = (i, j) is the edge {i, m + j}.
__global__ void k_bip_write(const int64_t* rowptr, const int32_t* col, int32_t m, int64_t nnz, int64_t* net_ptr,
                            int32_t* pins) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = m;
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (rowptr[mid] <= p) lo = mid; else hi = mid;
    }
    pins[2 * p] = lo;
    pins[2 * p + 1] = m + col[p];
    net_ptr[p] = 2 * p;
  }
}

void model(Ctx& c, int model, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, int64_t* net_ptr,
           int32_t* pins, int32_t cap_nets, int64_t cap_pins, int32_t* k_out, int32_t* l_out, int64_t* np_out,
           hipStream_t s) {
  VMO_REQUIRE(m >= 1 && n >= 1, "matrix needs m, n >= 1");
  VMO_REQUIRE(model == VMO_ROW_NET || model == VMO_COLUMN_NET || model == VMO_SYMMETRIC || model == VMO_BIPARTITE,
              "unknown model");
  VMO_REQUIRE(rowptr && net_ptr && k_out && l_out && np_out, "NULL argument");
  vmo_hypergraph a{n, m, rowptr, col, nullptr, nullptr};  // rows as nets over columns
  validate_hypergraph(c, &a, false, s);
  int64_t nnz = read1(rowptr + m, s);
  if (model == VMO_ROW_NET) {
    VMO_REQUIRE(cap_nets >= m && cap_pins >= nnz, "output capacity too small");
    VMO_HIP(hipMemcpyAsync(net_ptr, rowptr, 8 * ((int64_t)m + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) VMO_HIP(hipMemcpyAsync(pins, col, 4 * nnz, hipMemcpyDeviceToDevice, s));
    *k_out = n; *l_out = m; *np_out = nnz;
  } else if (model == VMO_COLUMN_NET) {
    VMO_REQUIRE(cap_nets >= n && cap_pins >= nnz, "output capacity too small");
    csr_transpose(c, m, n, rowptr, col, net_ptr, pins, s);
    *k_out = m; *l_out = n; *np_out = nnz;
  } else if (model == VMO_BIPARTITE) {
    VMO_REQUIRE((int64_t)m + n < (int64_t(1) << 31), "m + n must be below 2^31");
    VMO_REQUIRE(nnz < (int64_t(1) << 31), "too many nonzeros for the bipartite model");
    VMO_REQUIRE(cap_nets >= nnz && cap_pins >= 2 * nnz, "output capacity too small");
    if (nnz > 0) VMO_LAUNCH(k_bip_write, gsz(nnz), kMT, 0, s, rowptr, col, m, nnz, net_ptr, pins);
    VMO_LAUNCH(k_set_last, 1, 1, 0, s, net_ptr + nnz, 2 * nnz);
    *k_out = m + n; *l_out = (int32_t)nnz; *np_out = 2 * nnz;
  } else {
    VMO_REQUIRE(m == n, "the symmetric model needs a square matrix");
    int64_t l = 0;
    if (nnz > 0) {
      Buf<int32_t> flag(c.pool, nnz + 1), pos(c.pool, nnz + 1);
      VMO_LAUNCH(k_sym_flag, gsz(nnz), kMT, 0, s, rowptr, col, m, nnz, flag.p);
      scan_exclusive<int32_t>(c, flag.p, pos.p, nnz, pos.p + nnz, s);
      int64_t no = read1(pos.p + nnz, s);
      if (no > 0) {
        Buf<uint64_t> keys(c.pool, no);
        VMO_LAUNCH(k_sym_keys, gsz(nnz), kMT, 0, s, rowptr, col, m, n, nnz, flag.p, pos.p, keys.p);
        radix_sort<uint64_t>(c, keys.p, nullptr, no, bits_for((uint64_t)n * (uint64_t)n - 1), s);
        Buf<int32_t> uf(c.pool, no + 1), up(c.pool, no + 1);
        VMO_LAUNCH(k_uniq_flag, gsz(no), kMT, 0, s, keys.p, no, uf.p);
        scan_exclusive<int32_t>(c, uf.p, up.p, no, up.p + no, s);
        l = read1(up.p + no, s);
        VMO_REQUIRE(cap_nets >= l && cap_pins >= 2 * l, "output capacity too small");
        VMO_LAUNCH(k_sym_write, gsz(no), kMT, 0, s, keys.p, uf.p, up.p, no, n, net_ptr, pins);
      }
    }
    VMO_LAUNCH(k_set_last, 1, 1, 0, s, net_ptr + l, 2 * l);
    *k_out = n; *l_out = (int32_t)l; *np_out = 2 * l;
  }
  VMO_HIP(hipStreamSynchronize(s));
}

void dual(Ctx& c, const vmo_hypergraph* h, int64_t* dptr, int32_t* dpins, hipStream_t s) {
  validate_hypergraph(c, h, false, s);
  VMO_REQUIRE(dptr != nullptr, "dptr is NULL");
  csr_transpose(c, h->l, h->k, h->net_ptr, h->pins, dptr, dpins, s);
}

}  // namespace vmo
