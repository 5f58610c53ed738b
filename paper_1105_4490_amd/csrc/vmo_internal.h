// Internal declarations of the HIP implementation behind include/vmo.h.
// gfx950 only: 64-wide wavefronts, 256-thread blocks unless stated.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/vmo.h"

namespace vmo {

// ---------------------------------------------------------------- errors ----
struct Error : std::runtime_error {
  vmo_status status;
  Error(vmo_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define VMO_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::vmo::Error(e_ == hipErrorOutOfMemory ? VMO_E_NOMEM : VMO_E_DEVICE,        \
                         std::string(#call ": ") + hipGetErrorString(e_));              \
  } while (0)

#define VMO_REQUIRE(cond, msg)                                                          \
  do {                                                                                  \
    if (!(cond)) throw ::vmo::Error(VMO_E_INVALID, msg);                                \
  } while (0)

// ------------------------------------------------------------------ pool ----
// A fixed device region handed out by bump allocation and released all at
// once (the allocation-free entry points' workspace).
struct Arena {
  uint8_t* base = nullptr;
  size_t cap = 0, used = 0;
};

// Caching device allocator: blocks are kept after release and handed out
// again for requests of at most the same size class.  A pool serves one
// stream: calls synchronise that stream before returning, so a released
// block is idle when reused.  Its methods may be called from any thread.
// While an arena is set, get() takes blocks from it instead (never calling
// hipMalloc; VMO_E_UNSUPPORTED when it is exhausted) and put() of such a
// block does nothing.
class Pool {
 public:
  ~Pool();
  void* get(size_t bytes);
  void put(void* p);
  size_t held() const {
    std::lock_guard<std::mutex> g(mu_);
    return held_;
  }
  void trim();
  // Frees idle blocks, largest first, until at most cap bytes stay idle.
  void trim_to(size_t cap);
  size_t idle() const {
    std::lock_guard<std::mutex> g(mu_);
    return idle_;
  }
  void set_arena(Arena* a) {
    std::lock_guard<std::mutex> g(mu_);
    arena_ = a;
  }

 private:
  static size_t size_class(size_t bytes);
  void trim_locked();
  mutable std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::unordered_map<void*, size_t> size_;
  size_t held_ = 0, idle_ = 0;
  Arena* arena_ = nullptr;
};

template <class T>
struct Buf {
  Pool* pool = nullptr;
  T* p = nullptr;
  size_t n = 0;
  Buf() = default;
  Buf(Pool& pl, size_t count) : pool(&pl), n(count) {
    p = static_cast<T*>(pl.get((count > 0 ? count : 1) * sizeof(T)));
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : pool(o.pool), p(o.p), n(o.n) { o.p = nullptr; }
  Buf& operator=(Buf&& o) noexcept {
    release();
    pool = o.pool; p = o.p; n = o.n; o.p = nullptr;
    return *this;
  }
  ~Buf() { release(); }
  void release() {
    if (p && pool) pool->put(p);
    p = nullptr;
  }
  T* operator()() const { return p; }
};

// Live kernel timing: when on, selected launches are bracketed with HIP events
// on their stream; durations and algorithmic work (bytes or interactions,
// host-known or counted on the device) accumulate per kernel name.
struct ProfAcc {
  double ms = 0.0;
  int64_t launches = 0;
  double work = 0.0;
};
struct ProfPending {
  std::string name;
  hipEvent_t a, b;
  double work;
  int dslot;  // device counter slot, -1 if none
};
struct Prof {
  bool on = false;
  int every = 1;                          // time every n-th launch of a name
  bool count = true;                      // kernels count their work on the device
  std::map<std::string, int64_t> seen;    // launches per name since enabled
  std::map<std::string, ProfAcc> acc;
  std::vector<ProfPending> pend;
  unsigned long long* dcnt = nullptr;
  int nslot = 0, cap = 0;
  std::vector<hipEvent_t> spare;          // events of flushed records, reused
};

// Online launch-configuration tuner.  A kernel family has a few candidate
// configurations that give identical results; the first calls in each size
// bucket try every candidate (twice), timed with HIP events and normalised
// by the work the kernel reports on the device; later calls use the fastest.
struct TuneRec {
  int family, bucket, cfg;
  hipEvent_t a, b;
  int dslot;     // device work counter, or -1: work known on the host
  double hwork;
};
struct TuneStat {
  double ms_per_work[8] = {};
  int n[8] = {};
};
struct Tuner {
  static constexpr int kMaxCfg = 8;
  std::map<std::pair<int, int>, TuneStat> stat;
  std::vector<TuneRec> pend;
  unsigned long long* dwork = nullptr;
  int nslot = 0, cap = 0;
};

struct Ctx {
  int device = 0;
  std::string err;
  Pool pool;
  Prof prof;
  Tuner tune;
  int* dflag = nullptr;  // device error flag of bounded device-side waits
  unsigned long long* wslots = nullptr;  // the walk's interaction counters (kept zero between walks)
  // Allocation-free call in progress: the pool draws from an arena, the
  // device error flag lives in it (arena_flag), and neither the tuner nor live
  // timing create events or device counters.
  bool noalloc = false;
  int* arena_flag = nullptr;
  // Calls that return before their work is done: the event recorded on the
  // stream of the last such call (tail_on while it may be pending), which a
  // call on another stream waits for before reusing pool blocks; and the
  // sticky word their device-side checks set (kAsync* bits), which vmo_sync
  // turns into VMO_E_INVALID.
  hipEvent_t tail = nullptr;
  hipStream_t tail_stream = nullptr;
  bool tail_on = false;
  int* aflag = nullptr;
  size_t pool_cap = 0;  // idle pool bytes kept after a synchronising call (0: no bound)
  // While a layout runs: the largest level's vertex count, so that the tree's
  // node arrays and the walk's parts are requested at one size for every
  // level (the pool then hands the same blocks to each level instead of
  // keeping one set per level).
  int64_t layout_kmax = 0;
  ~Ctx();
};
enum : int { kAsyncPermutation = 1, kAsyncPartner = 2, kAsyncCsr = 4 };
// Waits for the last asynchronous call's work if it ran on another stream.
void join_tail(Ctx& c, hipStream_t s);
// Marks the end of an asynchronous call on s.
void mark_tail(Ctx& c, hipStream_t s);
// The context's sticky asynchronous-check word (allocated and zeroed on first use).
int* async_flag(Ctx& c);
// ORs a call's check word into the sticky word (on the stream, no wait).
void post_async_check(Ctx& c, const int* word, hipStream_t s);
// After the stream is synchronised: throws VMO_E_INVALID naming the checks
// that failed since the last vmo_sync, and clears the word.
void check_async_flag(Ctx& c, hipStream_t s);
// Trims the pool to its bound after a synchronising call (waits for s first).
void trim_pool(Ctx& c, hipStream_t s);

// Calls of the calling host thread read device scalars into plain host
// memory instead of its pinned buffer (which the first use would allocate).
bool& thread_noalloc();

// Allocation-free cut: the static arena's address on `device` (looked up once
// per device, with the device current), and the call itself.
constexpr int32_t kNoAllocMaxVerts = 1 << 20, kNoAllocMaxNets = 1 << 20;
void noalloc_init(int device);
void cut_noalloc(Ctx& c, const vmo_hypergraph* h, const int32_t* part, int32_t nparts, double* part_weight,
                 vmo_cut_result* out, hipStream_t s);

// Tuner: the configuration to use for (family, bucket) among ncfg.  *timed is
// set while some candidate has fewer than two timed launches (pending ones
// included): the caller then brackets the launch with begin/end.  Once every
// candidate has two, the bucket's pending timings are read (one wait on their
// events) and the fastest candidate is used, untimed, from then on.  begin
// records the start event and returns a zeroed device work counter for the
// kernel; end records the stop event; flush reads what is pending.
int tune_pick(Ctx& c, int family, int bucket, int ncfg, bool* timed);
unsigned long long* tune_begin(Ctx& c, int family, int bucket, int cfg, hipStream_t s);
void tune_begin_host(Ctx& c, int family, int bucket, int cfg, double work, hipStream_t s);
void tune_end(Ctx& c, hipStream_t s);
void tune_flush(Ctx& c);
enum : int { kTuneAssign = 1, kTuneSort = 2 };  // tuner families: Lloyd assignment, radix sort


// The context's device error flag (allocated and zeroed on first use), and
// its check after the stream's work: throws VMO_E_DEVICE if a kernel set it.
int* device_flag(Ctx& c);
void check_device_flag(Ctx& c, hipStream_t s);

// Returns a handle for prof_end (-1 when profiling is off).  If dwork is not
// NULL it receives a zeroed device counter the kernel adds its work to.
// dwork != NULL: *dwork receives a device counter slot for the launch's work,
// which the caller's kernels write (it is not cleared).
int prof_begin(Ctx& c, const char* name, double work, hipStream_t s, unsigned long long** dwork);
void prof_end(Ctx& c, int h, hipStream_t s);
void prof_restart(Ctx& c, int h, hipStream_t s);  // records the start event of h again
// Collect finished events (call after the stream is synchronised).
void prof_flush(Ctx& c);
void prof_discard(Ctx& c);

// Device scalar readback (synchronises `s`).  The value lands in a small
// pinned host buffer of the calling thread (allocated once): a copy into
// pageable memory goes through the runtime's staging path, which costs tens
// of microseconds more per read.
constexpr size_t kPinnedBytes = 4096;
void* pinned_scratch();  // kPinnedBytes of pinned host memory per host thread
template <class T>
T read1(const T* dptr, hipStream_t s) {
  static_assert(sizeof(T) <= kPinnedBytes, "read1 reads one scalar");
  T* h = static_cast<T*>(pinned_scratch());
  VMO_HIP(hipMemcpyAsync(h, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  VMO_HIP(hipStreamSynchronize(s));
  return *h;
}
// n bytes from the device into host memory dst, through the pinned buffer
// when they fit (synchronises `s`).
inline void read_bytes(void* dst, const void* src, size_t n, hipStream_t s) {
  if (n == 0) return;
  if (n <= kPinnedBytes) {
    void* h = pinned_scratch();
    VMO_HIP(hipMemcpyAsync(h, src, n, hipMemcpyDeviceToHost, s));
    VMO_HIP(hipStreamSynchronize(s));
    std::memcpy(dst, h, n);
  } else {
    VMO_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s));
    VMO_HIP(hipStreamSynchronize(s));
  }
}

inline unsigned nblocks(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 0x7fffffff) b = 0x7fffffff;
  return (unsigned)b;
}

#define VMO_LAUNCH(kernel, grid, block, shmem, stream, ...)                                   \
  do {                                                                                        \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__);          \
    VMO_HIP(hipGetLastError());                                                               \
  } while (0)

// ------------------------------------------------------------ randomness ----
// SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden gamma,
// each output is the mix function of the state.  rng3 chains three streams:
// the (c+1)-th output of the stream seeded by the (b+1)-th output of the
// stream seeded by the (a+1)-th output of the stream seeded by `seed`.
__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
__host__ __device__ inline uint64_t rng3(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t h = sm_mix(seed + kGamma * (a + 1));
  h = sm_mix(h + kGamma * (b + 1));
  return sm_mix(h + kGamma * (c + 1));
}
enum : uint64_t { kTagInit = 1, kTagProlong = 2, kTagMatch = 3, kTagKmeans = 16 };

// Ordered-integer image of a float: a < b  <=>  fkey(a) < fkey(b).
__host__ __device__ inline uint32_t fkey(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float fkey_inv(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, u);
}

// 128-bit unsigned as two words (exact D^2 sums of the k-means++ draw).
struct U128 {
  uint64_t lo, hi;
};
__host__ __device__ inline U128 u128_add(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
  return r;
}
__host__ __device__ inline U128 u128_sub(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
  return r;
}
__host__ __device__ inline bool u128_gt(U128 a, U128 b) {
  return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}
__host__ __device__ inline bool u128_zero(U128 a) { return a.lo == 0 && a.hi == 0; }

// ---------------------------------------------------------------- prims ----
// Exclusive scan of n values (out may alias in); *total (device, optional)
// receives the sum.  T: int32_t, int64_t, uint64_t, U128.
template <class T>
void scan_exclusive(Ctx& c, const T* in, T* out, int64_t n, T* total, hipStream_t s);
// Exclusive scan of n ints whose sums over consecutive groups of kScanPart
// items are given (parts[ceil(n / kScanPart)], formed by the producer of in):
// one launch.  n <= kScanPartMax.
constexpr int kScanPart = 256;
constexpr int64_t kScanPartMax = (int64_t)2048 * 2048;
void scan_exclusive_parts(Ctx& c, const int32_t* in, int32_t* out, int64_t n, const int32_t* parts, hipStream_t s);

// Stable LSD radix sort of keys (uint32_t or uint64_t) on bits [0, bits), with
// optional int32 values carried along.  Sorted output overwrites keys/vals.
template <class K>
void radix_sort(Ctx& c, K* keys, int32_t* vals, int64_t n, int bits, hipStream_t s);

// Fill helpers.
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
void iota_i32(int32_t* p, int64_t n, hipStream_t s);

// Device-side validation of a hypergraph's pins (range, strictly ascending)
// and of optional weights/costs (finite, >= 0 or > 0).  Throws VMO_E_INVALID.
void validate_hypergraph(Ctx& c, const vmo_hypergraph* h, bool positive_wc, hipStream_t s);
void validate_finite(Ctx& c, const float* x, int64_t n, const char* what, hipStream_t s);

// Validation of several ordering jobs with two host round trips in all:
// hypergraph structure, weights and costs (>= 0), coordinates (finite, if
// given), graph-mode edges (net_ptr[e] = 2e).  npins receives net_ptr[l] of
// each job.  Errors name the job.
struct JobCheck {
  const vmo_hypergraph* h;
  const float* x;       // coordinates to check, or NULL
  bool x_required;
  bool graph;
};
void validate_jobs(Ctx& c, const std::vector<JobCheck>& jobs, std::vector<int64_t>& npins, hipStream_t s);
// Consistency of an ordering result of k vertices and P parts (heap ids, block
// boundaries, part ids, vperm a permutation); returns its node count.
int32_t check_ordering(Ctx& c, int32_t k, int32_t P, const vmo_order_out* in, hipStream_t s);

// Transpose of a CSR incidence (rows -> columns): out row j lists, ascending,
// the input rows containing j.  nrows, ncols, ptr [nrows+1], idx -> optr
// [ncols+1], oidx [ptr[nrows]].
void csr_transpose(Ctx& c, int32_t nrows, int32_t ncols, const int64_t* ptr, const int32_t* idx,
                   int64_t* optr, int32_t* oidx, hipStream_t s);

// Components: label[v] = minimum vertex id of v's component.
void components(Ctx& c, int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins,
                int32_t* label, hipStream_t s);

inline int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

// FP64 sum of c[val[q]] for q = b .. e-1 (1 each when c is NULL), one by
// one in that order, by a whole wavefront: its lanes load 64 costs at a time
// into `stage` (64 floats of LDS owned by the wavefront), then every lane
// adds them in order (the loads of a chunk are in flight together instead of
// one dependent load per term).  All lanes return the sum.
__device__ inline double wave_ordered_cost_sum(const float* c, const int32_t* val, int64_t b, int64_t e,
                                               float* stage) {
  if (!c) return (double)(e > b ? e - b : 0);  // n ones, exact below 2^53
  const int lane = threadIdx.x & 63;
  double a = 0.0;
  for (int64_t q0 = b; q0 < e; q0 += 64) {
    const int m = e - q0 < 64 ? (int)(e - q0) : 64;
    const float v = lane < m ? c[val[q0 + lane]] : 0.0f;
    // the previous chunk's reads are done before the stage is overwritten
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    stage[lane] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (m == 64) {
      const float4* s4 = reinterpret_cast<const float4*>(stage);
#pragma unroll
      for (int r = 0; r < 16; r += 4) {
        const float4 u0 = s4[r], u1 = s4[r + 1], u2 = s4[r + 2], u3 = s4[r + 3];
        a += (double)u0.x; a += (double)u0.y; a += (double)u0.z; a += (double)u0.w;
        a += (double)u1.x; a += (double)u1.y; a += (double)u1.z; a += (double)u1.w;
        a += (double)u2.x; a += (double)u2.y; a += (double)u2.z; a += (double)u2.w;
        a += (double)u3.x; a += (double)u3.y; a += (double)u3.z; a += (double)u3.w;
      }
    } else {
      for (int i = 0; i < m; ++i) a += (double)stage[i];
    }
  }
  return a;
}

}  // namespace vmo
