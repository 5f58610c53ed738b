// Device primitives: caching pool, scans, LSD radix sort, fills, input
// validation, CSR transpose and connected components.
#include "vmo_internal.h"

namespace vmo {

// ------------------------------------------------------------------ pool ----
size_t Pool::size_class(size_t b) {
  if (b <= 4096) return (b + 255) & ~size_t(255);
  int lg = 63 - __builtin_clzll(b);
  size_t g = size_t(1) << (lg - 2);
  return (b + g - 1) & ~(g - 1);
}

void Pool::trim_to(size_t cap) {
  std::lock_guard<std::mutex> g(mu_);
  while (idle_ > cap && !free_.empty()) {
    auto it = std::prev(free_.end());  // the largest idle block
    (void)hipFree(it->second);
    held_ -= it->first;
    idle_ -= it->first;
    size_.erase(it->second);
    free_.erase(it);
  }
}

void* Pool::get(size_t bytes) {
  std::lock_guard<std::mutex> g(mu_);
  if (arena_) {
    const size_t b = (bytes + 255) & ~size_t(255);
    if (b > arena_->cap - arena_->used)
      throw Error(VMO_E_UNSUPPORTED, "the input needs more workspace than the " + std::to_string(arena_->cap >> 20) +
                                         " MiB static arena of the allocation-free call holds");
    void* p = arena_->base + arena_->used;
    arena_->used += b;
    return p;
  }
  size_t cls = size_class(bytes);
  auto it = free_.lower_bound(cls);
  if (it != free_.end() && it->first <= 2 * cls) {
    void* p = it->second;
    idle_ -= it->first;
    free_.erase(it);
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_locked();
    e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(VMO_E_NOMEM, "device allocation of " + std::to_string(cls) + " bytes failed");
    }
  }
  size_[p] = cls;
  held_ += cls;
  return p;
}

void Pool::put(void* p) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = size_.find(p);  // arena blocks are not in size_: nothing to do
  if (it == size_.end()) return;
  free_.emplace(it->second, p);
  idle_ += it->second;
}

void Pool::trim() {
  std::lock_guard<std::mutex> g(mu_);
  trim_locked();
}

void Pool::trim_locked() {
  for (auto& kv : free_) {
    (void)hipFree(kv.second);
    held_ -= size_[kv.second];
    size_.erase(kv.second);
  }
  free_.clear();
  idle_ = 0;
}

Pool::~Pool() {
  for (auto& kv : size_) (void)hipFree(kv.first);
}

// --------------------------------------------------------------- profile ----
namespace {
// Pinned buffers of threads that have ended, handed to the next threads that
// need one.  Held through pointers that are never deleted, so that a thread
// ending during or after static destruction still finds them.
std::mutex& pinned_mu() {
  static std::mutex* m = new std::mutex;
  return *m;
}
std::vector<void*>& pinned_free() {
  static std::vector<void*>* v = new std::vector<void*>;
  return *v;
}
// The pinned scalar buffer of a host thread.  When the thread ends it goes
// back to the list above, with no HIP call: the thread-local state of the HIP
// runtime and of a preloaded profiler tool may already be destroyed by then
// (the order in which the libraries' thread-local objects are destroyed is
// unspecified), and a HIP call from here would run into it.
struct PinnedScratch {
  void* p = nullptr;
  ~PinnedScratch() {
    if (!p) return;
    std::lock_guard<std::mutex> g(pinned_mu());
    pinned_free().push_back(p);
  }
};
thread_local PinnedScratch t_pinned;
thread_local bool t_noalloc = false;
alignas(256) thread_local uint8_t t_plain[kPinnedBytes];
}  // namespace

bool& thread_noalloc() { return t_noalloc; }

void* pinned_scratch() {
  if (t_noalloc) return t_plain;  // plain host memory: copies into it are staged by the runtime
  if (!t_pinned.p) {
    {
      std::lock_guard<std::mutex> g(pinned_mu());
      if (!pinned_free().empty()) {
        t_pinned.p = pinned_free().back();
        pinned_free().pop_back();
      }
    }
    if (!t_pinned.p) VMO_HIP(hipHostMalloc(&t_pinned.p, kPinnedBytes, hipHostMallocDefault));
  }
  return t_pinned.p;
}

Ctx::~Ctx() {
  prof_discard(*this);
  for (hipEvent_t e : prof.spare) (void)hipEventDestroy(e);
  if (prof.dcnt) (void)hipFree(prof.dcnt);
  if (wslots) (void)hipFree(wslots);
  for (auto& r : tune.pend) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (tune.dwork) (void)hipFree(tune.dwork);
  if (dflag) (void)hipFree(dflag);
  if (aflag) (void)hipFree(aflag);
  if (tail) (void)hipEventDestroy(tail);
}

// ------------------------------------------------------- asynchronous calls ----
void join_tail(Ctx& c, hipStream_t s) {
  if (c.tail_on && c.tail_stream != s) {
    VMO_HIP(hipEventSynchronize(c.tail));
    c.tail_on = false;
  }
}

void mark_tail(Ctx& c, hipStream_t s) {
  if (!c.tail) VMO_HIP(hipEventCreateWithFlags(&c.tail, hipEventDisableTiming));
  VMO_HIP(hipEventRecord(c.tail, s));
  c.tail_stream = s;
  c.tail_on = true;
}

int* async_flag(Ctx& c) {
  if (!c.aflag) {
    VMO_HIP(hipMalloc(&c.aflag, sizeof(int)));
    VMO_HIP(hipMemset(c.aflag, 0, sizeof(int)));
  }
  return c.aflag;
}

__global__ void k_or_word(const int* src, int* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *src) atomicOr(dst, *src);
}

void post_async_check(Ctx& c, const int* word, hipStream_t s) {
  int* f = async_flag(c);
  VMO_LAUNCH(k_or_word, 1, 64, 0, s, word, f);
}

void check_async_flag(Ctx& c, hipStream_t s) {
  if (!c.aflag) return;
  const int v = read1(c.aflag, s);
  if (!v) return;
  VMO_HIP(hipMemsetAsync(c.aflag, 0, sizeof(int), s));
  VMO_HIP(hipStreamSynchronize(s));
  std::string m = "an earlier asynchronous call rejected its input:";
  if (v & kAsyncPermutation) m += " vperm is not a permutation of the vertices;";
  if (v & kAsyncPartner) m += " a row has no partner column (mu[i] in [m, 2m));";
  if (v & kAsyncCsr) m += " CSR arrays invalid (rowptr not non-decreasing from 0, or a column outside [0, n) or not ascending);";
  throw Error(VMO_E_INVALID, m);
}

void trim_pool(Ctx& c, hipStream_t s) {
  if (c.pool_cap == 0 || c.pool.idle() <= c.pool_cap) return;
  VMO_HIP(hipStreamSynchronize(s));
  c.tail_on = false;
  c.pool.trim_to(c.pool_cap);
}

// ----------------------------------------------------------------- tuner ----
int tune_pick(Ctx& c, int family, int bucket, int ncfg, bool* timed) {
  if (c.noalloc) {
    // no timing (it would create events): the best candidate known so far,
    // else the first (all candidates give the same results)
    *timed = false;
    const auto it = c.tune.stat.find({family, bucket});
    int best = -1;
    if (it != c.tune.stat.end())
      for (int i = 0; i < ncfg; ++i)
        if (it->second.n[i] > 0 &&
            (best < 0 || it->second.ms_per_work[i] / it->second.n[i] < it->second.ms_per_work[best] / it->second.n[best]))
          best = i;
    return best < 0 ? 0 : best;
  }
  int tot[Tuner::kMaxCfg] = {};
  bool pending = false;
  {
    const TuneStat& st = c.tune.stat[{family, bucket}];
    for (int i = 0; i < ncfg; ++i) tot[i] = st.n[i];
  }
  for (const TuneRec& r : c.tune.pend)
    if (r.family == family && r.bucket == bucket) {
      ++tot[r.cfg];
      pending = true;
    }
  for (int i = 0; i < ncfg; ++i)
    if (tot[i] < 2) {
      *timed = true;
      return i;
    }
  if (pending) tune_flush(c);
  *timed = false;
  const TuneStat& st = c.tune.stat[{family, bucket}];
  int best = -1;
  for (int i = 0; i < ncfg; ++i)
    if (st.n[i] > 0 && (best < 0 || st.ms_per_work[i] / st.n[i] < st.ms_per_work[best] / st.n[best])) best = i;
  return best < 0 ? 0 : best;
}

unsigned long long* tune_begin(Ctx& c, int family, int bucket, int cfg, hipStream_t s) {
  Tuner& t = c.tune;
  if (t.nslot == t.cap) {
    VMO_HIP(hipStreamSynchronize(s));
    tune_flush(c);
    if (t.cap == 0) {
      t.cap = 1024;
      VMO_HIP(hipMalloc(&t.dwork, sizeof(unsigned long long) * t.cap));
    }
  }
  TuneRec r;
  r.family = family; r.bucket = bucket; r.cfg = cfg;
  r.dslot = t.nslot++;
  r.hwork = 0.0;
  VMO_HIP(hipMemsetAsync(t.dwork + r.dslot, 0, sizeof(unsigned long long), s));
  VMO_HIP(hipEventCreate(&r.a));
  VMO_HIP(hipEventCreate(&r.b));
  VMO_HIP(hipEventRecord(r.a, s));
  t.pend.push_back(r);
  return t.dwork + r.dslot;
}

void tune_begin_host(Ctx& c, int family, int bucket, int cfg, double work, hipStream_t s) {
  TuneRec r;
  r.family = family; r.bucket = bucket; r.cfg = cfg;
  r.dslot = -1;
  r.hwork = work;
  VMO_HIP(hipEventCreate(&r.a));
  VMO_HIP(hipEventCreate(&r.b));
  VMO_HIP(hipEventRecord(r.a, s));
  c.tune.pend.push_back(r);
}

void tune_end(Ctx& c, hipStream_t s) { VMO_HIP(hipEventRecord(c.tune.pend.back().b, s)); }

void tune_flush(Ctx& c) {
  Tuner& t = c.tune;
  if (t.pend.empty()) return;
  // the timed launches have finished (and written their work counts) before
  // the counts are read
  for (auto& r : t.pend) VMO_HIP(hipEventSynchronize(r.b));
  std::vector<unsigned long long> w(t.nslot);
  if (t.nslot > 0)
    VMO_HIP(hipMemcpy(w.data(), t.dwork, sizeof(unsigned long long) * t.nslot, hipMemcpyDeviceToHost));
  for (auto& r : t.pend) {
    float ms = 0.0f;
    VMO_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    const double wk = r.dslot >= 0 ? (double)w[r.dslot] : r.hwork;
    if (wk > 0) {
      TuneStat& st = t.stat[{r.family, r.bucket}];
      st.ms_per_work[r.cfg] += (double)ms / wk;
      st.n[r.cfg] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  t.pend.clear();
  t.nslot = 0;
}


int prof_begin(Ctx& c, const char* name, double work, hipStream_t s, unsigned long long** dwork) {
  if (dwork) *dwork = nullptr;
  if (!c.prof.on || c.noalloc) return -1;
  if (c.prof.seen[name]++ % c.prof.every != 0) return -1;
  ProfPending p;
  p.name = name;
  p.work = work;
  p.dslot = -1;
  if (dwork && c.prof.count) {
    if (c.prof.nslot == c.prof.cap) {
      VMO_HIP(hipStreamSynchronize(s));
      prof_flush(c);
      if (c.prof.cap == 0) {
        c.prof.cap = 4096;
        VMO_HIP(hipMalloc(&c.prof.dcnt, sizeof(unsigned long long) * c.prof.cap));
      }
    }
    p.dslot = c.prof.nslot++;
    *dwork = c.prof.dcnt + p.dslot;
  }
  for (hipEvent_t* e : {&p.a, &p.b}) {
    if (!c.prof.spare.empty()) {
      *e = c.prof.spare.back();
      c.prof.spare.pop_back();
    } else {
      VMO_HIP(hipEventCreate(e));
    }
  }
  VMO_HIP(hipEventRecord(p.a, s));
  c.prof.pend.push_back(p);
  return (int)c.prof.pend.size() - 1;
}

void prof_restart(Ctx& c, int h, hipStream_t s) {
  if (h < 0) return;
  VMO_HIP(hipEventRecord(c.prof.pend[h].a, s));
}

void prof_end(Ctx& c, int h, hipStream_t s) {
  if (h < 0) return;
  VMO_HIP(hipEventRecord(c.prof.pend[h].b, s));
}

void prof_flush(Ctx& c) {
  if (c.prof.pend.empty()) return;
  for (auto& p : c.prof.pend) VMO_HIP(hipEventSynchronize(p.b));
  std::vector<unsigned long long> cnt(c.prof.nslot);
  if (c.prof.nslot > 0)
    VMO_HIP(hipMemcpy(cnt.data(), c.prof.dcnt, sizeof(unsigned long long) * c.prof.nslot, hipMemcpyDeviceToHost));
  for (auto& p : c.prof.pend) {
    float ms = 0.0f;
    VMO_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    ProfAcc& a = c.prof.acc[p.name];
    a.ms += ms;
    a.launches += 1;
    a.work += p.dslot >= 0 ? (double)cnt[p.dslot] : p.work;
    c.prof.spare.push_back(p.a);
    c.prof.spare.push_back(p.b);
  }
  c.prof.pend.clear();
  c.prof.nslot = 0;
}

void prof_discard(Ctx& c) {
  for (auto& p : c.prof.pend) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c.prof.pend.clear();
  c.prof.nslot = 0;
}

// ------------------------------------------------------------------ scan ----
constexpr int kScanT = 256, kScanI = 8, kScanTile = kScanT * kScanI;

template <class T> __device__ __forceinline__ T tzero() { return T(0); }
template <> __device__ __forceinline__ U128 tzero<U128>() { return U128{0, 0}; }
template <class T> __device__ __forceinline__ T tadd(T a, T b) { return a + b; }
template <> __device__ __forceinline__ U128 tadd<U128>(U128 a, U128 b) { return u128_add(a, b); }

// Block-wide exclusive scan of one value per thread; *tot = block sum.
template <class T>
__device__ T block_excl(T v, T* sh, T* tot) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanT; off <<= 1) {
    T a = t >= off ? sh[t - off] : tzero<T>();
    __syncthreads();
    if (t >= off) sh[t] = tadd(sh[t], a);
    __syncthreads();
  }
  T ex = t > 0 ? sh[t - 1] : tzero<T>();
  *tot = sh[kScanT - 1];
  __syncthreads();
  return ex;
}

template <class T>
__global__ __launch_bounds__(kScanT) void k_scan_reduce(const T* __restrict__ in, int64_t n, T* part) {
  __shared__ T sh[kScanT];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanI;
  T s = tzero<T>();
#pragma unroll
  for (int i = 0; i < kScanI; ++i)
    if (base + i < n) s = tadd(s, in[base + i]);
  T tot;
  (void)block_excl(s, sh, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// part: NULL (one tile), the tiles' exclusive offsets (sum_parts == 0), or
// the totals of groups of sum_parts items (sum_parts > 0; a tile holds
// kScanTile / sum_parts groups), whose sum over the earlier tiles each block
// forms itself (integer sums: any order gives the same offset)
template <class T>
__global__ __launch_bounds__(kScanT) void k_scan_down(const T* in, T* out, int64_t n, const T* part,
                                                      int sum_parts, T* total, int last_block) {
  __shared__ T sh[kScanT];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanI;
  T v[kScanI];
  T s = tzero<T>();
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    v[i] = base + i < n ? in[base + i] : tzero<T>();
    s = tadd(s, v[i]);
  }
  T off = tzero<T>();
  if (part && sum_parts) {
    T o = tzero<T>();
    const int np = (int)blockIdx.x * (kScanTile / sum_parts);
    for (int i = threadIdx.x; i < np; i += kScanT) o = tadd(o, part[i]);
    (void)block_excl(o, sh, &off);
  } else if (part) {
    off = part[blockIdx.x];
  }
  T tot;
  T ex = block_excl(s, sh, &tot);
  T run = tadd(off, ex);
#pragma unroll
  for (int i = 0; i < kScanI; ++i) {
    if (base + i < n) out[base + i] = run;
    run = tadd(run, v[i]);
  }
  if (total && (int)blockIdx.x == last_block && threadIdx.x == kScanT - 1) *total = run;
}

template <class T>
void scan_exclusive(Ctx& c, const T* in, T* out, int64_t n, T* total, hipStream_t s) {
  if (n <= 0) {
    if (total) VMO_HIP(hipMemsetAsync(total, 0, sizeof(T), s));
    return;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    VMO_LAUNCH((k_scan_down<T>), 1, kScanT, 0, s, in, out, n, (const T*)nullptr, 0, total, 0);
    return;
  }
  Buf<T> part(c.pool, nb);
  VMO_LAUNCH((k_scan_reduce<T>), (unsigned)nb, kScanT, 0, s, in, n, part.p);
  if (nb <= kScanTile) {
    // few tiles: each block adds up the earlier tiles' totals itself
    VMO_LAUNCH((k_scan_down<T>), (unsigned)nb, kScanT, 0, s, in, out, n, (const T*)part.p, kScanTile, total,
               (int)(nb - 1));
    return;
  }
  scan_exclusive<T>(c, part.p, part.p, nb, total, s);
  VMO_LAUNCH((k_scan_down<T>), (unsigned)nb, kScanT, 0, s, in, out, n, (const T*)part.p, 0, (T*)nullptr, 0);
}

void scan_exclusive_parts(Ctx& c, const int32_t* in, int32_t* out, int64_t n, const int32_t* parts, hipStream_t s) {
  (void)c;
  static_assert(kScanTile % kScanPart == 0, "a tile holds whole groups");
  VMO_REQUIRE(n >= 1 && n <= kScanPartMax, "scan size out of range");
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  VMO_LAUNCH((k_scan_down<int32_t>), (unsigned)nb, kScanT, 0, s, in, out, n, parts, kScanPart, (int32_t*)nullptr, 0);
}

template void scan_exclusive<int32_t>(Ctx&, const int32_t*, int32_t*, int64_t, int32_t*, hipStream_t);
template void scan_exclusive<int64_t>(Ctx&, const int64_t*, int64_t*, int64_t, int64_t*, hipStream_t);
template void scan_exclusive<uint64_t>(Ctx&, const uint64_t*, uint64_t*, int64_t, uint64_t*, hipStream_t);
template void scan_exclusive<U128>(Ctx&, const U128*, U128*, int64_t, U128*, hipStream_t);

// ------------------------------------------------------------ radix sort ----
// LSD radix sort, 8-bit digits, one histogram launch for all digit positions
// and one scatter launch per digit.  A scatter block takes the next tile in
// start order (an atomic counter), counts its digits, publishes the counts,
// and finds the keys of its digits in earlier tiles by looking back over the
// published words of those tiles (decoupled look-back): a word is 0 (not
// ready), an aggregate of that tile alone, or an inclusive prefix.  Earlier
// tiles belong to blocks that already run, so every wait ends; the wait is
// still bounded, and a bound that runs out sets the context's device error
// flag.  A tile is `ri` rounds of 256 keys; the tile count is tuned online
// per size (radix_sort).
constexpr int kRsT = 256, kRsMaxI = 16;
constexpr uint64_t kStA = 1ull << 62, kStP = 2ull << 62, kStMask = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 24;

template <class K>
__global__ __launch_bounds__(kRsT) void k_rs_hist(const K* __restrict__ keys, int64_t n, int passes,
                                                  uint32_t* ghist) {
  __shared__ uint32_t h[8][256];
  const int t = threadIdx.x;
  for (int p = 0; p < 8; ++p) h[p][t] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kRsT + t; i < n; i += (int64_t)gridDim.x * kRsT) {
    const K key = keys[i];
    for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(int)((key >> (8 * p)) & 255u)], 1u);
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (h[p][t]) atomicAdd(&ghist[p * 256 + t], h[p][t]);
}

// RI: rounds per tile (a power of two up to kRsMaxI); the LDS counts and the
// key registers are sized for it, so that short tiles leave room for more
// blocks per CU.  Loads that do not depend on each other are issued together:
// the scan of the pass's digit totals runs while the tile number is fetched,
// the values are loaded with the keys, and the look-back reads four earlier
// tiles' words at a time.
template <class K, int RI>
__global__ __launch_bounds__(kRsT) void k_rs_scatter(const K* __restrict__ kin, const int32_t* __restrict__ vin,
                                                     K* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                                                     int shift, const uint32_t* __restrict__ ghist,
                                                     uint64_t* status, uint32_t* tile_ctr, int* err) {
  constexpr int ri = RI;
  // per (round, wavefront, digit): count, then exclusive offset in the tile
  __shared__ uint16_t cnt[RI][kRsT / 64][256];
  __shared__ int run[256];
  __shared__ int wsum[kRsT / 64];
  __shared__ int tile_sh;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) tile_sh = (int)atomicAdd(tile_ctr, 1u);
  // exclusive scan of the digit totals of this pass (the same for every
  // tile): within each wavefront by shuffles, then the earlier wavefronts'
  // totals
  const int g = (int)ghist[t];
  int inc = g;
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(inc, off, 64);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wsum[w] = inc;
  uint32_t* cnt32 = reinterpret_cast<uint32_t*>(&cnt[0][0][0]);
  for (int e = t; e < ri * (kRsT / 64) * 256 / 2; e += kRsT) cnt32[e] = 0u;
  __syncthreads();
  int pre = inc - g;
  for (int ww = 0; ww < w; ++ww) pre += wsum[ww];
  const int64_t tile = tile_sh;
  const int64_t base = tile * kRsT * ri;
  const uint64_t below = lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
  K key[RI];
  int32_t val[RI];
  int dig[RI], rk[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const int64_t idx = base + (int64_t)r * kRsT + t;
    const bool valid = idx < n;
    key[r] = valid ? kin[idx] : K(0);
    val[r] = valid && vin ? vin[idx] : 0;
  }
  // ranks of every round at once: lanes of a wavefront with equal digits are
  // found by eight ballots; each (round, wavefront, digit) count is written by
  // the first such lane
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const int64_t idx = base + (int64_t)r * kRsT + t;
    const bool valid = idx < n;
    dig[r] = valid ? (int)((key[r] >> shift) & 255u) : -1;
    const int d = valid ? dig[r] : 0;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    rk[r] = __popcll(m & below);
    if (valid && rk[r] == 0) cnt[r][w][d] = (uint16_t)__popcll(m);
  }
  __syncthreads();
  // digit t: offsets over (round, wavefront) in order; c = its count in the tile
  int c = 0;
  for (int r = 0; r < ri; ++r)
    for (int ww = 0; ww < kRsT / 64; ++ww) {
      const int v = cnt[r][ww][t];
      cnt[r][ww][t] = (uint16_t)c;
      c += v;
    }
  // publish this tile's count of digit t, then look back for the keys of
  // digit t in earlier tiles: up to four words per round trip, taken in
  // order from the nearest; a word not yet written ends the round there
  uint64_t* st = status + tile * 256 + t;
  uint64_t excl = 0;
  if (tile == 0) {
    __hip_atomic_store(st, kStP | (uint64_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(st, kStA | (uint64_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t pt = tile - 1;
    int spins = 0;
    while (true) {
      uint64_t v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        v[q] = pt - q >= 0 ? __hip_atomic_load(status + (pt - q) * 256 + t, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : kStP;  // not reached: tile 0's word is an inclusive prefix
      int q = 0;
      bool done = false;
      for (; q < 4; ++q) {
        const uint64_t f = v[q] & ~kStMask;
        if (f == 0) break;
        excl += v[q] & kStMask;
        if (f == kStP) {
          done = true;
          break;
        }
      }
      if (done) break;
      pt -= q;
      if (q < 4) {
        if (++spins > kSpinLimit) {
          atomicExch(err, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __hip_atomic_store(st, kStP | (excl + (uint64_t)c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  run[t] = (int)(pre + excl);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    if (dig[r] < 0) continue;
    const int d = dig[r];
    const int dest = run[d] + cnt[r][w][d] + rk[r];
    kout[dest] = key[r];
    if (vin) vout[dest] = val[r];
  }
}

int* device_flag(Ctx& c) {
  if (c.noalloc) return c.arena_flag;
  if (!c.dflag) {
    VMO_HIP(hipMalloc(&c.dflag, sizeof(int)));
    VMO_HIP(hipMemset(c.dflag, 0, sizeof(int)));
  }
  return c.dflag;
}

void check_device_flag(Ctx& c, hipStream_t s) {
  int* f = c.noalloc ? c.arena_flag : c.dflag;
  if (!f) return;
  const int v = read1(f, s);
  if (v) {
    VMO_HIP(hipMemsetAsync(f, 0, sizeof(int), s));
    VMO_HIP(hipStreamSynchronize(s));
    throw Error(VMO_E_DEVICE, "a device-side wait ran out of its bound (internal error)");
  }
}

template <class K>
void radix_sort(Ctx& c, K* keys, int32_t* vals, int64_t n, int bits, hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int passes = (bits + 7) / 8;
  // tiles of ri rounds: the target tile count is tuned online per size bucket
  // (fewer tiles: shorter look-back chains; more: more blocks in flight)
  static const int kTarget[8] = {4, 8, 16, 32, 64, 128, 256, 512};
  const int bucket = bits_for((uint64_t)n);
  bool tuned = false;
  const int cfg = n > (int64_t)4 * kRsT ? tune_pick(c, kTuneSort, bucket, 8, &tuned) : 7;
  int ri = 1;
  while (ri < kRsMaxI && n > (int64_t)kTarget[cfg] * kRsT * ri) ri *= 2;
  if (tuned) tune_begin_host(c, kTuneSort, bucket, cfg, (double)n * passes, s);
  const int64_t tile = (int64_t)kRsT * ri;
  const int64_t ntiles = (n + tile - 1) / tile;
  int* err = device_flag(c);
  Buf<K> k2(c.pool, n);
  Buf<int32_t> v2(c.pool, vals ? n : 1);
  // [passes][256] digit totals, [passes] tile counters, [passes][ntiles][256] words
  const size_t zbytes = sizeof(uint32_t) * (256 * 8 + 8) + sizeof(uint64_t) * (size_t)passes * ntiles * 256;
  Buf<uint8_t> z(c.pool, zbytes);
  uint32_t* ghist = reinterpret_cast<uint32_t*>(z.p);
  uint32_t* ctr = ghist + 256 * 8;
  uint64_t* status = reinterpret_cast<uint64_t*>(ctr + 8);
  VMO_HIP(hipMemsetAsync(z.p, 0, zbytes, s));
  const int64_t hb = (n + kRsT - 1) / kRsT;
  VMO_LAUNCH((k_rs_hist<K>), (unsigned)(hb < 512 ? hb : 512), kRsT, 0, s, keys, n, passes, ghist);
  K* ka = keys; K* kb = k2.p;
  int32_t* va = vals; int32_t* vb = vals ? v2.p : nullptr;
  for (int ps = 0; ps < passes; ++ps) {
#define VMO_RS_SCATTER(R)                                                                                     \
  VMO_LAUNCH((k_rs_scatter<K, R>), (unsigned)ntiles, kRsT, 0, s, ka, va, kb, vb, n, 8 * ps, ghist + 256 * ps, \
             status + (size_t)ps * ntiles * 256, ctr + ps, err)
    switch (ri) {
      case 1: VMO_RS_SCATTER(1); break;
      case 2: VMO_RS_SCATTER(2); break;
      case 4: VMO_RS_SCATTER(4); break;
      case 8: VMO_RS_SCATTER(8); break;
      default: VMO_RS_SCATTER(16); break;
    }
#undef VMO_RS_SCATTER
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    VMO_HIP(hipMemcpyAsync(keys, ka, sizeof(K) * n, hipMemcpyDeviceToDevice, s));
    if (vals) VMO_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  }
  if (tuned) tune_end(c, s);
}
template void radix_sort<uint32_t>(Ctx&, uint32_t*, int32_t*, int64_t, int, hipStream_t);
template void radix_sort<uint64_t>(Ctx&, uint64_t*, int32_t*, int64_t, int, hipStream_t);

// ----------------------------------------------------------------- fills ----
template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_iota(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}
static unsigned gs_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n > 0) VMO_LAUNCH(k_fill<int32_t>, gs_blocks(n), 256, 0, s, p, v, n);
}
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
  if (n > 0) VMO_LAUNCH(k_fill<int64_t>, gs_blocks(n), 256, 0, s, p, v, n);
}
void iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n > 0) VMO_LAUNCH(k_iota, gs_blocks(n), 256, 0, s, p, n);
}

// ------------------------------------------------------------ validation ----
__global__ void k_check_ptr(const int64_t* ptr, int32_t l, int* bad) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
    if (ptr[e + 1] < ptr[e]) atomicOr(bad, 1);
    if (e == 0 && ptr[0] != 0) atomicOr(bad, 1);
  }
}
// pins of net e: in range and strictly ascending (checked per pin with its
// predecessor inside the same net, net found by binary search)
// Pins of every net: in [0, k) and strictly ascending.  kChkG lanes per net
// (consecutive lanes read consecutive pins); a wavefront takes kChkRun runs of
// 64 / kChkG consecutive nets.
constexpr int kChkG = 16, kChkRun = 16, kChkPerWave = 64 / kChkG;
static unsigned chk_blocks(int64_t nets) {
  const int64_t waves = (nets + kChkPerWave * kChkRun - 1) / (kChkPerWave * kChkRun);
  return (unsigned)((waves + 3) / 4);  // blocks of 256 threads
}
__device__ __forceinline__ int check_net_pins(const int64_t* ptr, const int32_t* pins, int32_t k, int64_t e, int gl) {
  int flags = 0;
  const int64_t b = ptr[e], en = ptr[e + 1];
  for (int64_t p = b + gl; p < en; p += kChkG) {
    const int32_t v = pins[p];
    if (v < 0 || v >= k) flags |= 2;
    else if (p > b && pins[p - 1] >= v) flags |= 4;
  }
  return flags;
}
__global__ void k_check_pins(const int64_t* ptr, const int32_t* pins, int32_t l, int32_t k, int* bad) {
  const int gl = threadIdx.x & (kChkG - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t e0 = wave * kChkPerWave * kChkRun + ((threadIdx.x & 63) / kChkG);
  int flags = 0;
  for (int r = 0; r < kChkRun; ++r) {
    const int64_t e = e0 + (int64_t)r * kChkPerWave;
    if (e >= l) break;
    flags |= check_net_pins(ptr, pins, k, e, gl);
  }
  if (flags) atomicOr(bad, flags);
}
__global__ void k_check_vals(const float* v, int64_t n, int positive, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float a = v[i];
    if (!(a >= 0.0f) || !(a < __builtin_inff()) || (positive && !(a > 0.0f))) atomicOr(bad, 8);
  }
}
__global__ void k_check_finite(const float* v, int64_t n, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float a = v[i];
    if (!(a == a) || a == __builtin_inff() || a == -__builtin_inff()) atomicOr(bad, 16);
  }
}

void validate_hypergraph(Ctx& c, const vmo_hypergraph* h, bool positive_wc, hipStream_t s) {
  VMO_REQUIRE(h != nullptr, "hypergraph is NULL");
  VMO_REQUIRE(h->k >= 1, "hypergraph needs k >= 1");
  VMO_REQUIRE(h->l >= 0, "hypergraph needs l >= 0");
  VMO_REQUIRE(h->net_ptr != nullptr, "net_ptr is NULL");
  Buf<int> bad(c.pool, 1);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  if (h->l > 0) VMO_LAUNCH(k_check_ptr, gs_blocks(h->l), 256, 0, s, h->net_ptr, h->l, bad.p);
  int b0 = read1(bad.p, s);
  VMO_REQUIRE(b0 == 0, "net_ptr must start at 0 and be non-decreasing");
  int64_t np = read1(h->net_ptr + h->l, s);
  VMO_REQUIRE(np >= 0 && np < (int64_t(1) << 31) * 2, "too many pins");
  if (np > 0) {
    VMO_REQUIRE(h->pins != nullptr, "pins is NULL");
    VMO_LAUNCH(k_check_pins, chk_blocks(h->l), 256, 0, s, h->net_ptr, h->pins, h->l, h->k, bad.p);
  }
  if (h->w) VMO_LAUNCH(k_check_vals, gs_blocks(h->k), 256, 0, s, h->w, (int64_t)h->k, positive_wc ? 1 : 0, bad.p);
  if (h->c && h->l > 0) VMO_LAUNCH(k_check_vals, gs_blocks(h->l), 256, 0, s, h->c, (int64_t)h->l, positive_wc ? 1 : 0, bad.p);
  int b = read1(bad.p, s);
  VMO_REQUIRE(!(b & 2), "a pin is out of range [0, k)");
  VMO_REQUIRE(!(b & 4), "pins of a net must be strictly ascending");
  VMO_REQUIRE(!(b & 8), positive_wc ? "weights and costs must be finite and > 0" : "weights and costs must be finite and >= 0");
}

// ----------------------------------------------------- batched validation ----
// Checks of many jobs in one launch each: a table of jobs with cumulative
// element offsets; a thread finds its job by bisection.
struct CheckJob {
  const int64_t* ptr;
  const int32_t* pins;
  const float* w;
  const float* c;
  const float* x;
  int32_t k, l;
  int32_t graph, pad;
  int64_t np;
};
__device__ __forceinline__ int32_t job_of(const int64_t* cum, int32_t nj, int64_t i) {
  int32_t lo = 0, hi = nj;  // last j with cum[j] <= i
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    if (cum[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}
// pass 1: pointer arrays (start at 0, non-decreasing) over cum = prefix of l
__global__ void k_check_ptr_all(const CheckJob* jb, const int64_t* cum, int32_t nj, int64_t total, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = job_of(cum, nj, i);
    const int64_t e = i - cum[j];
    const int64_t* ptr = jb[j].ptr;
    if (ptr[e + 1] < ptr[e] || (e == 0 && ptr[0] != 0)) atomicOr(&bad[j], 1);
  }
}
// pass 2: pins of every net (range, ascending) over cum = prefix of l; a
// wavefront keeps the job range it found (its nets mostly share one job)
__global__ void k_check_pins_all(const CheckJob* jb, const int64_t* cum, int32_t nj, int64_t total, int* bad) {
  const int gl = threadIdx.x & (kChkG - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t i0 = wave * kChkPerWave * kChkRun + ((threadIdx.x & 63) / kChkG);
  int32_t j = -1;
  int64_t jlo = 0, jhi = 0;
  int flags = 0;
  for (int r = 0; r < kChkRun; ++r) {
    const int64_t i = i0 + (int64_t)r * kChkPerWave;
    if (i >= total) break;
    if (i < jlo || i >= jhi) {
      if (flags) atomicOr(&bad[j], flags);
      flags = 0;
      j = job_of(cum, nj, i);
      jlo = cum[j];
      jhi = j + 1 < nj ? cum[j + 1] : total;
    }
    const CheckJob& J = jb[j];
    flags |= check_net_pins(J.ptr, J.pins, J.k, i - jlo, gl);
  }
  if (flags) atomicOr(&bad[j], flags);
}
// pass 2: per vertex (weights, 4 coordinates) over cum = prefix of k
__global__ void k_check_vertices_all(const CheckJob* jb, const int64_t* cum, int32_t nj, int64_t total, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = job_of(cum, nj, i);
    const CheckJob& J = jb[j];
    const int64_t v = i - cum[j];
    if (J.w) {
      const float a = J.w[v];
      if (!(a >= 0.0f) || !(a < __builtin_inff())) atomicOr(&bad[j], 8);
    }
    if (J.x)
      for (int d = 0; d < 4; ++d) {
        const float a = J.x[(int64_t)d * J.k + v];
        if (!(a == a) || a == __builtin_inff() || a == -__builtin_inff()) atomicOr(&bad[j], 16);
      }
  }
}
// pass 2: per net (costs, graph-mode edge pointers) over cum = prefix of l + 1
__global__ void k_check_nets_all(const CheckJob* jb, const int64_t* cum, int32_t nj, int64_t total, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = job_of(cum, nj, i);
    const CheckJob& J = jb[j];
    const int64_t e = i - cum[j];  // 0..l
    if (J.c && e < J.l) {
      const float a = J.c[e];
      if (!(a >= 0.0f) || !(a < __builtin_inff())) atomicOr(&bad[j], 8);
    }
    if (J.graph && J.ptr[e] != 2 * e) atomicOr(&bad[j], 32);
  }
}
__global__ void k_net_ends_all(const CheckJob* jb, int32_t nj, int64_t* ends) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nj; j += gridDim.x * blockDim.x)
    ends[j] = jb[j].ptr[jb[j].l];
}

void validate_jobs(Ctx& c, const std::vector<JobCheck>& jobs, std::vector<int64_t>& npins, hipStream_t s) {
  const int32_t nj = (int32_t)jobs.size();
  npins.assign(nj, 0);
  std::vector<CheckJob> hj(nj);
  for (int32_t j = 0; j < nj; ++j) {
    const vmo_hypergraph* h = jobs[j].h;
    const std::string who = nj > 1 ? "job " + std::to_string(j) + ": " : "";
    VMO_REQUIRE(h != nullptr, who + "hypergraph is NULL");
    VMO_REQUIRE(h->k >= 1, who + "hypergraph needs k >= 1");
    VMO_REQUIRE(h->l >= 0, who + "hypergraph needs l >= 0");
    VMO_REQUIRE(h->net_ptr != nullptr, who + "net_ptr is NULL");
    VMO_REQUIRE(!jobs[j].x_required || jobs[j].x != nullptr, who + "x is NULL");
    hj[j] = CheckJob{h->net_ptr, h->pins, h->w, h->c, jobs[j].x, h->k, h->l, jobs[j].graph ? 1 : 0, 0, 0};
  }
  Buf<CheckJob> dj(c.pool, nj);
  Buf<int> bad(c.pool, nj);
  Buf<int64_t> ends(c.pool, nj), cum(c.pool, nj);
  std::vector<int64_t> hc(nj);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int) * nj, s));
  VMO_HIP(hipMemcpyAsync(dj.p, hj.data(), sizeof(CheckJob) * nj, hipMemcpyHostToDevice, s));
  // pass 1: pointer arrays and their ends
  int64_t tot = 0;
  for (int32_t j = 0; j < nj; ++j) { hc[j] = tot; tot += hj[j].l; }
  VMO_HIP(hipMemcpyAsync(cum.p, hc.data(), 8 * nj, hipMemcpyHostToDevice, s));
  if (tot > 0) VMO_LAUNCH(k_check_ptr_all, gs_blocks(tot), 256, 0, s, dj.p, cum.p, nj, tot, bad.p);
  VMO_LAUNCH(k_net_ends_all, (unsigned)((nj + 255) / 256), 256, 0, s, dj.p, nj, ends.p);
  std::vector<int> hb(nj);
  read_bytes(hb.data(), bad.p, sizeof(int) * nj, s);
  read_bytes(npins.data(), ends.p, sizeof(int64_t) * nj, s);
  for (int32_t j = 0; j < nj; ++j) {
    const std::string who = nj > 1 ? "job " + std::to_string(j) + ": " : "";
    VMO_REQUIRE(hb[j] == 0, who + "net_ptr must start at 0 and be non-decreasing");
    VMO_REQUIRE(npins[j] >= 0 && npins[j] < (int64_t(1) << 31) * 2, who + "too many pins");
    VMO_REQUIRE(npins[j] == 0 || jobs[j].h->pins != nullptr, who + "pins is NULL");
    hj[j].np = npins[j];
  }
  VMO_HIP(hipMemcpyAsync(dj.p, hj.data(), sizeof(CheckJob) * nj, hipMemcpyHostToDevice, s));
  // pass 2: pins, then vertices (weights, coordinates), then nets (costs, edges)
  Buf<int64_t> cum3(c.pool, nj), cum4(c.pool, nj);
  std::vector<int64_t> h3(nj), h4(nj);
  int64_t t2 = 0, t3 = 0, t4 = 0;
  for (int32_t j = 0; j < nj; ++j) {
    t2 += npins[j];
    h3[j] = t3; t3 += hj[j].k;
    h4[j] = t4; t4 += (int64_t)hj[j].l + 1;
  }
  VMO_HIP(hipMemcpyAsync(cum3.p, h3.data(), 8 * nj, hipMemcpyHostToDevice, s));
  VMO_HIP(hipMemcpyAsync(cum4.p, h4.data(), 8 * nj, hipMemcpyHostToDevice, s));
  // (pins are checked net by net: over the prefix of l, as pass 1)
  if (t2 > 0 && tot > 0) VMO_LAUNCH(k_check_pins_all, chk_blocks(tot), 256, 0, s, dj.p, cum.p, nj, tot, bad.p);
  VMO_LAUNCH(k_check_vertices_all, gs_blocks(t3), 256, 0, s, dj.p, cum3.p, nj, t3, bad.p);
  VMO_LAUNCH(k_check_nets_all, gs_blocks(t4), 256, 0, s, dj.p, cum4.p, nj, t4, bad.p);
  read_bytes(hb.data(), bad.p, sizeof(int) * nj, s);
  for (int32_t j = 0; j < nj; ++j) {
    const std::string who = nj > 1 ? "job " + std::to_string(j) + ": " : "";
    const int b = hb[j];
    VMO_REQUIRE(!(b & 2), who + "a pin is out of range [0, k)");
    VMO_REQUIRE(!(b & 4), who + "pins of a net must be strictly ascending");
    VMO_REQUIRE(!(b & 8), who + "weights and costs must be finite and >= 0");
    VMO_REQUIRE(!(b & 16), who + "x must be finite");
    VMO_REQUIRE(!(b & 32), who + "graph mode needs every net to be an edge {v, w}");
  }
}

void validate_finite(Ctx& c, const float* x, int64_t n, const char* what, hipStream_t s) {
  VMO_REQUIRE(x != nullptr, std::string(what) + " is NULL");
  Buf<int> bad(c.pool, 1);
  VMO_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  if (n > 0) VMO_LAUNCH(k_check_finite, gs_blocks(n), 256, 0, s, x, n, bad.p);
  VMO_REQUIRE(read1(bad.p, s) == 0, std::string(what) + " must be finite");
}

// -------------------------------------------------------------- transpose ----
__global__ void k_row_of(const int64_t* ptr, int32_t nrows, int64_t np, int32_t* row) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nrows;
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (ptr[mid] <= p) lo = mid; else hi = mid;
    }
    row[p] = lo;
  }
}
__global__ void k_count_cols(const int32_t* idx, int64_t np, int64_t* cnt) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd((unsigned long long*)&cnt[idx[p]], 1ull);
}
__global__ void k_widen(const int32_t* in, uint32_t* out, int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    out[p] = (uint32_t)in[p];
}

void csr_transpose(Ctx& c, int32_t nrows, int32_t ncols, const int64_t* ptr, const int32_t* idx,
                   int64_t* optr, int32_t* oidx, hipStream_t s) {
  int64_t np = read1(ptr + nrows, s);
  Buf<int64_t> cnt(c.pool, (size_t)ncols + 1);
  fill_i64(cnt.p, 0, (int64_t)ncols + 1, s);
  if (np > 0) {
    VMO_LAUNCH(k_count_cols, gs_blocks(np), 256, 0, s, idx, np, cnt.p);
    Buf<uint32_t> key(c.pool, np);
    VMO_LAUNCH(k_widen, gs_blocks(np), 256, 0, s, idx, key.p, np);
    VMO_LAUNCH(k_row_of, gs_blocks(np), 256, 0, s, ptr, nrows, np, oidx);
    radix_sort<uint32_t>(c, key.p, oidx, np, bits_for((uint64_t)(ncols > 0 ? ncols - 1 : 0)), s);
  }
  scan_exclusive<int64_t>(c, cnt.p, optr, ncols, optr + ncols, s);
}

// ------------------------------------------------------------- components ----
__device__ __forceinline__ int32_t uf_parent(int32_t* par, int32_t x) {
  return __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Root of x with path halving: a vertex that is not a root is pointed at its
// grandparent (still one of its ancestors; links only ever change roots, so
// the shortcut never undoes a link) and the search continues from there.
__device__ __forceinline__ int32_t uf_find(int32_t* par, int32_t x) {
  while (true) {
    const int32_t p = uf_parent(par, x);
    if (p == x) return x;
    const int32_t gp = uf_parent(par, p);
    if (gp == p) return p;
    __hip_atomic_store(&par[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}
// Link the pins of each net (consecutive pairs) into one tree; a root is
// always hooked under a smaller root, so every final root is its tree's
// smallest vertex -- the union step of Algorithm 1.
__global__ void k_cc_union(const int64_t* ptr, const int32_t* pins, int32_t l, int32_t* par) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = ptr[e], en = ptr[e + 1];
    for (int64_t p = b + 1; p < en; ++p) {
      int32_t a = pins[p - 1], bb = pins[p];
      while (true) {
        a = uf_find(par, a);
        bb = uf_find(par, bb);
        if (a == bb) break;
        if (a > bb) { int32_t t = a; a = bb; bb = t; }
        int32_t old = atomicCAS(&par[bb], bb, a);
        if (old == bb) break;
        bb = old;
      }
    }
  }
}
// Hooking rounds before the union-find: every net's consecutive pins (a, b)
// lower the parent of the larger of their current parents to the smaller one
// (atomicMin), then every vertex points at the end of its parent chain.
// Parents only decrease and stay in the vertex's component, so par[v] <= v
// holds throughout; after a round without a decrease the ends agree along
// every net, so every component points at its smallest vertex.
__global__ void k_cc_hook(const int64_t* ptr, const int32_t* pins, int32_t l, int32_t* par, int32_t* changed) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < l; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = ptr[e], en = ptr[e + 1];
    for (int64_t p = b + 1; p < en; ++p) {
      const int32_t ra = par[pins[p - 1]], rb = par[pins[p]];
      if (ra == rb) continue;
      const int32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
      if (atomicMin(&par[hi], lo) > lo) *changed = 1;
    }
  }
}
__global__ void k_cc_jump(int32_t* par, int32_t k) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t p = par[v], g = par[p];
    while (g != p) {  // strictly decreasing ids: ends
      p = g;
      g = par[p];
    }
    par[v] = p;
  }
}
__global__ void k_cc_final(int32_t* par, int32_t k, int32_t* label) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < k; v += (int64_t)gridDim.x * blockDim.x)
    label[v] = uf_find(par, (int32_t)v);
}

void components(Ctx& c, int32_t k, int32_t l, const int64_t* ptr, const int32_t* pins, int32_t* label,
                hipStream_t s) {
  Buf<int32_t> par(c.pool, k);
  iota_i32(par.p, k, s);
  if (l > 0) {
    // up to kHookRounds hooking rounds (one host check each); the union-find
    // then finishes from the forest they leave (at once if they converged)
    constexpr int kHookRounds = 32;
    Buf<int32_t> changed(c.pool, 1);
    for (int r = 0; r < kHookRounds; ++r) {
      fill_i32(changed.p, 0, 1, s);
      VMO_LAUNCH(k_cc_hook, gs_blocks(l), 256, 0, s, ptr, pins, l, par.p, changed.p);
      VMO_LAUNCH(k_cc_jump, gs_blocks(k), 256, 0, s, par.p, k);
      if (read1(changed.p, s) == 0) break;
    }
    VMO_LAUNCH(k_cc_union, gs_blocks(l), 256, 0, s, ptr, pins, l, par.p);
  }
  VMO_LAUNCH(k_cc_final, gs_blocks(k), 256, 0, s, par.p, k, label);
}

}  // namespace vmo
