// C ABI of include/vmo.h: argument checks, context handling, and dispatch to
// the device code.  No exception crosses this boundary.
#include <algorithm>
#include <climits>

#include "order_engine.h"

struct vmo_ctx_s : vmo::Ctx {};

namespace vmo {
void model(Ctx& c, int model, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, int64_t* net_ptr,
           int32_t* pins, int32_t cap_nets, int64_t cap_pins, int32_t* k_out, int32_t* l_out, int64_t* np_out,
           hipStream_t s);
void dual(Ctx& c, const vmo_hypergraph* h, int64_t* dptr, int32_t* dpins, hipStream_t s);
void cut(Ctx& c, const vmo_hypergraph* h, const int32_t* part, int32_t nparts, double* part_weight,
         vmo_cut_result* out, hipStream_t s);
void layout(Ctx& c, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, hipStream_t s);
void coarsen(Ctx& c, const vmo_hypergraph* h, uint64_t seed, uint64_t comp, int32_t level, int32_t match_max,
             int32_t* pi, int64_t* cptr, int32_t* cpins, float* cw, float* cc, int32_t* kc, int32_t* lc,
             hipStream_t s);
void tree(Ctx& c, const float* x, const float* w, int32_t k, int32_t cap, int32_t* ints, int32_t* cell2, float* flt,
          int32_t* order, int32_t max_nodes, int32_t* n_nodes, hipStream_t s);
void gradient(Ctx& c, const vmo_hypergraph* h, const float* x, float theta, int32_t cap, float* y, float* z,
              int64_t* nint, hipStream_t s);
void layout_steps(Ctx& c, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, int32_t it0, int32_t iters,
                  double* alpha, hipStream_t s);
void order_border(Ctx& c, const vmo_hypergraph* h, const vmo_order_out* in, int32_t P, int32_t b, int32_t* vperm_out,
                  hipStream_t s);
void order_schur(Ctx& c, const vmo_hypergraph* h, const float* x, const int32_t* mu, const vmo_order_out* in,
                 int32_t P, int32_t P3, uint64_t seed, int32_t t_max, int32_t* vperm_out, hipStream_t s);
void match(Ctx& c, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* a, uint32_t seed,
           int augment, int32_t* mrow, int32_t* mcol, int32_t* mu, int64_t* size_out, hipStream_t s);
void validate_mu(Ctx& c, const vmo_hypergraph* h, const int32_t* mu, hipStream_t s);
void matched_perms(Ctx& c, int32_t m, const int32_t* vperm, const int32_t* mu, int32_t* rperm, int32_t* cperm,
                   hipStream_t s);
void finegrain(Ctx& c, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* x, float* xnz,
               hipStream_t s);
void refine_kl(Ctx& c, const vmo_hypergraph* h, int32_t* label, int32_t passes, int64_t* gain, int32_t* ngroups,
               hipStream_t s);
}  // namespace vmo

// Every call first waits for the work of the last asynchronous call if that
// ran on another stream (its pool blocks are then idle).
#define API_BEGIN(ctx, stream)                                    \
  if (!(ctx)) return VMO_E_INVALID;                               \
  vmo::Ctx& C = *static_cast<vmo::Ctx*>(ctx);                     \
  hipStream_t S = static_cast<hipStream_t>(stream);               \
  C.err.clear();                                                  \
  try {                                                           \
    VMO_HIP(hipSetDevice(C.device));                              \
    vmo::join_tail(C, S);

#define API_CATCH                                                 \
  catch (vmo::Error & e) {                                        \
    C.err = e.what();                                             \
    (void)hipStreamSynchronize(S);                                \
    (void)hipGetLastError();                                      \
    C.tail_on = false;                                            \
    vmo::prof_discard(C);                                         \
    return e.status;                                              \
  }                                                               \
  catch (std::exception & e) {                                    \
    C.err = e.what();                                             \
    (void)hipStreamSynchronize(S);                                \
    (void)hipGetLastError();                                      \
    C.tail_on = false;                                            \
    vmo::prof_discard(C);                                         \
    return VMO_E_DEVICE;                                          \
  }                                                               \
  return VMO_OK;

// A call that returns after its work is done (it has host outputs).
#define API_END                                                   \
    vmo::check_device_flag(C, S);                                 \
    vmo::prof_flush(C);                                           \
    vmo::tune_flush(C);                                           \
    vmo::trim_pool(C, S);                                         \
  }                                                               \
  API_CATCH

// A call whose outputs are device arrays: it returns once its work is
// queued (after whatever readbacks it needs on the way); vmo_sync reports
// what its device-side checks found.  With live timing on it waits, as the
// timings are read at its end.
#define API_END_ASYNC                                             \
    if (C.prof.on) {                                              \
      vmo::check_device_flag(C, S);                               \
      vmo::prof_flush(C);                                         \
    }                                                             \
    vmo::tune_flush(C);                                           \
    vmo::mark_tail(C, S);                                         \
  }                                                               \
  API_CATCH

extern "C" {

vmo_status vmo_create(vmo_ctx* out, int device, size_t pool_bytes) {
  if (!out) return VMO_E_INVALID;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return VMO_E_DEVICE;
  }
  vmo_ctx_s* c = new (std::nothrow) vmo_ctx_s();
  if (!c) return VMO_E_NOMEM;
  c->device = device;
  c->pool_cap = pool_bytes;
  // the allocation-free entry point's arena: its address on this device,
  // looked up once per device with the device current (the caller's current
  // device is restored)
  int prev = 0;
  const bool have_prev = hipGetDevice(&prev) == hipSuccess;
  if (hipSetDevice(device) == hipSuccess) vmo::noalloc_init(device);
  if (have_prev) (void)hipSetDevice(prev);
  (void)hipGetLastError();
  *out = c;
  return VMO_OK;
}

vmo_status vmo_destroy(vmo_ctx ctx) {
  if (!ctx) return VMO_E_INVALID;
  (void)hipSetDevice(ctx->device);
  if (ctx->tail_on) (void)hipEventSynchronize(ctx->tail);  // pending work still uses pool blocks
  delete ctx;
  return VMO_OK;
}

vmo_status vmo_sync(vmo_ctx ctx, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  VMO_HIP(hipStreamSynchronize(S));
  C.tail_on = false;
  vmo::check_async_flag(C, S);
  API_END
}

const char* vmo_last_error(vmo_ctx ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

size_t vmo_pool_bytes(vmo_ctx ctx) { return ctx ? ctx->pool.held() : 0; }

vmo_status vmo_model(vmo_ctx ctx, int model, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col,
                     int64_t* net_ptr, int32_t* pins, int32_t cap_nets, int64_t cap_pins, int32_t* k, int32_t* l,
                     int64_t* npins, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::model(C, model, m, n, rowptr, col, net_ptr, pins, cap_nets, cap_pins, k, l, npins, S);
  API_END
}

vmo_status vmo_dual(vmo_ctx ctx, const vmo_hypergraph* h, int64_t* dptr, int32_t* dpins, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::dual(C, h, dptr, dpins, S);
  API_END_ASYNC
}

vmo_status vmo_components(vmo_ctx ctx, const vmo_hypergraph* h, int32_t* label, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::validate_hypergraph(C, h, false, S);
  VMO_REQUIRE(label != nullptr, "label is NULL");
  vmo::components(C, h->k, h->l, h->net_ptr, h->pins, label, S);
  API_END_ASYNC
}

vmo_status vmo_cut(vmo_ctx ctx, const vmo_hypergraph* h, const int32_t* part, int32_t nparts, double* part_weight,
                   vmo_cut_result* out, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::cut(C, h, part, nparts, part_weight, out, S);
  API_END
}

vmo_status vmo_cut_noalloc(vmo_ctx ctx, const vmo_hypergraph* h, const int32_t* part, int32_t nparts,
                           double* part_weight, vmo_cut_result* out, vmo_stream stream) {
  if (!ctx) return VMO_E_INVALID;
  vmo::Ctx& C = *static_cast<vmo::Ctx*>(ctx);
  hipStream_t S = static_cast<hipStream_t>(stream);
  C.err.clear();
  try {
    VMO_HIP(hipSetDevice(C.device));
    vmo::cut_noalloc(C, h, part, nparts, part_weight, out, S);
  } catch (vmo::Error& e) {
    C.err = e.what();
    (void)hipStreamSynchronize(S);
    (void)hipGetLastError();
    return e.status;
  } catch (std::exception& e) {
    C.err = e.what();
    (void)hipStreamSynchronize(S);
    (void)hipGetLastError();
    return VMO_E_DEVICE;
  }
  return VMO_OK;
}

vmo_status vmo_bisect(vmo_ctx ctx, const float* x, int32_t k, uint64_t seed, int32_t t_max, uint8_t* side,
                      float* centres, int32_t* iters, int32_t* split, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  VMO_REQUIRE(k >= 1, "k must be >= 1");
  VMO_REQUIRE(t_max >= 0, "t_max must be >= 0");
  VMO_REQUIRE(side && centres && iters && split, "NULL output");
  vmo::validate_finite(C, x, 4 * (int64_t)k, "x", S);
  std::vector<vmo::JobHost> jobs(1);
  memset(&jobs[0], 0, sizeof(vmo::JobHost));
  jobs[0].h.k = k;
  jobs[0].mode = VMO_NET;
  jobs[0].order = VMO_SBD;
  jobs[0].x = x;
  jobs[0].P = 2;
  jobs[0].seed = seed;
  jobs[0].job_index = 0;
  vmo::Engine e(C, S);
  e.setup(jobs);
  int sp = 0, it = 0;
  if (e.S > 0) {
    e.two_means(0, e.S, 0, e.Np, t_max, true);
    int32_t st = vmo::read1(e.cur.state.p, S);
    sp = st == vmo::kStDone ? 1 : 0;
    it = vmo::read1(e.cur.iters.p, S);
  }
  vmo::bisect_outputs(e, side, centres, sp);
  VMO_HIP(hipStreamSynchronize(S));
  *iters = sp ? it : 0;
  *split = sp;
  API_END
}

// Host checks of an ordering job's scalars and output pointers.
static void check_order_scalars(int mode, int order, int32_t P, int32_t t_max, const vmo_order_out* out) {
  VMO_REQUIRE(mode == VMO_NET || mode == VMO_GRAPH, "mode must be VMO_NET or VMO_GRAPH");
  VMO_REQUIRE(order == VMO_SBD || order == VMO_BBD, "order must be VMO_SBD or VMO_BBD");
  VMO_REQUIRE(P >= 1 && P <= (1 << 24), "P must be in [1, 2^24]");
  VMO_REQUIRE(t_max >= 0, "t_max must be >= 0");
  VMO_REQUIRE(out && out->vperm && out->part && out->node_heap && out->node_vptr && out->split_cut && out->n_nodes,
              "NULL output array");
}

static void run_order(vmo::Ctx& C, std::vector<vmo::JobHost>& jobs, const std::vector<int64_t>& npins, int32_t t_max,
                      bool plain, hipStream_t S) {
  vmo::Engine e(C, S);
  e.setup(jobs);
  e.set_edges(jobs, npins);
  e.run_levels(t_max, plain);
  e.finish(jobs);
}

vmo_status vmo_order(vmo_ctx ctx, const vmo_hypergraph* h, int mode, int order, const float* x,
                     const vmo_layout_params* lp, int32_t P, uint64_t seed, int32_t t_max, const vmo_order_out* out,
                     vmo_stream stream) {
  API_BEGIN(ctx, stream)
  check_order_scalars(mode, order, P, t_max, out);
  VMO_REQUIRE(x || lp, "x is NULL and no layout parameters were given");
  std::vector<int64_t> npins;
  vmo::validate_jobs(C, {vmo::JobCheck{h, x, false, mode == VMO_GRAPH}}, npins, S);
  vmo::Buf<float> xl;
  if (!x) {
    xl = vmo::Buf<float>(C.pool, 4 * (size_t)h->k);
    vmo::layout(C, h, lp, xl.p, S);
    x = xl.p;
  }
  std::vector<vmo::JobHost> jobs(1);
  memset(&jobs[0], 0, sizeof(vmo::JobHost));
  jobs[0].h = *h;
  jobs[0].mode = mode;
  jobs[0].order = order;
  jobs[0].x = x;
  jobs[0].P = P;
  jobs[0].seed = seed;
  jobs[0].job_index = 0;
  jobs[0].out = *out;
  run_order(C, jobs, npins, t_max, false, S);
  API_END_ASYNC
}

vmo_status vmo_order_sbd(vmo_ctx ctx, const vmo_hypergraph* h, int mode, const float* x, const vmo_layout_params* lp,
                         int32_t P, uint64_t seed, int32_t t_max, const vmo_order_out* out, vmo_stream stream) {
  return vmo_order(ctx, h, mode, VMO_SBD, x, lp, P, seed, t_max, out, stream);
}
vmo_status vmo_order_bbd(vmo_ctx ctx, const vmo_hypergraph* h, int mode, const float* x, const vmo_layout_params* lp,
                         int32_t P, uint64_t seed, int32_t t_max, const vmo_order_out* out, vmo_stream stream) {
  return vmo_order(ctx, h, mode, VMO_BBD, x, lp, P, seed, t_max, out, stream);
}

vmo_status vmo_order_border(vmo_ctx ctx, const vmo_hypergraph* h, const vmo_order_out* in, int32_t P, int32_t b,
                            int32_t* vperm_out, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::order_border(C, h, in, P, b, vperm_out, S);
  API_END_ASYNC
}

vmo_status vmo_order_schur(vmo_ctx ctx, const vmo_hypergraph* h, const float* x, const int32_t* mu,
                           const vmo_order_out* in, int32_t P, int32_t P3, uint64_t seed, int32_t t_max,
                           int32_t* vperm_out, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::order_schur(C, h, x, mu, in, P, P3, seed, t_max, vperm_out, S);
  API_END_ASYNC
}

vmo_status vmo_match(vmo_ctx ctx, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* a,
                     uint32_t seed, int augment, int32_t* mrow, int32_t* mcol, int32_t* mu, int64_t* size,
                     vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::match(C, m, n, rowptr, col, a, seed, augment, mrow, mcol, mu, size, S);
  API_END
}

vmo_status vmo_order_matched(vmo_ctx ctx, const vmo_hypergraph* h, int order, const float* x,
                             const vmo_layout_params* lp, const int32_t* mu, int32_t P, uint64_t seed, int32_t t_max,
                             const vmo_order_out* out, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  check_order_scalars(VMO_GRAPH, order, P, t_max, out);
  VMO_REQUIRE(x || lp, "x is NULL and no layout parameters were given");
  std::vector<int64_t> npins;
  vmo::validate_jobs(C, {vmo::JobCheck{h, x, false, true}}, npins, S);
  vmo::validate_mu(C, h, mu, S);
  vmo::Buf<float> xl;
  if (!x) {
    xl = vmo::Buf<float>(C.pool, 4 * (size_t)h->k);
    vmo::layout(C, h, lp, xl.p, S);
    x = xl.p;
  }
  std::vector<vmo::JobHost> jobs(1);
  memset(&jobs[0], 0, sizeof(vmo::JobHost));
  jobs[0].h = *h;
  jobs[0].mode = VMO_GRAPH;
  jobs[0].order = order;
  jobs[0].x = x;
  jobs[0].P = P;
  jobs[0].seed = seed;
  jobs[0].job_index = 0;
  jobs[0].out = *out;
  jobs[0].mu = mu;
  run_order(C, jobs, npins, t_max, false, S);
  API_END_ASYNC
}

vmo_status vmo_matched_perms(vmo_ctx ctx, int32_t m, const int32_t* vperm, const int32_t* mu, int32_t* rperm,
                             int32_t* cperm, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::matched_perms(C, m, vperm, mu, rperm, cperm, S);
  API_END_ASYNC
}

vmo_status vmo_refine_kl(vmo_ctx ctx, const vmo_hypergraph* h, int32_t* label, int32_t passes, int64_t* gain,
                         int32_t* ngroups, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::refine_kl(C, h, label, passes, gain, ngroups, S);
  API_END_ASYNC
}

vmo_status vmo_finegrain(vmo_ctx ctx, int32_t m, int32_t n, const int64_t* rowptr, const int32_t* col, const float* x,
                         float* xnz, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::finegrain(C, m, n, rowptr, col, x, xnz, S);
  API_END_ASYNC
}

static vmo_status order_batch(vmo_ctx ctx, int32_t njobs, const vmo_job* jobs, int32_t t_max, bool plain,
                              vmo_stream stream) {
  API_BEGIN(ctx, stream)
  VMO_REQUIRE(njobs >= 1 && jobs != nullptr, "need at least one job");
  std::vector<vmo::JobHost> J(njobs);
  std::vector<vmo::JobCheck> chk(njobs);
  for (int32_t i = 0; i < njobs; ++i) {
    const vmo_job& a = jobs[i];
    check_order_scalars(a.mode, a.order, a.P, t_max, &a.out);
    chk[i] = vmo::JobCheck{&a.h, a.x, true, a.mode == VMO_GRAPH};
  }
  std::vector<int64_t> npins;
  vmo::validate_jobs(C, chk, npins, S);
  for (int32_t i = 0; i < njobs; ++i) {
    const vmo_job& a = jobs[i];
    memset(&J[i], 0, sizeof(vmo::JobHost));
    J[i].h = a.h;
    J[i].mode = a.mode;
    J[i].order = a.order;
    J[i].x = a.x;
    J[i].P = a.P;
    J[i].seed = a.seed;
    J[i].job_index = a.job_index;
    J[i].out = a.out;
  }
  run_order(C, J, npins, t_max, plain, S);
  API_END_ASYNC
}

vmo_status vmo_order_batch(vmo_ctx ctx, int32_t njobs, const vmo_job* jobs, int32_t t_max, vmo_stream stream) {
  return order_batch(ctx, njobs, jobs, t_max, false, stream);
}
vmo_status vmo_order_batch_plain(vmo_ctx ctx, int32_t njobs, const vmo_job* jobs, int32_t t_max, vmo_stream stream) {
  return order_batch(ctx, njobs, jobs, t_max, true, stream);
}

void vmo_layout_defaults(vmo_layout_params* p, uint64_t seed) {
  if (!p) return;
  p->seed = seed;
  p->coarsest_iters = 100;
  p->level_iters = 30;
  p->min_coarse = 64;
  p->max_levels = 40;
  p->leaf_cap = 8;
  p->match_max_net = 64;
  p->theta = 0.5f;
  p->step0_frac = 0.1f;
  p->decay = 0.9f;
  p->jitter = 1e-3f;
  p->stall = 0.95f;
  p->pack_gap = 0.1f;
}

size_t vmo_layout_bytes(int32_t k, int32_t l, int64_t npins) {
  if (k < 0 || l < 0 || npins < 0) return 0;
  // What the pool holds after a layout: the tree's node arrays, requested
  // once for the largest level (17 nodes per point: 80 B record, FP64 charges
  // 40 B, child lists 64 B, counts 8 B), the walk's parts, requested once for
  // the most any level needs (4 KiB per point up to 200,000 points, 256 B
  // above), per point the descent's records (32 B) and coarsening scratch
  // (64 B); per level the tree's point arrays (70 B), 16 B per vertex, 12 B
  // per net and 8 B per pin (x 2.5 for all levels, which shrink about twofold
  // each); the layout's own 16 B per net and 24 B per pin; and a quarter more
  // for the pool's size classes.
  const double kd = (double)k, ld = (double)l, pd = (double)npins;
  const double parts = std::max(256.0 * kd, 4096.0 * std::min(kd, 300000.0));
  const double per_v = 17.0 * 192.0 + 32.0 + 64.0 + 2.5 * (70.0 + 16.0);
  const double lvl = 2.5 * (12.0 * ld + 8.0 * pd);
  return (size_t)(1.25 * (kd * per_v + parts + lvl + 16.0 * ld + 24.0 * pd)) + ((size_t)1 << 20);
}

vmo_status vmo_layout(vmo_ctx ctx, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::layout(C, h, p, x, S);
  API_END_ASYNC
}

vmo_status vmo_coarsen(vmo_ctx ctx, const vmo_hypergraph* h, uint64_t seed, uint64_t comp, int32_t level,
                       int32_t match_max_net, int32_t* pi, int64_t* cptr, int32_t* cpins, float* cw, float* cc,
                       int32_t* kc, int32_t* lc, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::coarsen(C, h, seed, comp, level, match_max_net, pi, cptr, cpins, cw, cc, kc, lc, S);
  API_END
}

vmo_status vmo_tree(vmo_ctx ctx, const float* x, const float* w, int32_t k, int32_t leaf_cap, int32_t* ints,
                    int32_t* cell2, float* flt, int32_t* order, int32_t max_nodes, int32_t* n_nodes,
                    vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::tree(C, x, w, k, leaf_cap, ints, cell2, flt, order, max_nodes, n_nodes, S);
  API_END_ASYNC
}

vmo_status vmo_gradient(vmo_ctx ctx, const vmo_hypergraph* h, const float* x, float theta, int32_t leaf_cap, float* y,
                        float* z, int64_t* interactions, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::gradient(C, h, x, theta, leaf_cap, y, z, interactions, S);
  API_END_ASYNC
}

vmo_status vmo_layout_steps(vmo_ctx ctx, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, int32_t it0,
                            int32_t iters, double* alpha, vmo_stream stream) {
  API_BEGIN(ctx, stream)
  vmo::layout_steps(C, h, p, x, it0, iters, alpha, S);
  API_END_ASYNC
}

vmo_status vmo_profile(vmo_ctx ctx, int every) {
  if (!ctx || every == INT_MIN) return VMO_E_INVALID;
  ctx->prof.on = every != 0;
  ctx->prof.every = every > 0 ? every : (every < 0 ? -every : 1);
  ctx->prof.count = every >= 0;
  ctx->prof.seen.clear();
  if (!every) {
    vmo::prof_discard(*ctx);
    ctx->prof.acc.clear();
  }
  return VMO_OK;
}

vmo_status vmo_profile_read(vmo_ctx ctx, const char* kernel, vmo_profile_entry* out) {
  if (!ctx || !kernel || !out) return VMO_E_INVALID;
  auto it = ctx->prof.acc.find(kernel);
  if (it == ctx->prof.acc.end()) {
    out->total_ms = 0.0;
    out->launches = 0;
    out->work = 0.0;
    return VMO_OK;
  }
  out->total_ms = it->second.ms;
  out->launches = it->second.launches;
  out->work = it->second.work;
  return VMO_OK;
}

vmo_status vmo_profile_reset(vmo_ctx ctx) {
  if (!ctx) return VMO_E_INVALID;
  ctx->prof.acc.clear();
  return VMO_OK;
}

}  // extern "C"
