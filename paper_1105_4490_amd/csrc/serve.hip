// Serving loop: continuous batching of ordering jobs on one GPU.
//
// A worker thread owns a context, a HIP stream and an engine whose arrays are
// fixed arenas sized from the memory budget.  Jobs are admitted, in arrival
// order, when a slot and contiguous ranges of every arena (vertices, tree
// nodes, edges, nets, pins) are free; their matrix state then stays resident
// in the arenas.  Each tick runs one recursion level for the segments of every
// resident job in the same launches; jobs admitted meanwhile join at the next
// tick, and a job whose last segment finished is emitted and leaves, freeing
// its ranges.  Jobs that come without coordinates are laid out by a set of
// layout threads, each with its own context and stream, so several layouts
// run on the device at once and beside the ticks; a laid-out job joins the
// engine at the next tick.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "order_engine.h"

namespace vmo {
void layout(Ctx& c, const vmo_hypergraph* h, const vmo_layout_params* p, float* x, hipStream_t s);

// First-fit allocator of contiguous ranges of [0, cap).
class Ranges {
 public:
  void init(int64_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  bool alloc(int64_t n, int64_t* off) {
    if (n == 0) { *off = 0; return true; }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        int64_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest > 0) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(int64_t off, int64_t n) {
    if (n == 0) return;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t cap() const { return cap_; }

 private:
  int64_t cap_ = 0;
  std::map<int64_t, int64_t> free_;
};

struct Ticket {
  vmo_job job;
  bool layout = false;
  vmo_layout_params lp;
  int state = 0;  // 0 pending, 1 resident, 2 done
  vmo_status status = VMO_OK;
  std::string err;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int32_t slot = -1;
  int64_t voff = 0, nbase = 0, eoff = 0, noff = 0, poff = 0, npins = 0;
  int64_t lbytes = 0;  // estimated layout footprint while the layout is in flight
  Buf<float> xbuf;
};

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace vmo

struct vmo_layout_worker {
  vmo::Ctx ctx;  // its pool holds the workspace of the layouts it runs
  hipStream_t stream = nullptr;
  std::thread th;
};

struct vmo_server_s {
  vmo::Ctx ctx;
  hipStream_t stream = nullptr;
  vmo::Engine* eng = nullptr;
  vmo_serve_params prm;
  vmo::Ranges rv, rn, re, rl, rp;
  std::vector<int32_t> free_slots;
  std::thread worker;
  std::vector<vmo_layout_worker*> lw;
  std::mutex mu;
  std::condition_variable cv, done_cv, lcv;
  std::deque<uint64_t> pending;
  std::deque<uint64_t> lqueue;  // admitted, waiting for a layout thread
  std::deque<uint64_t> ready;   // laid out, waiting to join the engine
  std::deque<std::pair<uint64_t, std::pair<vmo_status, std::string>>> lfailed;
  bool blocked = false;         // the head of `pending` did not fit; cleared when ranges are released
  std::map<uint64_t, vmo::Ticket> tickets;
  std::vector<uint64_t> resident;
  uint64_t next_id = 1;
  bool stop = false;
  std::string fatal;
  vmo_serve_stats st;
  // layouts: their workspace is counted against lbudget (half for the
  // layouts in flight, by their estimated footprint; half for the blocks the
  // layout contexts keep cached between layouts)
  int64_t lbudget = 0, lbusy = 0;
};

namespace vmo {

// The budget: 40 % for the ordering arenas, 60 % for the layouts of jobs
// that come without coordinates.
constexpr double kArenaShare = 0.40;

// Arena capacities from the budget: per vertex 4 x 4 B grid coordinates
// twice, ids, positions, segment ids, sides and per-level scratch (~100 B);
// per tree node 24 B; per edge 8 B; per net 8 B; per pin 4 B.
static void arena_sizes(const vmo_serve_params& p, int64_t* V, int64_t* NTn, int64_t* En, int64_t* Ln, int64_t* Pn) {
  double b = (double)p.budget_bytes * kArenaShare;
  int64_t v = (int64_t)(b * 0.40 / 100.0);
  *V = v;
  *NTn = (int64_t)(b * 0.05 / 24.0);
  *En = (int64_t)(b * 0.25 / 8.0);
  *Ln = (int64_t)(b * 0.10 / 8.0);
  *Pn = (int64_t)(b * 0.20 / 4.0);
}

static bool try_admit(vmo_server_s* S, Ticket& T, int64_t npins) {
  const vmo_job& J = T.job;
  if (S->free_slots.empty()) return false;
  const int64_t lf = T.layout ? (int64_t)vmo_layout_bytes(J.h.k, J.h.l, npins) : 0;
  if (T.layout && S->lbusy + lf > S->lbudget / 2) return false;
  int64_t voff, nb, eo = 0, no = 0, po = 0;
  if (!S->rv.alloc(J.h.k, &voff)) return false;
  if (!S->rn.alloc(4 * (int64_t)J.P, &nb)) { S->rv.release(voff, J.h.k); return false; }
  bool ok = true;
  if (J.mode == VMO_GRAPH) ok = S->re.alloc(J.h.l, &eo);
  else {
    // l + 1 pointer entries: the end pointer of the last net is the job's own
    ok = S->rl.alloc((int64_t)J.h.l + 1, &no);
    if (ok && !S->rp.alloc(npins, &po)) { S->rl.release(no, (int64_t)J.h.l + 1); ok = false; }
  }
  if (!ok) {
    S->rv.release(voff, J.h.k);
    S->rn.release(nb, 4 * (int64_t)J.P);
    return false;
  }
  T.slot = S->free_slots.back();
  S->free_slots.pop_back();
  T.voff = voff; T.nbase = nb; T.eoff = eo; T.noff = no; T.poff = po; T.npins = npins;
  T.lbytes = lf;
  S->lbusy += lf;
  S->st.layout_bytes_peak = std::max(S->st.layout_bytes_peak, S->lbusy);
  return true;
}

// A job's layout is over (done or failed): its estimated footprint leaves
// the layouts in flight.  Called with S->mu held.
static void layout_done(vmo_server_s* S, Ticket& T) {
  S->lbusy -= T.lbytes;
  T.lbytes = 0;
  S->blocked = false;
}

static void release_ranges(vmo_server_s* S, Ticket& T) {
  const vmo_job& J = T.job;
  S->rv.release(T.voff, J.h.k);
  S->rn.release(T.nbase, 4 * (int64_t)J.P);
  if (J.mode == VMO_GRAPH) S->re.release(T.eoff, J.h.l);
  else {
    S->rl.release(T.noff, (int64_t)J.h.l + 1);
    S->rp.release(T.poff, T.npins);
  }
  S->free_slots.push_back(T.slot);
  S->blocked = false;
}

static JobHost host_job(const Ticket& T) {
  JobHost H;
  memset(&H, 0, sizeof H);
  H.h = T.job.h;
  H.mode = T.job.mode;
  H.order = T.job.order;
  H.x = T.job.x ? T.job.x : T.xbuf.p;
  H.P = T.job.P;
  H.seed = T.job.seed;
  H.job_index = T.job.job_index;
  H.out = T.job.out;
  return H;
}

static void finish_ticket(vmo_server_s* S, uint64_t id, vmo_status st, const std::string& err) {
  std::lock_guard<std::mutex> g(S->mu);
  Ticket& T = S->tickets[id];
  T.state = 2;
  T.status = st;
  T.err = err;
  T.t_done = now_ms();
  T.xbuf.release();
  S->st.completed += 1;
  S->done_cv.notify_all();
}

// A layout thread: lays out admitted jobs that came without coordinates.
static void layout_loop(vmo_server_s* S, vmo_layout_worker* W) {
  // a thread whose device cannot be selected fails every layout it takes
  const hipError_t dev = hipSetDevice(S->ctx.device);
  while (true) {
    uint64_t id;
    Ticket* T;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->lcv.wait(lk, [&] { return S->stop || !S->lqueue.empty(); });
      if (S->stop) break;
      id = S->lqueue.front();
      S->lqueue.pop_front();
      T = &S->tickets[id];
    }
    try {
      VMO_HIP(dev);
      T->xbuf = Buf<float>(W->ctx.pool, 4 * (size_t)T->job.h.k);
      layout(W->ctx, &T->job.h, &T->lp, T->xbuf.p, W->stream);
      check_device_flag(W->ctx, W->stream);
      VMO_HIP(hipStreamSynchronize(W->stream));
      tune_flush(W->ctx);
      trim_pool(W->ctx, W->stream);  // the cached blocks stay within this thread's share
      std::lock_guard<std::mutex> g(S->mu);
      layout_done(S, *T);
      S->ready.push_back(id);
    } catch (Error& e) {
      (void)hipStreamSynchronize(W->stream);
      (void)hipGetLastError();
      std::lock_guard<std::mutex> g(S->mu);
      layout_done(S, *T);
      S->lfailed.push_back({id, {e.status, e.what()}});
    }
    S->cv.notify_all();
  }
}

static void serve_loop(vmo_server_s* S) {
  // the same device that vmo_serve_create selected (and checked) on its thread
  (void)hipSetDevice(S->ctx.device);
  Engine& E = *S->eng;
  const bool threads = !S->lw.empty();
  while (true) {
    std::vector<uint64_t> admit;
    std::vector<std::pair<uint64_t, std::pair<vmo_status, std::string>>> failed;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        return S->stop || (!S->pending.empty() && !S->blocked) || !S->ready.empty() || !S->lfailed.empty() ||
               E.S > 0 || !S->resident.empty();
      });
      if (S->stop) break;
      // admit in arrival order while slots and ranges are free
      while (!S->pending.empty()) {
        uint64_t id = S->pending.front();
        Ticket& T = S->tickets[id];
        int64_t npins = 0;
        if (T.job.mode == VMO_NET && T.job.h.l > 0) {
          lk.unlock();
          try {
            npins = read1(T.job.h.net_ptr + T.job.h.l, S->stream);
          } catch (Error&) {
            npins = -1;
          }
          lk.lock();
        }
        if (npins < 0) {
          S->pending.pop_front();
          T.state = 2;
          T.status = VMO_E_INVALID;
          T.err = "cannot read the net pointer array";
          T.t_done = now_ms();
          S->st.completed += 1;
          S->done_cv.notify_all();
          continue;
        }
        if (!try_admit(S, T, npins)) {
          S->blocked = true;
          break;
        }
        S->pending.pop_front();
        T.state = 1;
        T.t_admit = now_ms();
        if (T.layout && threads) {
          S->lqueue.push_back(id);
          S->lcv.notify_one();
        } else {
          admit.push_back(id);
        }
      }
      for (uint64_t id : S->ready) admit.push_back(id);
      S->ready.clear();
      for (auto& f : S->lfailed) failed.push_back(f);
      S->lfailed.clear();
    }
    for (auto& f : failed) {
      {
        std::lock_guard<std::mutex> g(S->mu);
        release_ranges(S, S->tickets[f.first]);
      }
      finish_ticket(S, f.first, f.second.first, f.second.second);
    }
    for (uint64_t id : admit) {
      Ticket* T;
      {
        std::lock_guard<std::mutex> g(S->mu);
        T = &S->tickets[id];
      }
      try {
        if (!T->job.x && !T->xbuf.p) {
          T->xbuf = Buf<float>(S->ctx.pool, 4 * (size_t)T->job.h.k);
          layout(S->ctx, &T->job.h, &T->lp, T->xbuf.p, S->stream);
          check_device_flag(S->ctx, S->stream);
          trim_pool(S->ctx, S->stream);
          std::lock_guard<std::mutex> g(S->mu);
          layout_done(S, *T);
        }
        JobHost H = host_job(*T);
        E.arena_admit(T->slot, H, T->voff, T->nbase, T->eoff, T->noff, T->poff);
        std::lock_guard<std::mutex> g(S->mu);
        S->resident.push_back(id);
      } catch (Error& e) {
        (void)hipStreamSynchronize(S->stream);
        (void)hipGetLastError();
        {
          std::lock_guard<std::mutex> g(S->mu);
          release_ranges(S, *T);
        }
        finish_ticket(S, id, e.status, e.what());
      }
    }
    try {
      double t0 = now_ms();
      if (E.S > 0) {
        {
          // jobs whose segments this tick runs together
          std::vector<int32_t> in = E.segment_jobs();
          std::sort(in.begin(), in.end());
          const int64_t nj = (int64_t)(std::unique(in.begin(), in.end()) - in.begin());
          std::lock_guard<std::mutex> g(S->mu);
          S->st.max_tick_jobs = std::max(S->st.max_tick_jobs, nj);
          S->st.tick_jobs += nj;
        }
        E.tick(S->prm.t_max);
        check_device_flag(S->ctx, S->stream);
        tune_flush(S->ctx);
        prof_discard(S->ctx);
        std::lock_guard<std::mutex> g(S->mu);
        S->st.ticks += 1;
      }
      // jobs without segments are finished
      std::vector<int32_t> sj = E.segment_jobs();
      std::vector<char> busy(S->prm.max_jobs, 0);
      for (int32_t j : sj) busy[j] = 1;
      std::vector<uint64_t> fin;
      std::vector<int32_t> slots;
      std::vector<JobHost> hosts;
      {
        std::lock_guard<std::mutex> g(S->mu);
        std::vector<uint64_t> keep;
        for (uint64_t id : S->resident) {
          Ticket& T = S->tickets[id];
          if (busy[T.slot]) keep.push_back(id);
          else {
            fin.push_back(id);
            slots.push_back(T.slot);
            hosts.push_back(host_job(T));
          }
        }
        S->resident = keep;
      }
      if (!fin.empty()) {
        E.emit(slots, hosts);
        VMO_HIP(hipStreamSynchronize(S->stream));  // the outputs are complete before their tickets finish
        check_device_flag(S->ctx, S->stream);
        for (size_t i = 0; i < fin.size(); ++i) {
          E.arena_release(slots[i]);
          {
            std::lock_guard<std::mutex> g(S->mu);
            release_ranges(S, S->tickets[fin[i]]);
          }
          finish_ticket(S, fin[i], VMO_OK, "");
        }
      }
      std::lock_guard<std::mutex> g(S->mu);
      S->st.busy_ms += now_ms() - t0;
    } catch (std::exception& e) {
      // a device failure ends the server: fail every job it holds
      (void)hipStreamSynchronize(S->stream);
      std::vector<uint64_t> all;
      {
        std::lock_guard<std::mutex> g(S->mu);
        S->fatal = e.what();
        all = S->resident;
        for (uint64_t id : S->pending) all.push_back(id);
        S->resident.clear();
        S->pending.clear();
        S->stop = true;
      }
      for (uint64_t id : all) finish_ticket(S, id, VMO_E_DEVICE, S->fatal);
      break;
    }
  }
}

}  // namespace vmo

extern "C" {

void vmo_serve_defaults(vmo_serve_params* p) {
  if (!p) return;
  p->device = 0;
  p->budget_bytes = (size_t)8 << 30;
  p->max_jobs = 1024;
  p->t_max = 32;
  p->layout_threads = 4;
}

vmo_status vmo_serve_create(vmo_server* out, const vmo_serve_params* p) {
  if (!out || !p || p->max_jobs < 1 || p->t_max < 0 || p->budget_bytes < ((size_t)1 << 20) || p->layout_threads < 0 ||
      p->layout_threads > 64)
    return VMO_E_INVALID;
  vmo_server_s* S = new (std::nothrow) vmo_server_s();
  if (!S) return VMO_E_NOMEM;
  S->prm = *p;
  S->ctx.device = p->device;
  memset(&S->st, 0, sizeof S->st);
  try {
    VMO_HIP(hipSetDevice(p->device));
    VMO_HIP(hipStreamCreate(&S->stream));
    S->eng = new vmo::Engine(S->ctx, S->stream);
    int64_t V, NTn, En, Ln, Pn;
    vmo::arena_sizes(*p, &V, &NTn, &En, &Ln, &Pn);
    S->eng->arena_init(V, NTn, En, Ln, Pn, p->max_jobs);
    S->rv.init(V);
    S->rn.init(NTn);
    S->re.init(En);
    S->rl.init(Ln);
    S->rp.init(Pn);
    for (int32_t i = p->max_jobs - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->st.capacity_vertices = V;
    S->st.capacity_pins = Pn;
    S->st.capacity_edges = En;
    S->lbudget = (int64_t)((double)p->budget_bytes * (1.0 - vmo::kArenaShare));
    S->st.layout_budget_bytes = S->lbudget;
    const int nl = p->layout_threads > 0 ? p->layout_threads : 1;
    if (p->layout_threads == 0) S->ctx.pool_cap = (size_t)(S->lbudget / 2);
    for (int32_t i = 0; i < p->layout_threads; ++i) {
      vmo_layout_worker* W = new vmo_layout_worker();
      W->ctx.device = p->device;
      W->ctx.pool_cap = (size_t)(S->lbudget / (2 * nl));
      S->lw.push_back(W);
      VMO_HIP(hipStreamCreate(&W->stream));
    }
  } catch (vmo::Error& e) {
    for (vmo_layout_worker* W : S->lw) {
      if (W->stream) (void)hipStreamDestroy(W->stream);
      delete W;
    }
    delete S->eng;
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return e.status;
  }
  for (vmo_layout_worker* W : S->lw) W->th = std::thread(vmo::layout_loop, S, W);
  S->worker = std::thread(vmo::serve_loop, S);
  *out = S;
  return VMO_OK;
}

vmo_status vmo_serve_submit(vmo_server S, const vmo_job* job, const vmo_layout_params* lp, uint64_t* ticket) {
  if (!S || !job || !ticket) return VMO_E_INVALID;
  const vmo_job& J = *job;
  if (J.h.k < 1 || J.h.l < 0 || J.P < 1 || !J.h.net_ptr || !J.out.vperm || !J.out.part || !J.out.node_heap ||
      !J.out.node_vptr || !J.out.split_cut || !J.out.n_nodes)
    return VMO_E_INVALID;
  if (J.mode != VMO_NET && J.mode != VMO_GRAPH) return VMO_E_INVALID;
  if (J.order != VMO_SBD && J.order != VMO_BBD) return VMO_E_INVALID;
  if (!J.x && !lp) return VMO_E_INVALID;
  if (J.h.k > S->rv.cap() || 4 * (int64_t)J.P > S->rn.cap() ||
      (J.mode == VMO_GRAPH ? J.h.l > S->re.cap() : (int64_t)J.h.l + 1 > S->rl.cap()))
    return VMO_E_UNSUPPORTED;
  if (J.mode == VMO_NET && J.h.l > 0) {
    int64_t np = 0;
    if (hipSetDevice(S->ctx.device) != hipSuccess ||
        hipMemcpy(&np, J.h.net_ptr + J.h.l, sizeof np, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      return VMO_E_INVALID;
    }
    if (np > S->rp.cap()) return VMO_E_UNSUPPORTED;
    if (!J.x && (int64_t)vmo_layout_bytes(J.h.k, J.h.l, np) > S->lbudget / 2) return VMO_E_UNSUPPORTED;
  }
  if (!J.x && J.mode == VMO_GRAPH && (int64_t)vmo_layout_bytes(J.h.k, J.h.l, 2 * (int64_t)J.h.l) > S->lbudget / 2)
    return VMO_E_UNSUPPORTED;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return VMO_E_DEVICE;
  uint64_t id = S->next_id++;
  vmo::Ticket& T = S->tickets[id];
  T.job = J;
  T.layout = !J.x;
  if (lp) T.lp = *lp;
  T.t_submit = vmo::now_ms();
  S->pending.push_back(id);
  S->st.submitted += 1;
  *ticket = id;
  S->cv.notify_all();
  return VMO_OK;
}

vmo_status vmo_serve_poll(vmo_server S, uint64_t ticket, int32_t* done, vmo_status* job_status, double* latency_ms) {
  if (!S || !done) return VMO_E_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return VMO_E_INVALID;
  *done = it->second.state == 2;
  if (*done) {
    if (job_status) *job_status = it->second.status;
    if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
  }
  return VMO_OK;
}

vmo_status vmo_serve_wait(vmo_server S, uint64_t ticket, vmo_status* job_status, double* latency_ms) {
  if (!S) return VMO_E_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return VMO_E_INVALID;
  S->done_cv.wait(lk, [&] { return it->second.state == 2; });
  if (job_status) *job_status = it->second.status;
  if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
  return VMO_OK;
}

vmo_status vmo_serve_forget(vmo_server S, uint64_t ticket) {
  if (!S) return VMO_E_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end() || it->second.state != 2) return VMO_E_INVALID;
  S->tickets.erase(it);
  return VMO_OK;
}

vmo_status vmo_serve_get_stats(vmo_server S, vmo_serve_stats* out) {
  if (!S || !out) return VMO_E_INVALID;
  std::lock_guard<std::mutex> g(S->mu);
  *out = S->st;
  out->resident = (int64_t)S->resident.size();
  out->pending = (int64_t)S->pending.size();
  return VMO_OK;
}

const char* vmo_serve_error(vmo_server S, uint64_t ticket) {
  if (!S) return "NULL server";
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return "unknown ticket";
  return it->second.err.c_str();
}

vmo_status vmo_serve_destroy(vmo_server S) {
  if (!S) return VMO_E_INVALID;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv.notify_all();
    S->lcv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  for (vmo_layout_worker* W : S->lw)
    if (W->th.joinable()) W->th.join();
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (auto& kv : S->tickets)
      if (kv.second.state != 2) {
        kv.second.state = 2;
        kv.second.status = VMO_E_BUSY;
        kv.second.err = "server destroyed";
      }
    S->done_cv.notify_all();
  }
  (void)hipSetDevice(S->ctx.device);
  (void)hipStreamSynchronize(S->stream);
  delete S->eng;
  (void)hipStreamDestroy(S->stream);
  // coordinates still held by tickets go back to their layout pools first
  S->tickets.clear();
  for (vmo_layout_worker* W : S->lw) {
    (void)hipStreamSynchronize(W->stream);
    (void)hipStreamDestroy(W->stream);
    delete W;
  }
  delete S;
  return VMO_OK;
}

}  // extern "C"
