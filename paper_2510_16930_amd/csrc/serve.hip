// Request server: many HOQRI runs (Alg. 2) in flight on one GPU.
//
// Engine step: every admitted request moves by one mode update, i.e. the
// core from its current factors, then (unless it just finished) TTMcTC for
// its current mode and the orthonormalisation of the result. The core,
// TTMcTC and QR kernels are launched once per step for all requests together
// (batched launches over per-step descriptor tables), so the launch count of
// a step does not grow with the number of requests and small requests share
// the machine instead of queueing behind each other's launch latency.
//
// One synchronisation per step: after the cores, the host reads every
// request's f = ||G||^2 and breakdown flag, decides which requests finish
// (stop rule at a sweep boundary, or max_sweeps), and launches the rest.
// Admission is first-come first-served by footprint: the head of the queue is
// taken when a slot is (about to be) free and its plan workspace fits in the
// arena. Plans are built by a builder thread on its own stream, so building
// (sorts, slice tables, two synchronisations) overlaps the engine steps;
// built plans join the batch at the next step.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "passes.h"

namespace hoqri {
namespace {

constexpr size_t kGranule = 256;

class Arena {
 public:
  explicit Arena(size_t bytes) : size_(bytes / kGranule * kGranule) {
    if (size_ > 0) free_[0] = size_;
  }
  bool alloc(size_t bytes, size_t* off) {
    const size_t need = align_up(bytes < 1 ? 1 : bytes, kGranule);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const size_t o = it->first, sz = it->second;
        free_.erase(it);
        if (sz > need) free_[o + need] = sz - need;
        live_[o] = need;
        used_ += need;
        *off = o;
        return true;
      }
    }
    return false;
  }
  bool release(size_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return false;
    size_t o = off, sz = it->second;
    live_.erase(it);
    used_ -= sz;
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && nx->first == o + sz) {
      sz += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(o);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == o) {
        o = pv->first;
        sz += pv->second;
        free_.erase(pv);
      }
    }
    free_[o] = sz;
    return true;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  int32_t live_blocks() const { return (int32_t)live_.size(); }

 private:
  size_t size_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  std::map<size_t, size_t> live_;  // offset -> bytes
};

struct Pending {
  hoqri_request r;
  std::vector<int64_t> dims;
  std::vector<int32_t> ranks;
  std::vector<float*> U;
  size_t need;
  hoqri_status pre;  // error found at submit/admission, reported as the result
};

struct Built {
  Pending q;
  hoqri_plan* plan;
  size_t off;
};

struct Active {
  Pending q;
  hoqri_plan* plan;
  size_t off;
  int slot;
  int t, n;          // sweeps done, current mode
  bool fresh;        // the core of the starting factors is still to be formed
  double f_prev;     // f at the start of the current sweep
  double rel;
  int64_t admitted;
};

}  // namespace
}  // namespace hoqri

struct hoqri_arena {
  hoqri::Arena a;
  explicit hoqri_arena(size_t b) : a(b) {}
};

struct hoqri_server {
  hoqri_server_opts o;
  int device = -1;
  char* base = nullptr;        // arena region for plans
  hoqri::Arena* arena = nullptr;
  hoqri::Staging st[2];
  char* pinned = nullptr;      // 2 staging halves + f / status read-back
  double* d_f = nullptr;       // [max_slots] f of each slot's latest core
  int32_t* d_stat = nullptr;   // [max_slots] sticky breakdown flags
  int32_t* d_skip = nullptr;   // [max_slots] updates kept for rank deficiency
  double* h_f = nullptr;
  int32_t* h_stat = nullptr;
  int32_t* h_skip = nullptr;
  std::vector<hoqri::Active> active;  // engine thread only
  std::vector<int> free_slots;        // engine thread only
  int64_t step_no = 0;
  // step graph (use_graphs): the executable graph of the last step's launches,
  // updated in place when the next step's launches have the same topology
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;  // private stream the step is captured on (the caller's may be the null stream)
  int64_t graph_instantiations = 0, graph_updates = 0;
  // time_passes: events around the last step's TTMcTC launches (read at the
  // next step, after its synchronisation) and the totals so far
  hipEvent_t ttm_ev[2] = {nullptr, nullptr};
  bool ttm_pending = false;
  double ttm_pending_bytes = 0.0, ttm_pending_flops = 0.0;
  int64_t ttm_steps = 0;
  double ttm_ms = 0.0, ttm_bytes = 0.0, ttm_flops = 0.0;
  // shared with the builder thread (guarded by mu)
  std::mutex mu;
  std::condition_variable cv_build;   // builder: work or memory became available
  std::condition_variable cv_ready;   // engine: a plan was built (or failed)
  std::deque<hoqri::Pending> queue;
  std::deque<hoqri::Built> ready;
  std::deque<hoqri_result> done;      // finished, not yet handed out
  int n_active = 0;
  int building = 0;
  bool stop = false;
  hoqri_status builder_error = HOQRI_OK;
  std::thread builder;
};

using namespace hoqri;

namespace {

size_t stage_bytes(int slots) { return align_up(65536 + (size_t)slots * 4096); }

// Captures the launches of a step into a graph (on the server's private
// stream: capture records work without running it, and the caller's stream may
// be the null stream, which cannot be captured) and launches it on `s` as one
// launch: the executable graph of the previous step is updated in place when
// the topology (the sequence of kernels and copies) is unchanged, else a new
// one is instantiated. The captured copies read the pinned staging tables at
// replay time, which hold this step's tables.
template <class F>
hoqri_status graph_step(hoqri_server* S, hipStream_t s, F&& launches) {
  HOQRI_HIP_TRY(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
  const hoqri_status ls = launches(S->cap);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(S->cap, &g);
  if (ls != HOQRI_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return ls != HOQRI_OK ? ls : HOQRI_ERR_HIP;
  }
  bool updated = false;
  if (S->gexec) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    updated = hipGraphExecUpdate(S->gexec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
    if (!updated) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(S->gexec);
      S->gexec = nullptr;
    }
  }
  if (!updated) {
    if (hipGraphInstantiate(&S->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      S->gexec = nullptr;
      (void)hipGraphDestroy(g);
      return HOQRI_ERR_HIP;
    }
    ++S->graph_instantiations;
  } else {
    ++S->graph_updates;
  }
  (void)hipGraphDestroy(g);
  HOQRI_HIP_TRY(hipGraphLaunch(S->gexec, s));
  return HOQRI_OK;
}

hoqri_result make_result(const Pending& q, hoqri_status st) {
  hoqri_result r{};
  r.id = q.r.id;
  r.status = st;
  return r;
}

// Finishing a request: factors back to the caller's row order, the core to the
// caller's buffer, optional orthonormality check; the plan is released after
// the step's final synchronisation.
hoqri_status finish_copy(hoqri_server* S, Active& a, hipStream_t s, double* d_err) {
  hoqri_plan* p = a.plan;
  HOQRI_TRY(from_labels(p, a.q.U.data(), s));
  int64_t PK = 1;
  for (int n = 0; n < p->N; ++n) PK *= p->K[n];
  HOQRI_HIP_TRY(hipMemcpyAsync(a.q.r.d_G, p->sc.G, (size_t)PK * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (S->o.report_orth_err && d_err)
    for (int n = 0; n < p->N; ++n)
      HOQRI_TRY(launch_orth_err(p->dims[n], p->K[n], a.q.U[n], d_err + n, p->sc.orth_ws, p->sc.orth_ws_bytes, s));
  return HOQRI_OK;
}

// Builder thread: takes the head of the queue when the batch has room for it
// (slots in use + built + building below max_slots plus a small lookahead)
// and its workspace fits in the arena, builds its plan on its own stream, and
// hands it to the engine. A request that does not fit waits; none overtakes it.
void builder_loop(hoqri_server* S) {
  hipStream_t bs = nullptr;
  hoqri_status err = HOQRI_OK;
  if (hipSetDevice(S->device) != hipSuccess || hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess)
    err = HOQRI_ERR_HIP;
  std::unique_lock<std::mutex> lk(S->mu);
  if (err != HOQRI_OK) {
    S->builder_error = err;
    S->cv_ready.notify_all();
    return;
  }
  const int lookahead = 2;
  while (true) {
    size_t off = 0;
    S->cv_build.wait(lk, [&] {
      if (S->stop) return true;
      if (S->queue.empty()) return false;
      if (S->n_active + (int)S->ready.size() >= S->o.max_slots + lookahead) return false;
      const Pending& q = S->queue.front();
      if (q.pre != HOQRI_OK || q.need > S->arena->size()) return true;  // fails at once
      return S->arena->alloc(q.need, &off);
    });
    if (S->stop) break;
    Pending q = std::move(S->queue.front());
    S->queue.pop_front();
    if (q.pre != HOQRI_OK || q.need > S->arena->size()) {
      S->done.push_back(make_result(q, q.pre != HOQRI_OK ? q.pre : HOQRI_ERR_NOMEM));
      S->cv_ready.notify_all();
      continue;
    }
    S->building = 1;
    lk.unlock();
    hoqri_plan* plan = nullptr;
    hoqri_status st = hoqri_plan_create(&plan, q.r.order, q.dims.data(), q.ranks.data(), q.r.nnz, q.r.d_idx,
                                        q.r.d_vals, S->base + off, q.need, bs);
    if (st == HOQRI_OK)
      for (int n = 0; n < plan->N; ++n) {
        if (!segpass_supported(plan, n) || !plan->yfuse) st = HOQRI_ERR_UNSUPPORTED;
        else if (plan->md[n].R < plan->K[n]) st = HOQRI_ERR_BREAKDOWN;  // fewer nonempty slices than K_n
      }
    lk.lock();
    S->building = 0;
    if (st != HOQRI_OK) {
      if (plan) hoqri_plan_destroy(plan);
      S->arena->release(off);
      S->done.push_back(make_result(q, st));
    } else {
      S->ready.push_back(Built{std::move(q), plan, off});
    }
    S->cv_ready.notify_all();
  }
  lk.unlock();
  (void)hipStreamDestroy(bs);
}

// Engine thread: built plans join the batch (their plan build has completed:
// the builder synchronised its stream).
hoqri_status admit(hoqri_server* S, hipStream_t s) {
  std::deque<Built> take;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->builder_error != HOQRI_OK) return S->builder_error;
    if (S->active.empty() && S->ready.empty() && (S->building || !S->queue.empty()))
      S->cv_ready.wait_for(lk, std::chrono::milliseconds(2));  // nothing to run yet
    int room = (int)S->free_slots.size();
    if (S->o.max_admit_per_step > 0 && room > S->o.max_admit_per_step) room = S->o.max_admit_per_step;
    while (room > 0 && !S->ready.empty()) {
      take.push_back(std::move(S->ready.front()));
      S->ready.pop_front();
      --room;
    }
    S->n_active += (int)take.size();
  }
  for (Built& b : take) {
    Active a{};
    a.q = std::move(b.q);
    a.plan = b.plan;
    a.off = b.off;
    a.slot = S->free_slots.back();
    S->free_slots.pop_back();
    a.admitted = S->step_no;
    a.fresh = true;
    HOQRI_TRY(to_labels(a.plan, a.q.U.data(), s));
    HOQRI_TRY(fill_i32(S->d_stat + a.slot, 1, 0, s));
    HOQRI_TRY(fill_i32(S->d_skip + a.slot, 1, 0, s));
    S->active.push_back(std::move(a));
  }
  return HOQRI_OK;
}

template <class Job, class Group>
hoqri_status run_groups(std::vector<Job>& jobs, Staging& st, hipStream_t s,
                        bool (*stage)(const Job* const*, int, Staging&, Group*),
                        hoqri_status (*launch)(const Group&, hipStream_t)) {
  // group by kernel instance (and its launch shape), keep request order inside a group
  std::vector<int> order(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) order[i] = (int)i;
  auto rank = [&](int x) { return std::make_tuple(jobs[x].key, jobs[x].threads, jobs[x].shmem); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rank(x) < rank(y); });
  std::vector<Group> groups;
  size_t i = 0;
  while (i < order.size()) {
    size_t j = i;
    std::vector<const Job*> g;
    while (j < order.size() && jobs[order[j]].key == jobs[order[i]].key && jobs[order[j]].threads == jobs[order[i]].threads &&
           jobs[order[j]].shmem == jobs[order[i]].shmem) {
      g.push_back(&jobs[order[j]]);
      ++j;
    }
    Group grp;
    if (!stage(g.data(), (int)g.size(), st, &grp)) return HOQRI_ERR_NOMEM;
    groups.push_back(grp);
    i = j;
  }
  HOQRI_HIP_TRY(st.upload(s));
  for (const Group& grp : groups) HOQRI_TRY(launch(grp, s));
  return HOQRI_OK;
}

}  // namespace

extern "C" hoqri_status hoqri_arena_create(size_t bytes, hoqri_arena** arena) {
  if (!arena || bytes < kGranule) return HOQRI_ERR_ARG;
  *arena = new (std::nothrow) hoqri_arena(bytes);
  return *arena ? HOQRI_OK : HOQRI_ERR_NOMEM;
}

extern "C" hoqri_status hoqri_arena_alloc(hoqri_arena* arena, size_t bytes, size_t* offset) {
  if (!arena || !offset) return HOQRI_ERR_ARG;
  return arena->a.alloc(bytes, offset) ? HOQRI_OK : HOQRI_ERR_NOMEM;
}

extern "C" hoqri_status hoqri_arena_free(hoqri_arena* arena, size_t offset) {
  if (!arena) return HOQRI_ERR_ARG;
  return arena->a.release(offset) ? HOQRI_OK : HOQRI_ERR_ARG;
}

extern "C" hoqri_status hoqri_arena_stats(const hoqri_arena* arena, size_t* used, size_t* largest_free,
                                          int32_t* live_blocks) {
  if (!arena) return HOQRI_ERR_ARG;
  if (used) *used = arena->a.used();
  if (largest_free) *largest_free = arena->a.largest_free();
  if (live_blocks) *live_blocks = arena->a.live_blocks();
  return HOQRI_OK;
}

extern "C" void hoqri_arena_destroy(hoqri_arena* arena) { delete arena; }

extern "C" hoqri_status hoqri_server_create(const hoqri_server_opts* opts, hoqri_server** server) {
  if (!opts || !server || !opts->d_arena) return HOQRI_ERR_ARG;
  *server = nullptr;
  if (opts->max_slots < 1 || opts->max_slots > 1024 || opts->max_sweeps < 1 || opts->max_sweeps > kMaxSweeps ||
      !(opts->tol >= 0.0))
    return HOQRI_ERR_ARG;
  const int slots = opts->max_slots;
  const size_t sb = stage_bytes(slots);
  const size_t fixed = 2 * sb + align_up((size_t)slots * 8) + 2 * align_up((size_t)slots * 4);
  if (opts->arena_bytes < fixed + kGranule) return HOQRI_ERR_NOMEM;
  hoqri_server* S = new (std::nothrow) hoqri_server();
  if (!S) return HOQRI_ERR_NOMEM;
  S->o = *opts;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return HOQRI_ERR_HIP;
  }
  const size_t host_bytes = 2 * sb + (size_t)slots * 16 + 64;
  if (hipHostMalloc((void**)&S->pinned, host_bytes, hipHostMallocDefault) != hipSuccess) {
    delete S;
    return HOQRI_ERR_HIP;
  }
  char* d = (char*)opts->d_arena;
  S->st[0].bind(S->pinned, d, sb);
  S->st[1].bind(S->pinned + sb, d + sb, sb);
  S->d_f = (double*)(d + 2 * sb);
  S->d_stat = (int32_t*)(d + 2 * sb + align_up((size_t)slots * 8));
  S->d_skip = (int32_t*)(d + 2 * sb + align_up((size_t)slots * 8) + align_up((size_t)slots * 4));
  S->h_f = (double*)(S->pinned + 2 * sb);
  S->h_stat = (int32_t*)(S->pinned + 2 * sb + (size_t)slots * 8);
  S->h_skip = (int32_t*)(S->pinned + 2 * sb + (size_t)slots * 12);
  S->base = d + fixed;
  S->arena = new (std::nothrow) Arena(opts->arena_bytes - fixed);
  if (!S->arena) {
    (void)hipHostFree(S->pinned);
    delete S;
    return HOQRI_ERR_NOMEM;
  }
  for (int i = slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  if (opts->time_passes && !opts->use_graphs) {
    for (auto& e : S->ttm_ev) {
      if (hipEventCreate(&e) != hipSuccess) {
        (void)hipHostFree(S->pinned);
        delete S->arena;
        delete S;
        return HOQRI_ERR_HIP;
      }
    }
  }
  // graph capture runs on a private stream of default priority
  if (opts->use_graphs && hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking) != hipSuccess) {
    S->cap = nullptr;
    (void)hipHostFree(S->pinned);
    delete S->arena;
    delete S;
    return HOQRI_ERR_HIP;
  }
  try {
    S->builder = std::thread(builder_loop, S);
  } catch (...) {
    if (S->cap) (void)hipStreamDestroy(S->cap);
    (void)hipHostFree(S->pinned);
    delete S->arena;
    delete S;
    return HOQRI_ERR_NOMEM;
  }
  *server = S;
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_server_submit(hoqri_server* S, const hoqri_request* r) {
  if (!S || !r || !r->dims || !r->ranks || !r->d_idx || !r->d_vals || !r->d_U || !r->d_G) return HOQRI_ERR_ARG;
  if (r->order < 2 || r->order > kMaxOrder) return HOQRI_ERR_ARG;
  Pending q;
  q.r = *r;
  q.dims.assign(r->dims, r->dims + r->order);
  q.ranks.assign(r->ranks, r->ranks + r->order);
  q.U.assign(r->d_U, r->d_U + r->order);
  for (float* u : q.U)
    if (!u) return HOQRI_ERR_ARG;
  q.r.dims = nullptr;
  q.r.ranks = nullptr;
  q.r.d_U = nullptr;
  q.need = 0;
  q.pre = hoqri_plan_workspace_size(r->order, q.dims.data(), q.ranks.data(), r->nnz, &q.need);
  if (q.pre == HOQRI_ERR_HIP) return q.pre;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->queue.push_back(std::move(q));
  }
  S->cv_build.notify_one();
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_server_step(hoqri_server* S, hipStream_t s, hoqri_result* results, int32_t cap,
                                          int32_t* n_results) {
  if (!S || !n_results || (cap > 0 && !results) || cap < 0) return HOQRI_ERR_ARG;
  *n_results = 0;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HOQRI_ERR_HIP;
  if (dev != S->device) return HOQRI_ERR_ARG;
  Staging& st = S->st[S->step_no & 1];
  st.off = st.mark = 0;

  HOQRI_TRY(admit(S, s));
  std::vector<Active>& act = S->active;
  if (!act.empty()) {
    // 1. cores of the starting factors of newly admitted requests (f into
    // their slots); the others' cores came from their last mode update
    std::vector<CoreJob> cj;
    for (Active& a : act) {
      if (!a.fresh) continue;
      Operands op{OP_FP32, a.plan->sc.Up, a.plan->sc.Uh};
      cj.emplace_back();
      HOQRI_TRY(prepare_core(a.plan, op, a.plan->sc.G, S->d_f + a.slot, &cj.back()));
      a.fresh = false;
    }
    if (!cj.empty()) HOQRI_TRY((run_groups<CoreJob, CoreGroup>(cj, st, s, stage_core_group, launch_core_group)));
    const int slots = S->o.max_slots;
    HOQRI_HIP_TRY(hipMemcpyAsync(S->h_f, S->d_f, (size_t)slots * 8, hipMemcpyDeviceToHost, s));
    HOQRI_HIP_TRY(hipMemcpyAsync(S->h_stat, S->d_stat, (size_t)slots * 4, hipMemcpyDeviceToHost, s));
    HOQRI_HIP_TRY(hipMemcpyAsync(S->h_skip, S->d_skip, (size_t)slots * 4, hipMemcpyDeviceToHost, s));
    HOQRI_HIP_TRY(hipStreamSynchronize(s));
    if (S->ttm_pending) {  // the previous step's TTMcTC launches are complete
      float ms = 0.f;
      HOQRI_HIP_TRY(hipEventElapsedTime(&ms, S->ttm_ev[0], S->ttm_ev[1]));
      S->ttm_ms += ms;
      S->ttm_bytes += S->ttm_pending_bytes;
      S->ttm_flops += S->ttm_pending_flops;
      ++S->ttm_steps;
      S->ttm_pending = false;
    }

    // 2. decisions at sweep boundaries (same rule as hoqri_run with check_every = 1)
    std::vector<int> finishing, going;
    std::vector<hoqri_status> fin_status;
    for (size_t i = 0; i < act.size(); ++i) {
      Active& a = act[i];
      const double f = S->h_f[a.slot];
      if (S->h_stat[a.slot] != 0) {
        finishing.push_back((int)i);
        fin_status.push_back(HOQRI_ERR_BREAKDOWN);
        continue;
      }
      if (a.n == 0) {
        bool stop = a.t >= S->o.max_sweeps;
        if (a.t >= 1) {
          a.rel = f > 0 ? std::fabs(f - a.f_prev) / f : 0.0;
          if (S->o.tol > 0.0 && std::fabs(f - a.f_prev) <= S->o.tol * f) stop = true;
        }
        a.f_prev = f;
        if (stop) {
          finishing.push_back((int)i);
          fin_status.push_back(HOQRI_OK);
          continue;
        }
      }
      going.push_back((int)i);
    }

    // 3. TTMcTC (storing Y_(n)), orthonormalisation and the core of the
    // updated factors (f into the slot) for the continuing requests
    if (!going.empty()) {
      std::vector<TtmJob> tj(going.size());
      std::vector<OrthJob> oj(going.size());
      std::vector<YCoreJob> yj(going.size());
      for (size_t k = 0; k < going.size(); ++k) {
        Active& a = act[going[k]];
        hoqri_plan* p = a.plan;
        Operands op{OP_FP32, p->sc.Up, p->sc.Uh};
        HOQRI_TRY(prepare_ttm(p, a.n, op, p->sc.G, p->sc.A, nullptr, &tj[k], true));
        HOQRI_TRY(prepare_orth(p->md[a.n].R, p->K[a.n], p->sc.A, p->sc.Up[a.n], nullptr, S->d_stat + a.slot,
                               p->sc.orth_ws, p->sc.orth_ws_bytes, true, &oj[k],
                               S->o.keep_on_breakdown ? S->d_skip + a.slot : nullptr, p->dims[a.n]));
        HOQRI_TRY(prepare_ycore(p, a.n, p->sc.G, S->d_f + a.slot, &yj[k]));
      }
      // the launches of this step: table uploads from pinned memory and one
      // batched launch per kernel kind (no memset nodes)
      const bool timed = S->ttm_ev[0] && !S->o.use_graphs;
      if (timed) {
        // algorithmic work of this step's passes (float32 operands)
        double by = 0.0, fl = 0.0;
        for (int i : going) {
          const hoqri_plan* p = act[i].plan;
          const int n = act[i].n, N = p->N;
          double PK = 1.0, P = 1.0, rows = 0.0;
          for (int m = 0; m < N; ++m) {
            PK *= p->K[m];
            if (m != n) {
              P *= p->K[m];
              rows += (double)p->md[m].R * p->K[m] * 4.0;
            }
          }
          by += (double)p->nnz * 4.0 * N + 8.0 * (double)p->md[n].R + rows + 4.0 * (double)p->dims[n] * p->K[n];
          fl += 2.0 * (double)p->nnz * P + 2.0 * (double)p->md[n].R * PK;
        }
        S->ttm_pending_bytes = by;
        S->ttm_pending_flops = fl;
      }
      auto launches = [&](hipStream_t ls) -> hoqri_status {
        if (timed) HOQRI_HIP_TRY(hipEventRecord(S->ttm_ev[0], ls));
        HOQRI_TRY((run_groups<TtmJob, TtmGroup>(tj, st, ls, stage_ttm_group, launch_ttm_group)));
        if (timed) {
          HOQRI_HIP_TRY(hipEventRecord(S->ttm_ev[1], ls));
          S->ttm_pending = true;
        }
        std::vector<const OrthJob*> op(oj.size());
        for (size_t k = 0; k < oj.size(); ++k) op[k] = &oj[k];
        OrthGroup og;
        if (!stage_orth_group(op.data(), (int)op.size(), st, &og)) return HOQRI_ERR_NOMEM;
        std::vector<const YCoreJob*> yp(yj.size());
        for (size_t k = 0; k < yj.size(); ++k) yp[k] = &yj[k];
        YCoreGroup yg;
        if (!stage_ycore_group(yp.data(), (int)yp.size(), st, &yg)) return HOQRI_ERR_NOMEM;
        HOQRI_HIP_TRY(st.upload(ls));
        HOQRI_TRY(launch_orth_group(og, ls));
        HOQRI_TRY(launch_ycore_group(yg, ls));
        return HOQRI_OK;
      };
      if (S->o.use_graphs) HOQRI_TRY(graph_step(S, s, launches));
      else HOQRI_TRY(launches(s));
      for (int i : going) {
        Active& a = act[i];
        if (++a.n == a.plan->N) {
          a.n = 0;
          ++a.t;
        }
      }
    }

    // 4. results of the finishing requests
    if (!finishing.empty()) {
      for (size_t k = 0; k < finishing.size(); ++k) {
        Active& a = act[finishing[k]];
        // orthonormality errors go to the plan's own scalar area
        if (fin_status[k] == HOQRI_OK) HOQRI_TRY(finish_copy(S, a, s, a.plan->sc.f_dev + 8));
      }
      HOQRI_HIP_TRY(hipStreamSynchronize(s));
      for (size_t k = 0; k < finishing.size(); ++k) {
        Active& a = act[finishing[k]];
        hoqri_result r = make_result(a.q, fin_status[k]);
        r.sweeps = a.t;
        r.norm_x2 = a.plan->normx2;
        r.f = S->h_f[a.slot];
        r.fit = 1.0 - std::sqrt(std::fmax(r.norm_x2 - r.f, 0.0)) / std::sqrt(r.norm_x2);
        r.rel_change = a.rel;
        r.skipped_updates = S->h_skip[a.slot];
        r.admitted_step = a.admitted;
        r.finished_step = S->step_no;
        if (S->o.report_orth_err && fin_status[k] == HOQRI_OK) {
          double e[kMaxOrder] = {0, 0, 0, 0};
          HOQRI_HIP_TRY(hipMemcpy(e, a.plan->sc.f_dev + 8, a.plan->N * sizeof(double), hipMemcpyDeviceToHost));
          for (int n = 0; n < a.plan->N; ++n) r.orth_err_max = std::max(r.orth_err_max, e[n]);
        }
        {
          std::lock_guard<std::mutex> lk(S->mu);
          S->done.push_back(r);
          S->arena->release(a.off);
          --S->n_active;
        }
        S->free_slots.push_back(a.slot);
        hoqri_plan_destroy(a.plan);
        a.plan = nullptr;
      }
      S->cv_build.notify_one();
      std::vector<Active> keep;
      keep.reserve(act.size());
      for (Active& a : act)
        if (a.plan) keep.push_back(std::move(a));
      act.swap(keep);
    }
  }
  ++S->step_no;
  int32_t k = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    while (k < cap && !S->done.empty()) {
      results[k++] = S->done.front();
      S->done.pop_front();
    }
  }
  *n_results = k;
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_server_info(const hoqri_server* S, int32_t* queued, int32_t* active, size_t* used) {
  if (!S) return HOQRI_ERR_ARG;
  hoqri_server* M = const_cast<hoqri_server*>(S);
  std::lock_guard<std::mutex> lk(M->mu);
  // waiting, being built, built but not yet in the batch; results not yet handed out count as active
  if (queued) *queued = (int32_t)(M->queue.size() + M->ready.size()) + M->building;
  if (active) *active = M->n_active + (int32_t)M->done.size();
  if (used) *used = M->arena->used();
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_server_ttm_stats(const hoqri_server* S, int64_t* steps, double* ms, double* bytes,
                                               double* flops) {
  if (!S || !steps || !ms || !bytes || !flops) return HOQRI_ERR_ARG;
  *steps = S->ttm_steps;
  *ms = S->ttm_ms;
  *bytes = S->ttm_bytes;
  *flops = S->ttm_flops;
  return HOQRI_OK;
}

extern "C" void hoqri_server_destroy(hoqri_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_build.notify_all();
  if (S->builder.joinable()) S->builder.join();
  for (Built& b : S->ready)
    if (b.plan) hoqri_plan_destroy(b.plan);
  for (Active& a : S->active)
    if (a.plan) hoqri_plan_destroy(a.plan);
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  if (S->cap) (void)hipStreamDestroy(S->cap);
  for (hipEvent_t e : S->ttm_ev)
    if (e) (void)hipEventDestroy(e);
  if (S->pinned) (void)hipHostFree(S->pinned);
  delete S->arena;
  delete S;
}
