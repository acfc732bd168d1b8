// Serving loop: a device-resident plan cache and continuously batched solves.
//
// Many map-making solves of uneven size share one GPU.  Plans (pointing, band spectra, BJ
// blocks) stay on the device under a caller-chosen geometry key.  Submitted requests wait in
// one queue; n_slots worker threads, each with its own non-blocking HIP stream, take the
// oldest request whose workspace fits the memory budget and run it with a workspace of its
// own, so the kernels of several requests overlap on the device and a request that arrives
// while others run starts as soon as a slot and memory are free.  A request that does not fit
// lets later ones pass, at most max_bypass times, so that large requests are not starved.
// With size classes, requests whose work (samples x right-hand sides) reaches large_work run at
// most large_slots at a time; small requests pass a held large one freely.
// Idle workspaces stay with their plan for reuse; under memory pressure idle workspaces are
// released first, then unpinned plans, least recently used first.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "mm_internal.h"

namespace mm {

using Clock = std::chrono::steady_clock;

struct CacheEntry {
  uint64_t key = 0;
  Plan* plan = nullptr;
  int64_t plan_bytes = 0;      // the plan, including its own workspace
  int64_t work_each = 0;       // bytes of one extra solve workspace
  bool own_work_free = true;   // the plan's own workspace is available to a request
  std::vector<Work*> idle;     // extra workspaces not in use
  int32_t pins = 0;            // queued + running requests
  uint64_t last_use = 0;
  bool building = false;
};

struct Request {
  uint64_t ticket = 0;
  CacheEntry* entry = nullptr;
  const float* d = nullptr;
  int32_t k = 0;
  int64_t ld_d = 0;
  double* x = nullptr;
  mm_solve_opts opts{};
  int64_t extra_bytes = 0;     // block-solve workspace on top of a solve workspace
  int32_t bypassed = 0;
  bool large = false;          // size class (n_samples x k >= the server's large_work)
  Clock::time_point t_submit, t_start, t_end;
  bool done = false;
  mm_status status = MM_PENDING;
  std::string error;
  std::vector<mm_solve_info> info;
  int32_t slot = -1;
  // set at admission
  Work* work = nullptr;
  bool uses_own = false;
  int64_t reserved = 0;        // bytes reserved at admission (new workspace + block extra)
};

struct Server {
  int device = 0;
  int64_t budget = 0;
  int32_t n_slots = 4;
  int32_t max_bypass = 16;
  int64_t large_work = 0;    // size classes: work n_samples x k at which a request is large
  int32_t large_slots = 1;   // large requests running at once
  int32_t running_large = 0;
  int32_t peak_large = 0;
  std::mutex mu;
  std::condition_variable cv_work;   // workers: admissible request or stop
  std::condition_variable cv_state;  // plan builds finished, requests finished
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::unordered_map<uint64_t, std::unique_ptr<CacheEntry>> cache;
  int64_t in_use = 0;
  int64_t peak = 0;
  uint64_t next_ticket = 1;
  uint64_t tick = 0;
  int32_t running = 0;
  int32_t peak_running = 0;
  int64_t submitted = 0, completed = 0, hits = 0, misses = 0, evictions = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
};

namespace {

int64_t block_extra_bytes(const Plan* P, const mm_solve_opts& o, int32_t k) {
  if (o.block == 0 || o.block == 1 || k < 2) return 0;
  const int64_t t = o.block < 0 ? std::min<int32_t>(32, k) : std::min<int32_t>(o.block, std::min(32, k));
  const int64_t nu = 3 * P->n_kept;
  // R, Z, W, MR (t columns each), Gram partials (at most 1024 workgroups x 32 x 32) and the
  // small t x t matrices
  return 4 * t * nu * static_cast<int64_t>(sizeof(double)) +
         static_cast<int64_t>(1024 * 1024 * sizeof(double)) + 65536;
}

void note_bytes(Server* S) { S->peak = std::max(S->peak, S->in_use); }

// Free idle workspaces, then evict unpinned plans (LRU), until `need` more bytes fit.
// Called with S->mu held.
bool reclaim_locked(Server* S, int64_t need) {
  if (S->in_use + need <= S->budget) return true;
  for (auto& kv : S->cache) {
    CacheEntry* e = kv.second.get();
    while (!e->idle.empty() && S->in_use + need > S->budget) {
      Work* w = e->idle.back();
      e->idle.pop_back();
      S->in_use -= w->bytes;
      work_free(w);
      delete w;
    }
  }
  while (S->in_use + need > S->budget) {
    CacheEntry* victim = nullptr;
    for (auto& kv : S->cache) {
      CacheEntry* e = kv.second.get();
      if (e->building || e->pins > 0) continue;
      if (!victim || e->last_use < victim->last_use) victim = e;
    }
    if (!victim) return false;
    for (Work* w : victim->idle) {
      S->in_use -= w->bytes;
      work_free(w);
      delete w;
    }
    S->in_use -= victim->plan_bytes;
    destroy_plan(victim->plan);
    ++S->evictions;
    S->cache.erase(victim->key);
  }
  return true;
}

// Admission cost of a request now: a free workspace of its plan costs nothing.
int64_t admission_cost(const Request* r) {
  const CacheEntry* e = r->entry;
  const int64_t ws = (e->own_work_free || !e->idle.empty()) ? 0 : e->work_each;
  return ws + r->extra_bytes;
}

void finish_unrun_locked(Server* S, Request* r, mm_status st, const std::string& msg) {
  r->entry->pins -= 1;
  r->status = st;
  r->error = msg;
  r->done = true;
  S->completed += 1;
}

Request* try_admit_locked(Server* S);

// Pick the next request to run (S->mu held); reserves its memory.  When nothing runs and no
// queued request fits, the memory is held by plans that queued requests pin, and waiting
// cannot free it: the head request then fails with MM_ERR_BUDGET and the scan repeats.
Request* pick_locked(Server* S) {
  while (true) {
    Request* r = try_admit_locked(S);
    if (r != nullptr || S->queue.empty() || S->running > 0) return r;
    Request* head = S->queue.front();
    S->queue.pop_front();
    finish_unrun_locked(S, head, MM_ERR_BUDGET,
                        "request could not be admitted: the memory budget is held by the plans "
                        "of other queued requests");
    S->cv_state.notify_all();
  }
}

Request* try_admit_locked(Server* S) {
  for (size_t i = 0; i < S->queue.size(); ++i) {
    Request* r = S->queue[i];
    // a large request held by the size rule does not block later (small) ones
    if (r->large && S->running_large >= S->large_slots) continue;
    const int64_t cost = admission_cost(r);
    if (S->in_use + cost > S->budget) reclaim_locked(S, cost);
    if (S->in_use + cost <= S->budget) {
      for (size_t j = 0; j < i; ++j)
        if (!(S->queue[j]->large && S->running_large >= S->large_slots))
          S->queue[j]->bypassed += 1;
      S->queue.erase(S->queue.begin() + static_cast<std::ptrdiff_t>(i));
      CacheEntry* e = r->entry;
      if (e->own_work_free) {
        e->own_work_free = false;
        r->uses_own = true;
        r->work = &e->plan->work;
      } else if (!e->idle.empty()) {
        r->work = e->idle.back();
        e->idle.pop_back();
      } else {
        r->work = nullptr;  // allocated by the worker outside the lock
      }
      r->reserved = cost;
      S->in_use += cost;
      note_bytes(S);
      return r;
    }
    if (r->bypassed >= S->max_bypass) return nullptr;  // it waits at the head
  }
  return nullptr;
}

mm_status run_request(Server* S, Request* r, hipStream_t s) {
  Plan* P = r->entry->plan;
  Work& W = *r->work;
  if (r->opts.block != 0 && r->opts.block != 1 && r->k > 1)
    return block_solve(P, W, r->d, r->k, r->ld_d, r->x, &r->opts, r->info.data(), s);
  mm_status worst = MM_OK;
  std::string msg;
  for (int32_t j = 0; j < r->k; ++j) {
    const mm_status st = pcg_solve(P, W, r->d + j * r->ld_d, r->x + j * 3 * P->n_kept, &r->opts,
                                   &r->info[j], s);
    if (st == MM_ERR_HIP || st == MM_ERR_OOM || st == MM_ERR_INVALID || st == MM_ERR_UNSUPPORTED)
      return st;
    if (st != MM_OK && worst == MM_OK) {
      worst = st;
      msg = last_error_cstr();
    }
  }
  if (worst != MM_OK) set_error(msg);
  (void)S;
  return worst;
}

// Runs one admitted request on the slot's stream.  Never throws: any exception becomes the
// request's status, so that nothing can reach std::terminate from a worker thread.
mm_status serve_request(Server* S, Request* r, hipStream_t s) {
  try {
    if (r->work == nullptr) {
      std::unique_ptr<Work> w(new Work());
      const mm_status st = work_alloc(r->entry->plan, w.get());
      if (st != MM_OK) return st;
      r->work = w.release();
    }
    return run_request(S, r, s);
  } catch (const std::bad_alloc&) {
    return fail(MM_ERR_OOM, "host allocation failed");
  } catch (const std::exception& ex) {
    return fail(MM_ERR_HIP, std::string("internal error: ") + ex.what());
  } catch (...) {
    return fail(MM_ERR_HIP, "internal error: unknown exception in a serving worker");
  }
}

// Bookkeeping after a request ran (S->mu held).  Never throws: a workspace that cannot be put
// back in the idle pool is released instead.
void finish_request_locked(Server* S, Request* r, mm_status st) noexcept {
  CacheEntry* e = r->entry;
  // the reservation covered a new workspace (if any) and the block extra: the extra is
  // released now, a new workspace stays accounted while it lives in the idle pool
  S->in_use -= r->extra_bytes;
  if (r->uses_own) {
    e->own_work_free = true;
  } else if (r->work != nullptr) {
    bool kept = false;
    try {
      e->idle.push_back(r->work);
      kept = true;
    } catch (...) {
    }
    if (!kept) {
      S->in_use -= r->work->bytes;
      work_free(r->work);
      delete r->work;
    }
  } else {
    S->in_use -= r->reserved - r->extra_bytes;  // allocation failed: nothing to keep
  }
  r->work = nullptr;
  e->pins -= 1;
  e->last_use = ++S->tick;
  r->status = st;
  try {
    r->error = st == MM_OK ? std::string() : std::string(last_error_cstr());
  } catch (...) {
  }
  r->t_end = Clock::now();
  r->done = true;
  S->running -= 1;
  if (r->large) S->running_large -= 1;
  S->completed += 1;
}

void worker_loop(Server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t s = S->streams[slot];
  while (true) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        if (S->stop) return true;
        r = pick_locked(S);
        return r != nullptr;
      });
      if (r == nullptr) return;  // stopping
      r->slot = slot;
      r->t_start = Clock::now();
      S->running += 1;
      S->peak_running = std::max(S->peak_running, S->running);
      if (r->large) {
        S->running_large += 1;
        S->peak_large = std::max(S->peak_large, S->running_large);
      }
    }
    const mm_status st = serve_request(S, r, s);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      finish_request_locked(S, r, st);
    }
    S->cv_work.notify_all();
    S->cv_state.notify_all();
  }
}

// Thread body.  The loop only throws on a failure of the synchronisation primitives
// themselves; the thread then ends (the other slots keep serving) instead of terminating the
// process.
void worker(Server* S, int slot) noexcept {
  try {
    worker_loop(S, slot);
  } catch (...) {
  }
}

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

int64_t plan_estimate(const mm_geometry* g) {
  // pointing copies and per-sample plan data, pixel-domain vectors, a workspace
  int64_t b = 16 * g->n_samples + 120 * g->n_pix_global;
  int32_t lambda_max = 0;
  for (int i = 0; i < g->n_bands; ++i) {
    b += 4 * 65538;  // band spectrum upper bound (2^17 / 2 + 1)
    if (g->band_ncoef) lambda_max = std::max(lambda_max, g->band_ncoef[i] - 1);
  }
  // unfused products (flag or direct product): FP32 time-domain work vectors of the plan's
  // workspace
  const bool unfused = (g->flags & MM_FLAG_UNFUSED) != 0 || g->toeplitz_algo == MM_TOEPLITZ_DIRECT;
  if (unfused && lambda_max > 0) b += 8 * g->n_samples;
  // segments beyond 2^15: the spectrum-step table (NC <= 2^16 points per band) and the tiles
  // of the four-step transform (one per CU, at most 256 CUs)
  if (!unfused && lambda_max > 12288)
    b += (static_cast<int64_t>(g->n_bands) + 256) * 65536 * static_cast<int64_t>(sizeof(float2));
  return b;
}

}  // namespace

}  // namespace mm

using namespace mm;

extern "C" {

mm_status mm_server_create(const mm_server_opts* opts, mm_server_t** out) {
  if (!out) return fail(MM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  std::unique_ptr<Server> S;
  // On any failure: stop and join the workers already started and release the streams, so
  // that no joinable std::thread is ever destroyed (which would terminate the process).
  auto teardown = [&]() {
    if (!S) return;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    for (std::thread& t : S->workers)
      if (t.joinable()) t.join();
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    S->workers.clear();
    S->streams.clear();
  };
  try {
    S.reset(new Server());
    mm_status st = MM_OK;
    hipError_t e = hipGetDevice(&S->device);
    if (e != hipSuccess) return fail(MM_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    mm_server_opts o{};
    if (opts) o = *opts;
    S->n_slots = o.n_slots > 0 ? o.n_slots : 4;
    if (S->n_slots > 64) return fail(MM_ERR_INVALID, "n_slots > 64");
    S->max_bypass = o.max_bypass >= 0 ? o.max_bypass : 16;
    S->large_work = o.large_work > 0 ? o.large_work : 0;
    S->large_slots = o.large_slots > 0 ? o.large_slots : 1;
    if (o.hbm_budget > 0) {
      S->budget = o.hbm_budget;
    } else {
      size_t free_b = 0, total_b = 0;
      e = hipMemGetInfo(&free_b, &total_b);
      if (e != hipSuccess) return fail(MM_ERR_HIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
      S->budget = static_cast<int64_t>(0.8 * static_cast<double>(free_b));
    }
    S->streams.reserve(static_cast<size_t>(S->n_slots));
    S->workers.reserve(static_cast<size_t>(S->n_slots));
    for (int i = 0; i < S->n_slots && st == MM_OK; ++i) {
      hipStream_t s = nullptr;
      e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) {
        st = fail(MM_ERR_HIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
      } else {
        S->streams.push_back(s);
      }
    }
    if (st != MM_OK) {
      teardown();
      return st;
    }
    Server* raw = S.get();
    for (int i = 0; i < raw->n_slots; ++i) raw->workers.emplace_back(worker, raw, i);
    *out = reinterpret_cast<mm_server_t*>(S.release());
    return MM_OK;
  } catch (const std::exception& ex) {
    teardown();
    return fail(MM_ERR_HIP, std::string("server creation failed: ") + ex.what());
  } catch (...) {
    teardown();
    return fail(MM_ERR_HIP, "server creation failed");
  }
}

mm_status mm_server_destroy(mm_server_t* server) {
  if (!server) return MM_OK;
  Server* S = reinterpret_cast<Server*>(server);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Request* r : S->queue) {
      try {
        finish_unrun_locked(S, r, MM_ERR_INVALID, "server destroyed before the request ran");
      } catch (...) {
        r->done = true;  // the message could not be stored; the status is set
      }
    }
    S->queue.clear();
  }
  S->cv_work.notify_all();
  for (std::thread& t : S->workers) {
    try {
      if (t.joinable()) t.join();
    } catch (...) {
      // join only fails on a thread that cannot be joined; detach so that destroying the
      // std::thread object cannot terminate the process
      if (t.joinable()) t.detach();
    }
  }
  for (auto& kv : S->cache) {
    CacheEntry* e = kv.second.get();
    for (Work* w : e->idle) {
      work_free(w);
      delete w;
    }
    if (e->plan) {
      destroy_plan(e->plan);
    }
  }
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  delete S;
  return MM_OK;
}

mm_status mm_server_plan(mm_server_t* server, const mm_geometry* g, uint64_t key,
                         mm_plan_info_t* info) {
  if (!server) return fail(MM_ERR_INVALID, "server is NULL");
  Server* S = reinterpret_cast<Server*>(server);
  CacheEntry* e = nullptr;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
      auto it = S->cache.find(key);
      if (it == S->cache.end()) break;
      if (it->second->building) {
        S->cv_state.wait(lk);
        continue;
      }
      e = it->second.get();
      e->last_use = ++S->tick;
      S->hits += 1;
      e->pins += 1;  // keep it while the info is read
      break;
    }
    if (e == nullptr) {
      if (!g) return fail(MM_ERR_INVALID, "geometry is NULL and the key is not cached");
      auto ne = std::make_unique<CacheEntry>();
      ne->key = key;
      ne->building = true;
      e = ne.get();
      S->cache.emplace(key, std::move(ne));
      S->misses += 1;
      reclaim_locked(S, plan_estimate(g));
    }
  }
  if (!e->building) {
    mm_status st = MM_OK;
    if (info) st = mm_plan_info(reinterpret_cast<const mm_plan_t*>(e->plan), info);
    std::lock_guard<std::mutex> lk(S->mu);
    e->pins -= 1;
    return st;
  }
  // build outside the lock
  Plan* P = nullptr;
  hipStream_t s = nullptr;
  mm_status st = MM_OK;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    st = fail(MM_ERR_HIP, "stream creation failed");
  } else {
    try {
      st = build_plan(g, s, &P);
    } catch (const std::bad_alloc&) {
      st = fail(MM_ERR_OOM, "host allocation failed");
    } catch (...) {
      st = fail(MM_ERR_HIP, "internal error while building a plan");
    }
    (void)hipStreamDestroy(s);
  }
  std::string err = st == MM_OK ? std::string() : std::string(last_error_cstr());
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (st == MM_OK) {
      const int64_t bytes = P->device_bytes;
      if (bytes > S->budget) {
        destroy_plan(P);
        P = nullptr;
        st = MM_ERR_BUDGET;
        err = "plan needs " + std::to_string(bytes) + " bytes, budget is " + std::to_string(S->budget);
      } else {
        e->plan = P;
        e->plan_bytes = bytes;
        e->work_each = work_bytes(P);
        e->building = false;
        e->last_use = ++S->tick;
        S->in_use += bytes;
        reclaim_locked(S, 0);
        note_bytes(S);
      }
    }
    if (st != MM_OK) S->cache.erase(key);
  }
  S->cv_state.notify_all();
  S->cv_work.notify_all();
  if (st != MM_OK) return fail(st, err);
  if (info) return mm_plan_info(reinterpret_cast<const mm_plan_t*>(P), info);
  return MM_OK;
}

mm_status mm_submit(mm_server_t* server, uint64_t key, const float* d, int32_t k, int64_t ld_d,
                    double* x, const mm_solve_opts* opts, uint64_t* ticket) {
  if (!server || !ticket) return fail(MM_ERR_INVALID, "server or ticket is NULL");
  Server* S = reinterpret_cast<Server*>(server);
  if (k < 1) return fail(MM_ERR_INVALID, "k < 1");
  if (opts && opts->tol < 0) return fail(MM_ERR_INVALID, "tol < 0");
  if (opts && opts->use_x0 && opts->block != 0 && opts->block != 1)
    return fail(MM_ERR_INVALID, "use_x0 is not supported with block != 0/1");
  if (opts && opts->precond != 0)
    return fail(MM_ERR_UNSUPPORTED, "served solves use the block-Jacobi preconditioner");
  try {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(MM_ERR_INVALID, "server is stopping");
    auto it = S->cache.find(key);
    if (it == S->cache.end() || it->second->building)
      return fail(MM_ERR_NOT_FOUND, "plan key not cached: call mm_server_plan first");
    CacheEntry* e = it->second.get();
    const Plan* P = e->plan;
    if (k > 1 && ld_d < P->n_samples) return fail(MM_ERR_INVALID, "ld_d < n_samples");
    if ((P->n_samples > 0 && !d) || (P->n_kept > 0 && !x)) return fail(MM_ERR_INVALID, "NULL vector");
    auto r = std::make_unique<Request>();
    r->ticket = S->next_ticket++;
    r->entry = e;
    r->d = d;
    r->k = k;
    r->ld_d = k > 1 ? ld_d : P->n_samples;
    r->x = x;
    if (opts) r->opts = *opts;
    r->extra_bytes = block_extra_bytes(P, r->opts, k);
    r->large = S->large_work > 0 && P->n_samples * static_cast<int64_t>(k) >= S->large_work;
    // the plan's own workspace is always there once free: only the block extra must fit
    if (e->plan_bytes + r->extra_bytes > S->budget)
      return fail(MM_ERR_BUDGET, "request can never fit the memory budget");
    r->info.assign(static_cast<size_t>(k), mm_solve_info{});
    r->t_submit = Clock::now();
    e->pins += 1;
    e->last_use = ++S->tick;
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs.emplace(r->ticket, std::move(r));
    S->submitted += 1;
  } catch (const std::bad_alloc&) {
    return fail(MM_ERR_OOM, "host allocation failed");
  }
  S->cv_work.notify_one();
  return MM_OK;
}

static mm_status finish_poll(Server* S, uint64_t ticket, mm_solve_info* info,
                             mm_request_times* times, bool wait) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(MM_ERR_NOT_FOUND, "unknown ticket");
  Request* r = it->second.get();
  if (wait) S->cv_state.wait(lk, [&] { return r->done; });
  if (!r->done) return MM_PENDING;
  if (info) std::copy(r->info.begin(), r->info.end(), info);
  if (times) {
    const bool ran = r->slot >= 0;
    times->queued_ms = ran ? ms_between(r->t_submit, r->t_start) : 0.0;
    times->run_ms = ran ? ms_between(r->t_start, r->t_end) : 0.0;
    times->total_ms = ran ? ms_between(r->t_submit, r->t_end) : 0.0;
    times->slot = r->slot;
    times->pad = 0;
  }
  const mm_status st = r->status;
  const std::string err = r->error;
  S->reqs.erase(it);
  if (st != MM_OK) return fail(st, err);
  return MM_OK;
}

mm_status mm_poll(mm_server_t* server, uint64_t ticket, mm_solve_info* info,
                  mm_request_times* times) {
  if (!server) return fail(MM_ERR_INVALID, "server is NULL");
  return finish_poll(reinterpret_cast<Server*>(server), ticket, info, times, false);
}

mm_status mm_wait(mm_server_t* server, uint64_t ticket, mm_solve_info* info,
                  mm_request_times* times) {
  if (!server) return fail(MM_ERR_INVALID, "server is NULL");
  return finish_poll(reinterpret_cast<Server*>(server), ticket, info, times, true);
}

mm_status mm_server_stats(mm_server_t* server, mm_server_stats_t* out) {
  if (!server || !out) return fail(MM_ERR_INVALID, "server or out is NULL");
  Server* S = reinterpret_cast<Server*>(server);
  std::lock_guard<std::mutex> lk(S->mu);
  out->hbm_budget = S->budget;
  out->bytes_in_use = S->in_use;
  out->peak_bytes = S->peak;
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->plan_hits = S->hits;
  out->plan_misses = S->misses;
  out->evictions = S->evictions;
  out->queued = static_cast<int32_t>(S->queue.size());
  out->running = S->running;
  out->peak_running = S->peak_running;
  out->peak_large = S->peak_large;
  out->n_plans = static_cast<int32_t>(S->cache.size());
  return MM_OK;
}

}  // extern "C"
