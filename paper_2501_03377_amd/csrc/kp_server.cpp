// Request server: a plan cache under an HBM budget, admission control and
// worker threads that run continuous batches (kp_server_* in kpcg.h).  A
// worker keeps a batch of max_batch slots running on one plan; a queued
// request of the same kind takes a free slot at the next iteration boundary
// and leaves it as soon as its own solve ends.  Every request is Algorithm 1
// with the pseudoinverse preconditioner of Algs. 4-7, run per slot by the
// solver (kp_slots.h); this file only schedules.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/kpcg.h"
#include "kp_budget.h"
#include "kp_slots.h"

namespace kp {
std::mutex& api_mutex();   // kp_solver.hip: serialises allocations with graph capture
}

namespace {

struct PlanKey {
  int nx, ny, nz, bc[3], prec;
  bool operator==(const PlanKey& o) const {
    return nx == o.nx && ny == o.ny && nz == o.nz && bc[0] == o.bc[0] && bc[1] == o.bc[1] &&
           bc[2] == o.bc[2] && prec == o.prec;
  }
};

PlanKey key_of(const kp_request& r) {
  PlanKey k{r.nx, r.ny, r.nz, {r.bc[0], r.bc[1], r.nz > 1 ? r.bc[2] : 0}, r.prec};
  return k;
}

// Requests that may share one kp_solve call.
bool same_batch(const kp_request& a, const kp_request& b) {
  return key_of(a) == key_of(b) && a.tol == b.tol && a.max_iter == b.max_iter &&
         a.flags == b.flags;
}

struct Pending {
  kp_request r;
  double t_submit;
};

// A plan instance belongs to one worker, which binds its own workspace to
// it: a plan then keeps its captured graphs from batch to batch, and the
// cache holds only the packed operators of each plan.
struct PlanEntry {
  PlanKey key;
  int owner = 0;         // worker
  kp_plan* plan = nullptr;
  bool busy = false;
  uint64_t last = 0;     // use tick, for LRU eviction
  size_t bytes = 0;      // resident operators
  int64_t ws_epoch = -1; // owner's workspace generation the plan is bound to
  int expect = 0;        // iterations the plan's last solve made (0: none yet)
};

struct Worker {
  std::thread th;
  hipStream_t stream = nullptr;
  double* stage = nullptr;    // device: eta batch then u batch
  size_t stage_bytes = 0;
  void* ws = nullptr;         // solver workspace shared by this worker's plans
  size_t ws_bytes = 0;
  int64_t ws_epoch = 0;       // bumped whenever ws is reallocated
};

}  // namespace

struct kp_server {
  int device = 0;
  int max_batch = 1;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;    // queue changed, memory freed, or stop
  std::condition_variable cv_done;    // completions available
  std::deque<Pending> queue;
  std::deque<kp_completion> done;
  std::vector<PlanEntry*> plans;
  std::vector<Worker> workers;
  kp::Budget mem;          // plans, workspaces and staging against the budget
  int running = 0;        // workers holding a plan for a batch
  uint64_t tick = 0;
  kp_server_stats st{};
  bool stop = false;
  char last_error[256] = "";      // most recent failed batch
  char last_error_out[256] = "";  // copy handed to the caller

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Most iterations per step of a continuous batch that no queued request
// waits to join: a step then runs until the first slot is expected to end
// (by the iteration count of the plan's last solve), so a solve takes few
// host round trips; a newcomer waits at most that long for a free slot.  A
// step's results do not depend on its length.
constexpr int kStepIters = 4;

size_t vec_bytes(const kp_request& r) { return (size_t)r.nx * r.ny * r.nz * sizeof(double); }

void complete(kp_server* s, const Pending& p, int status, const kp_result* res, int batch,
              int worker, double t_start, double t_end) {
  kp_completion c{};
  c.id = p.r.id;
  c.status = status;
  c.batch = batch;
  c.worker = worker;
  c.t_submit = p.t_submit;
  c.t_start = t_start;
  c.t_end = t_end;
  if (res) {
    c.iterations = res->iterations;
    c.rel_res = res->rel_res;
    c.true_rel_res = res->true_rel_res;
    c.err_est = res->err_est;
  }
  s->done.push_back(c);
  s->st.completed += 1;
  if (status == KP_ENOMEM) s->st.rejected += 1;
}

void account(kp_server* s, long long delta) { s->mem.add(delta); }

// Frees idle plans, least recently used first, until `need` more bytes fit the
// budget.  Called with the lock held; returns the plans to destroy (after
// unlocking) or sets *fits = false.
std::vector<kp_plan*> make_room(kp_server* s, size_t need, bool* fits) {
  std::vector<kp_plan*> victims;
  *fits = true;
  while (!s->mem.fits(need)) {
    PlanEntry* lru = nullptr;
    for (PlanEntry* e : s->plans)
      if (!e->busy && (!lru || e->last < lru->last)) lru = e;
    if (!lru) { *fits = false; break; }
    victims.push_back(lru->plan);
    account(s, -(long long)lru->bytes);
    s->plans.erase(std::find(s->plans.begin(), s->plans.end(), lru));
    delete lru;
    s->st.plans_evicted += 1;
  }
  return victims;
}

void destroy_plans(std::vector<kp_plan*>& v) {
  for (kp_plan* p : v) kp_plan_destroy(p);
  v.clear();
}

// Status of a slot whose solve has ended.
int slot_status(const kp::RhsState& x) {
  switch (x.done) {
    case kp::CONVERGED: case kp::ZERO_RHS: return KP_OK;
    case kp::BREAKDOWN: return KP_EBREAKDOWN;
    case kp::NONFINITE: return KP_ENONFINITE;
    default: return KP_NOT_CONVERGED;
  }
}

void worker_main(kp_server* s, int w) {
  (void)hipSetDevice(s->device);
  Worker& me = s->workers[w];
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    if (s->queue.empty()) break;   // stopping and drained

    // the oldest request opens a continuous batch of its kind
    std::vector<Pending> incoming;
    incoming.push_back(s->queue.front());
    s->queue.pop_front();
    const kp_request r0 = incoming[0].r;
    const PlanKey key = key_of(r0);
    const size_t vb = vec_bytes(r0);
    const size_t stage_need = 2 * vb * (size_t)s->max_batch;

    // acquire this worker's plan of this key, or make one within the budget
    PlanEntry* entry = nullptr;
    std::vector<kp_plan*> victims;
    size_t ws_need = 0;
    int fail = KP_OK;
    for (;;) {
      for (PlanEntry* e : s->plans)
        if (e->owner == w && e->key == key) { entry = e; break; }
      if (entry) entry->busy = true;   // not evictable while we make room
      kp_plan* fresh = nullptr;
      size_t fresh_bytes = 0;
      if (!entry) {
        lk.unlock();
        destroy_plans(victims);
        int rc = kp_plan_create(&fresh, key.nx, key.ny, key.nz, key.bc, key.prec, s->max_batch,
                                me.stream);
        if (rc == KP_OK) {
          fresh_bytes = kp_plan_resident_bytes(fresh);
          ws_need = kp_plan_workspace_bytes(fresh, s->max_batch);
        }
        lk.lock();
        if (rc != KP_OK) {
          fail = rc;
          snprintf(s->last_error, sizeof s->last_error, "kp_plan_create: status %d %s", rc,
                   kp_last_error());
          break;
        }
      } else {
        ws_need = kp_plan_workspace_bytes(entry->plan, s->max_batch);
      }
      const size_t grow = (me.stage_bytes < stage_need ? stage_need - me.stage_bytes : 0) +
                          (me.ws_bytes < ws_need ? ws_need - me.ws_bytes : 0);
      bool fits = false;
      std::vector<kp_plan*> v = make_room(s, grow + fresh_bytes, &fits);
      victims.insert(victims.end(), v.begin(), v.end());
      if (fits) {
        if (fresh) {
          entry = new PlanEntry();
          entry->key = key;
          entry->owner = w;
          entry->plan = fresh;
          entry->bytes = fresh_bytes;
          entry->busy = true;
          s->plans.push_back(entry);
          account(s, (long long)fresh_bytes);
          s->st.plans_created += 1;
        }
        account(s, (long long)grow);   // the buffers grow before the solve
        break;
      }
      // does not fit: wait until a running batch releases its plan (which
      // makes it evictable), or reject when no batch is running
      if (entry) entry->busy = false;
      entry = nullptr;
      if (fresh) {
        lk.unlock();
        kp_plan_destroy(fresh);
        lk.lock();
      }
      if (s->running == 0) { fail = KP_ENOMEM; break; }
      s->cv_work.wait(lk);
    }
    if (fail != KP_OK) {
      lk.unlock();
      destroy_plans(victims);
      lk.lock();
      const double t = s->now();
      complete(s, incoming[0], fail, nullptr, 1, w, t, t);
      s->cv_done.notify_all();
      s->cv_work.notify_all();
      continue;
    }
    entry->last = ++s->tick;
    s->running += 1;
    s->st.batches += 1;
    // the first requests of the batch: every queued one of the same kind
    bool waiting = false;   // a request of this kind is left queued
    for (auto it = s->queue.begin(); it != s->queue.end();) {
      if (same_batch(it->r, r0)) {
        if ((int)incoming.size() < s->max_batch) {
          incoming.push_back(*it);
          it = s->queue.erase(it);
          continue;
        }
        waiting = true;
      }
      ++it;
    }
    lk.unlock();
    destroy_plans(victims);

    // ---- buffers of this worker (no lock held; accounting under it) ----
    int rc = KP_OK;
    const char* failed = nullptr;   // failing step
    if (me.stage_bytes < stage_need) {
      std::lock_guard<std::mutex> alk(kp::api_mutex());
      if (me.stage) (void)hipFree(me.stage);
      me.stage = nullptr;
      const bool okm = hipMalloc((void**)&me.stage, stage_need) == hipSuccess;
      {
        std::lock_guard<std::mutex> mlk(s->mu);
        me.stage_bytes = kp::regrow(s->mem, me.stage_bytes, stage_need, okm);
      }
      if (!okm) { me.stage = nullptr; rc = KP_ENOMEM; failed = "hipMalloc of the slot buffers"; }
    }
    if (rc == KP_OK && me.ws_bytes < ws_need) {
      std::lock_guard<std::mutex> alk(kp::api_mutex());
      if (me.ws) (void)hipFree(me.ws);
      me.ws = nullptr;
      me.ws_epoch += 1;
      const bool okm = hipMalloc(&me.ws, ws_need) == hipSuccess;
      {
        std::lock_guard<std::mutex> mlk(s->mu);
        me.ws_bytes = kp::regrow(s->mem, me.ws_bytes, ws_need, okm);
      }
      if (!okm) { me.ws = nullptr; rc = KP_ENOMEM; failed = "hipMalloc of the worker workspace"; }
    }
    if (rc == KP_OK && entry->ws_epoch != me.ws_epoch) {
      // rebinding drops the plan's captured graphs (they point into the old buffer)
      rc = kp_plan_set_workspace(entry->plan, me.ws, me.ws_bytes);
      if (rc == KP_OK) entry->ws_epoch = me.ws_epoch;
      else failed = "kp_plan_set_workspace";
    }
    const size_t n = vb / sizeof(double);
    double* eta_b = me.stage;
    double* u_b = me.stage + n * (size_t)s->max_batch;
    if (rc == KP_OK) {
      kp_plan_set_stream(entry->plan, me.stream);
      rc = kp::slots_open(entry->plan, eta_b, u_b, r0.tol, r0.flags & ~KP_FLAG_NO_GRAPH);
      if (rc != KP_OK) failed = "slots_open";
    }

    // ---- the continuous batch: steps until no slot is busy ----
    std::vector<Pending> req(s->max_batch);
    std::vector<char> busy(s->max_batch, 0);
    std::vector<double> t_start(s->max_batch, 0.0);
    std::vector<int> iter_of(s->max_batch, 0);   // iterations made, from the last step
    std::vector<char> joined(s->max_batch, 0);   // starts in the next step
    int active = 0;
    std::vector<int> fin;
    for (;;) {
      // newcomers take free slots; they start at this step
      for (const Pending& p : incoming) {
        int slot = 0;
        while (busy[slot]) ++slot;
        req[slot] = p;
        busy[slot] = 1;
        iter_of[slot] = 0;
        joined[slot] = 1;
        active += 1;
        t_start[slot] = s->now();
        if (rc != KP_OK) continue;
        const hipMemcpyKind k =
            p.r.mem == KP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (hipMemcpyAsync(eta_b + n * slot, p.r.eta, vb, k, me.stream) != hipSuccess) {
          rc = KP_EHIP;
          failed = "hipMemcpyAsync of a right-hand side";
        } else if ((rc = kp::slots_mark(entry->plan, slot, kp::JOINING)) != KP_OK) {
          failed = "slots_mark";
        }
      }
      incoming.clear();
      if (active == 0) break;
      // one iteration per step while a request of this kind waits for a slot;
      // otherwise up to the first expected exit (a joining slot first takes
      // its start), at most kStepIters, within every slot's iteration cap
      int iters = (waiting || entry->expect == 0) ? 1 : kStepIters;
      for (int slot = 0; slot < s->max_batch; ++slot) {
        if (!busy[slot]) continue;
        const int left = entry->expect - iter_of[slot] + (joined[slot] ? 1 : 0);
        iters = std::min(iters, std::max(1, left));
        iters = std::min(iters, std::max(1, r0.max_iter - iter_of[slot]));
      }
      // launches cover the slots up to the last busy one (newcomers take the
      // lowest free slots)
      int nslots = 0;
      for (int slot = 0; slot < s->max_batch; ++slot)
        if (busy[slot]) nslots = slot + 1;
      const kp::RhsState* m = nullptr;
      if (rc == KP_OK && (rc = kp::slots_step(entry->plan, iters, nslots)) != KP_OK)
        failed = "slots_step";
      std::fill(joined.begin(), joined.end(), 0);
      if (rc == KP_OK && !(m = kp::slots_wait(entry->plan))) {
        rc = KP_EHIP;
        failed = "slots_wait";
      }
      // slots whose solve ended (with their exit step) leave; their answers
      // are copied out before the completion is posted
      fin.clear();
      for (int slot = 0; slot < s->max_batch && rc == KP_OK; ++slot) {
        if (!busy[slot]) continue;
        const kp::RhsState& x = m[slot];
        iter_of[slot] = x.iter;
        if (kp::terminal(x.done) && x.exit_gen == 2) {
          fin.push_back(slot);
          const kp_request& r = req[slot].r;
          if (r.u) {
            const hipMemcpyKind k =
                r.mem == KP_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
            if (hipMemcpyAsync(r.u, u_b + n * slot, vb, k, me.stream) != hipSuccess) {
              rc = KP_EHIP;
              failed = "hipMemcpyAsync of a solution";
            }
          }
        } else if (x.done == kp::RUNNING && x.iter >= r0.max_iter) {
          if ((rc = kp::slots_mark(entry->plan, slot, kp::CAPPED)) != KP_OK)
            failed = "slots_mark";
        }
      }
      if (rc == KP_OK && !fin.empty() && hipStreamSynchronize(me.stream) != hipSuccess) {
        rc = KP_EHIP;
        failed = "hipStreamSynchronize after the solution copies";
      }
      lk.lock();
      const double t_end = s->now();
      if (rc != KP_OK) {
        // every request still in the batch fails; no newcomer joins
        snprintf(s->last_error, sizeof s->last_error, "continuous batch on worker %d: %s (%s)",
                 w, failed ? failed : "?", kp_last_error());
        for (int slot = 0; slot < s->max_batch; ++slot)
          if (busy[slot]) complete(s, req[slot], rc, nullptr, active, w, t_start[slot], t_end);
        s->cv_done.notify_all();
        lk.unlock();
        break;
      }
      for (int slot : fin) {
        const kp::RhsState& x = m[slot];
        entry->expect = x.iter;
        kp_result res{};
        res.iterations = x.iter;
        res.rel_res = x.rel_res;
        res.true_rel_res = x.true_rel_res;
        res.err_est = x.err_est;
        complete(s, req[slot], slot_status(x), &res, active, w, t_start[slot], t_end);
        busy[slot] = 0;
        active -= 1;
      }
      if (!fin.empty()) s->cv_done.notify_all();
      // queued requests of the same kind take the free slots
      waiting = false;
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (same_batch(it->r, r0)) {
          if (active + (int)incoming.size() < s->max_batch) {
            incoming.push_back(*it);
            it = s->queue.erase(it);
            continue;
          }
          waiting = true;
        }
        ++it;
      }
      lk.unlock();
    }
    if (entry->plan) kp::slots_close(entry->plan);

    lk.lock();
    entry->busy = false;
    entry->last = ++s->tick;
    s->running -= 1;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

bool valid_request(const kp_request* r) {
  if (!r || !r->eta) return false;
  if (r->nx < 3 || r->ny < 3 || !(r->nz == 1 || r->nz >= 3)) return false;
  if ((double)r->nx * r->ny * r->nz >= 2147483648.0) return false;
  for (int a = 0; a < (r->nz > 1 ? 3 : 2); ++a)
    if (r->bc[a] < KP_BC_P || r->bc[a] > KP_BC_ND) return false;
  if (r->prec < KP_PREC_F64 || r->prec > KP_PREC_I8X6) return false;
  if (r->prec == KP_PREC_I8X7 || r->prec == KP_PREC_I8X6) {
    // the int8 split preconditioner's plans need every axis a multiple of 16
    // and at most 512
    const int n[3] = {r->nx, r->ny, r->nz};
    for (int a = 0; a < (r->nz > 1 ? 3 : 2); ++a)
      if (n[a] % 16 != 0 || n[a] > 512) return false;
  }
  if (!(r->tol > 0.0) || !std::isfinite(r->tol)) return false;
  if (r->max_iter < 1 || r->max_iter > 1000000) return false;
  if (r->flags & ~(KP_FLAG_NO_PRECOND | KP_FLAG_FLEX_BETA | KP_FLAG_RESIDUAL_ONLY | KP_FLAG_NO_GRAPH))
    return false;
  if (r->mem != KP_MEM_DEVICE && r->mem != KP_MEM_HOST) return false;
  if (r->mem == KP_MEM_DEVICE && (((uintptr_t)r->eta & 15u) || ((uintptr_t)r->u & 15u)))
    return false;
  return true;
}

}  // namespace

extern "C" {

int kp_server_create(kp_server** out, size_t hbm_budget, int workers, int max_batch) {
  if (!out || workers < 1 || workers > 64 || max_batch < 1 || max_batch > 65535) return KP_EINVAL;
  *out = nullptr;
  kp_server* s = new kp_server();
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; return KP_EHIP; }
  s->mem.limit = hbm_budget;
  s->max_batch = max_batch;
  s->t0 = std::chrono::steady_clock::now();
  s->workers.resize(workers);
  for (Worker& w : s->workers) {
    if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) {
      for (Worker& v : s->workers)
        if (v.stream) (void)hipStreamDestroy(v.stream);
      delete s;
      return KP_EHIP;
    }
  }
  for (int i = 0; i < workers; ++i) s->workers[i].th = std::thread(worker_main, s, i);
  *out = s;
  return KP_OK;
}

int kp_server_submit(kp_server* s, const kp_request* r) {
  if (!s || !valid_request(r)) return KP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return KP_EINVAL;
    s->queue.push_back(Pending{*r, s->now()});
    s->st.submitted += 1;
  }
  s->cv_work.notify_all();   // also wakes a worker waiting for memory; all re-check
  return KP_OK;
}

int kp_server_poll(kp_server* s, kp_completion* out, int max, double timeout_s) {
  if (!s || !out || max < 1 || !(timeout_s >= 0.0)) return KP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_s > 0.0)
    s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                        [&] { return !s->done.empty(); });
  int n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  return n;
}

double kp_server_now(const kp_server* s) { return s ? s->now() : 0.0; }

int kp_server_stats_get(kp_server* s, kp_server_stats* out) {
  if (!s || !out) return KP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->plans_cached = (int32_t)s->plans.size();
  out->queued = (int32_t)s->queue.size();
  out->hbm_used = s->mem.used;
  out->hbm_high_water = s->mem.high;
  out->hbm_budget = s->mem.limit;
  return KP_OK;
}

const char* kp_server_last_error(kp_server* s) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  std::memcpy(s->last_error_out, s->last_error, sizeof s->last_error);
  return s->last_error_out;
}

void kp_server_destroy(kp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (Worker& w : s->workers)
    if (w.th.joinable()) w.th.join();
  for (PlanEntry* e : s->plans) {
    kp_plan_destroy(e->plan);
    delete e;
  }
  for (Worker& w : s->workers) {
    if (w.stage) (void)hipFree(w.stage);
    if (w.ws) (void)hipFree(w.ws);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  delete s;
}

}  // extern "C"
