// Request server: continuous batching of dense t-SVD requests on one device.
//
// A worker thread owns the context while the server lives.  Each cycle it
//   1. admits waiting requests in arrival order while the free device budget
//      covers their footprint (Gram, split-K partials, finish sums and the
//      staged copy of a host-resident A) and a slot is free; host-resident A is
//      copied on the copy stream at once;
//   2. launches admitted requests as one batch (grouped Gram, team power
//      kernel, grouped finish) on an idle lane -- each lane is a compute
//      stream -- into the CUs that no running engine launch holds;
//   3. when a lane's completion event has fired, releases that batch's memory
//      and completes its tickets (latency = completion - submission, host
//      clock).
// The persistent engine launch of a batch holds one CU per workgroup until
// that workgroup finds the batch's queue empty; each workgroup then stores
// the batch's id into its entry of a flag array in coherent pinned host
// memory before it exits.  The worker counts a running launch's CUs as its
// grid minus the flags set, and a new batch takes only requests whose team
// fits the CUs left, with a grid of at most that many workgroups.  The grids
// of all running launches therefore never exceed the chip, so every launch's
// workgroups become resident once the short Gram and finish kernels around
// them drain, and no launch waits on another.  A request that arrives while a
// batch runs starts as soon as the running batch's teams release enough CUs
// (at once, when they already have), overlapping the rest of that batch.
// Team sizes and Gram chunking depend on the request alone, so each result is
// the same alone and in any mix.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batched.h"
#include "common.h"

namespace tsvd {
namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device allocation (256-byte granules), with
// coalescing of neighbouring free ranges.
class Arena {
 public:
  void init(char* base, size_t bytes) {
    base_ = base;
    cap_ = bytes;
    free_.clear();
    free_[0] = bytes;
    used_ = 0;
  }
  char* alloc(size_t bytes) {
    bytes = align256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_ += bytes;
      sizes_[off] = bytes;
      return base_ + off;
    }
    return nullptr;
  }
  void release(char* p) {
    if (!p) return;
    const size_t off = (size_t)(p - base_);
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t bytes = s->second, start = off;
    sizes_.erase(s);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + bytes) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        bytes += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = bytes;
  }
  size_t used() const { return used_; }
  size_t capacity() const { return cap_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
  std::map<size_t, size_t> sizes_;  // live allocations
};

enum ReqState { WAITING, ADMITTED, RUNNING, DONE };

struct Request {
  uint64_t ticket = 0;
  tsvd_problem prob = {};
  std::vector<int32_t> fixed;  // copy of opts.fixed_iters
  int32_t loc = TSVD_LOC_DEVICE;
  ReqState state = WAITING;
  Clock::time_point t_submit, t_done;
  char* ws = nullptr;        // per-problem workspace
  char* staged = nullptr;    // device copy of a host-resident A
  hipEvent_t copied = nullptr;
  size_t footprint = 0;
  int team = 0;             // power team size (workgroups), from the request alone
  tsvd_status status = TSVD_OK;
  tsvd_info info = {};
  std::vector<int32_t> iters;
  std::vector<double> lambda;
};

}  // namespace
}  // namespace tsvd

using namespace tsvd;

struct Lane {
  hipStream_t compute = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<uint64_t> running;
  tsvd::BatchPlan plan;
  std::vector<tsvd_problem> run_probs;
  char* batch_ws = nullptr;
  bool active = false;
  char* hpin = nullptr;  // pinned host staging of the batch's descriptors and results
  size_t hpin_bytes = 0;
  int* flags = nullptr;  // coherent pinned host memory, one int per power workgroup
  int batch_id = 0;      // what the current engine launch's workgroups store on exit
  int grid = 0;          // its workgroups
  // CUs the lane's engine launch may still hold: its grid less the workgroups that have left
  int live() const {
    if (!active) return 0;
    int gone = 0;
    const volatile int* f = flags;
    for (int i = 0; i < grid; i++) gone += f[i] == batch_id ? 1 : 0;
    return grid - gone;
  }
};

struct tsvd_server {
  tsvd_ctx* ctx = nullptr;
  tsvd_server_config cfg = {};
  hipStream_t copy = nullptr;
  std::vector<Lane> lanes;
  int next_batch_id = 1;
  char* pool = nullptr;
  Arena arena;    // request workspaces and staged copies of host A
  Arena tables;   // the running batches' tables and team buffers
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::thread worker;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> waiting;                    // arrival order
  std::unordered_map<uint64_t, Request*> reqs;     // every ticket not yet collected
  std::vector<uint64_t> admitted;                  // admitted, not yet launched
  int in_flight = 0;                               // admitted + running
  // statistics
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, batched_problems = 0;
  int64_t peak_bytes = 0, lanes_busy_max = 0, overlapped = 0;
  std::vector<double> latencies_ms;
  std::string error;

  int busy_lanes() const {
    int b = 0;
    for (const Lane& l : lanes) b += l.active ? 1 : 0;
    return b;
  }
};

namespace {

// Device bytes a request holds while admitted: its workspace (Gram, split-K
// partials, finish sums) and the staged copy of a host-resident A.
size_t request_footprint(const ProbPlan& p, const tsvd_problem& q, int32_t loc) {
  size_t f = p.ws_bytes;
  if (loc == TSVD_LOC_PINNED_HOST) f += align256((size_t)q.m * q.lda * 4);
  return f;
}

void finish_request(tsvd_server* s, Request* r, tsvd_status st) {
  r->status = st;
  r->state = DONE;
  r->t_done = Clock::now();
  const double ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  r->info.latency_ms = ms;
  if (st == TSVD_ERR_REJECTED) return;  // counted apart; not in the latency record
  s->latencies_ms.push_back(ms);
  if (st == TSVD_OK) s->completed++;
  else s->failed++;
}

void release_request(tsvd_server* s, Request* r) {
  s->arena.release(r->ws);
  s->arena.release(r->staged);
  r->ws = r->staged = nullptr;
  if (r->copied) {
    (void)hipEventDestroy(r->copied);
    r->copied = nullptr;
  }
  s->in_flight--;
}

// step 1: admission (called with the lock held)
void admit(tsvd_server* s) {
  while (!s->waiting.empty() && s->in_flight < s->cfg.max_slots) {
    Request* r = s->reqs[s->waiting.front()];
    BatchPlan one;
    tsvd_status st = batch_plan(s->ctx, 1, &r->prob, one);
    if (st != TSVD_OK) {  // arguments were checked at submit; planning limits remain
      s->waiting.pop_front();
      finish_request(s, r, st);
      s->cv_done.notify_all();
      continue;
    }
    const ProbPlan& p = one.P[0];
    r->team = p.G;
    r->footprint = request_footprint(p, r->prob, r->loc);
    if (r->footprint > s->arena.capacity() || one.batch_ws_bytes > s->tables.capacity()) {
      s->waiting.pop_front();
      s->rejected++;
      finish_request(s, r, TSVD_ERR_REJECTED);
      s->cv_done.notify_all();
      continue;
    }
    if (s->arena.used() + r->footprint > s->arena.capacity()) break;  // wait for memory
    r->ws = s->arena.alloc(p.ws_bytes);
    if (r->ws && r->loc == TSVD_LOC_PINNED_HOST) r->staged = s->arena.alloc((size_t)r->prob.m * r->prob.lda * 4);
    if (!r->ws || (r->loc == TSVD_LOC_PINNED_HOST && !r->staged)) {  // fragmented: wait for frees
      s->arena.release(r->ws);
      s->arena.release(r->staged);
      r->ws = r->staged = nullptr;
      break;
    }
    if (r->loc == TSVD_LOC_PINNED_HOST) {
      const size_t bytes = (size_t)r->prob.m * r->prob.lda * 4;
      if (hipEventCreateWithFlags(&r->copied, hipEventDisableTiming) != hipSuccess ||
          hipMemcpyAsync(r->staged, r->prob.A, bytes, hipMemcpyHostToDevice, s->copy) != hipSuccess ||
          hipEventRecord(r->copied, s->copy) != hipSuccess) {
        s->error = std::string("staging copy: ") + hipGetErrorString(hipGetLastError());
        s->waiting.pop_front();
        s->in_flight++;
        release_request(s, r);
        finish_request(s, r, TSVD_ERR_HIP);
        s->cv_done.notify_all();
        continue;
      }
      r->prob.A = r->staged;
    }
    s->waiting.pop_front();
    r->state = ADMITTED;
    s->admitted.push_back(r->ticket);
    s->in_flight++;
    s->peak_bytes = std::max<int64_t>(s->peak_bytes, (int64_t)s->arena.used());
  }
}

// step 2: launch the admitted requests as one batch on an idle lane (lock held)
void launch(tsvd_server* s) {
  if (s->admitted.empty()) return;
  Lane* L = nullptr;
  for (Lane& l : s->lanes)
    if (!l.active) {
      L = &l;
      break;
    }
  if (!L) return;
  // CUs no running engine launch holds.  Beside a running batch, a new one
  // launches only once 7/8 of the chip is free (a batch's grid is fixed at
  // launch: started into a small remainder, its teams would queue on few CUs
  // long after the running batch has ended; at the serving mix, two lanes gave
  // p50 196 / 179 / 164 / 155 ms with 4/8 .. 7/8 free, one lane 115 ms).  It takes admitted
  // requests in arrival order while their teams fit those CUs, and stops at
  // the first that does not (a request with a large team is not overtaken
  // indefinitely: it waits at the head until enough CUs are released).
  int free_cus = s->ctx->num_cu;
  for (const Lane& l : s->lanes) free_cus -= l.live();
  if (free_cus <= 0 || (s->busy_lanes() > 0 && 8 * free_cus < 7 * s->ctx->num_cu)) return;
  const int maxb = s->cfg.max_batch;
  std::vector<uint64_t> take;
  for (size_t i = 0; i < s->admitted.size() && (int)take.size() < maxb; i++) {
    if (s->reqs[s->admitted[i]]->team > free_cus) break;
    take.push_back(s->admitted[i]);
  }
  while (!take.empty()) {
    L->run_probs.clear();
    for (uint64_t t : take) L->run_probs.push_back(s->reqs[t]->prob);
    // the cap leaves every team as planned alone (each fits) and bounds the grid
    tsvd_status st = batch_plan(s->ctx, (int)take.size(), L->run_probs.data(), L->plan, free_cus);
    if (st != TSVD_OK) {
      for (uint64_t t : take) {
        Request* r = s->reqs[t];
        release_request(s, r);
        finish_request(s, r, st);
        s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), t));
      }
      s->cv_done.notify_all();
      return;
    }
    L->batch_ws = s->tables.alloc(L->plan.batch_ws_bytes);
    if (L->batch_ws) break;
    take.pop_back();  // tables too large for the free part of their region: a smaller batch
  }
  if (take.empty()) return;
  if (L->hpin_bytes < L->plan.host_bytes()) {  // the lane is idle: its old area is free
    if (L->hpin) (void)hipHostFree(L->hpin);
    L->hpin = nullptr;
    L->hpin_bytes = 0;
    const size_t want = 2 * L->plan.host_bytes();
    if (hipHostMalloc((void**)&L->hpin, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      L->hpin = nullptr;
    } else {
      L->hpin_bytes = want;
    }
  }
  for (uint64_t t : take) s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), t));
  std::vector<char*> pbase;
  for (uint64_t t : take) {
    Request* r = s->reqs[t];
    if (r->copied) (void)hipStreamWaitEvent(L->compute, r->copied, 0);
    pbase.push_back(r->ws);
    r->state = RUNNING;
  }
  const int id = s->next_batch_id++;
  tsvd_status st = batch_enqueue(s->ctx, L->run_probs.data(), L->plan, L->batch_ws, pbase.data(), L->compute, L->ev,
                                 L->hpin, L->flags, id);
  if (st == TSVD_OK && hipEventRecord(L->done, L->compute) != hipSuccess) st = TSVD_ERR_HIP;
  if (st != TSVD_OK) {
    s->error = s->ctx->last_error;
    (void)hipStreamSynchronize(L->compute);
    for (uint64_t t : take) {
      Request* r = s->reqs[t];
      release_request(s, r);
      finish_request(s, r, st);
    }
    s->tables.release(L->batch_ws);
    L->batch_ws = nullptr;
    s->cv_done.notify_all();
    return;
  }
  if (s->busy_lanes() > 0) s->overlapped++;
  L->running = take;
  L->batch_id = id;
  L->grid = L->plan.grid;
  L->active = true;
  s->lanes_busy_max = std::max<int64_t>(s->lanes_busy_max, s->busy_lanes());
  s->batches++;
  s->batched_problems += (int64_t)take.size();
}

// step 3: collect the finished batches (lock held)
void collect(tsvd_server* s) {
  for (Lane& L : s->lanes) {
    if (!L.active) continue;
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) continue;
    for (size_t i = 0; i < L.running.size(); i++) {
      Request* r = s->reqs[L.running[i]];
      tsvd_status st = TSVD_ERR_HIP;
      if (q == hipSuccess) {
        r->info.iters = r->iters.data();
        r->info.lambda = r->lambda.data();
        st = batch_problem_result(L.plan, L.run_probs[i], (int)i, &r->info);
        float tg = 0, te = 0, tf = 0, tt = 0;
        (void)hipEventElapsedTime(&tg, L.ev[0], L.ev[1]);
        (void)hipEventElapsedTime(&te, L.ev[1], L.ev[2]);
        (void)hipEventElapsedTime(&tf, L.ev[2], L.ev[3]);
        (void)hipEventElapsedTime(&tt, L.ev[0], L.ev[3]);
        r->info.t_gram_ms = tg;
        r->info.t_eig_ms = te;
        r->info.t_final_ms = tf;
        r->info.t_total_ms = tt;
        r->info.workspace_bytes = (int64_t)r->footprint;
        r->info.h2d_bytes = r->loc == TSVD_LOC_PINNED_HOST ? (int64_t)(r->prob.m * r->prob.lda * 4) : 0;
      } else {
        s->error = std::string("batch completion: ") + hipGetErrorString(q);
        (void)hipGetLastError();
      }
      release_request(s, r);
      finish_request(s, r, st);
    }
    s->tables.release(L.batch_ws);
    L.batch_ws = nullptr;
    L.running.clear();
    L.active = false;
    s->cv_done.notify_all();
  }
}

void worker_main(tsvd_server* s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    collect(s);
    admit(s);
    launch(s);
    const bool busy = s->busy_lanes() > 0;
    if (s->stop && s->waiting.empty() && s->admitted.empty() && !busy) break;
    if (busy) {
      // poll the device batch; new submissions wake the worker early
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    } else if (s->waiting.empty() || s->in_flight >= s->cfg.max_slots) {
      s->cv_work.wait(lk, [&] { return s->stop || (!s->waiting.empty() && s->in_flight < s->cfg.max_slots); });
    } else {
      // waiting requests that do not fit while nothing runs: memory is held by
      // admitted requests that launch next cycle
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

}  // namespace

extern "C" {

tsvd_status tsvd_server_create(tsvd_ctx* ctx, const tsvd_server_config* cfg, tsvd_server** out) {
  if (!ctx || !cfg || !out) return TSVD_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->hbm_budget <= 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "server hbm_budget must be > 0");
  if (cfg->max_slots < 0 || cfg->max_batch < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "negative slots or batch");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "hipSetDevice");
  if (cfg->lanes < 0 || cfg->lanes > 8) return fail(ctx, TSVD_ERR_INVALID_ARG, "lanes must be in [0, 8]");
  tsvd_server* s = new tsvd_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  if (s->cfg.max_slots == 0) s->cfg.max_slots = 256;
  if (s->cfg.max_batch == 0 || s->cfg.max_batch > s->cfg.max_slots) s->cfg.max_batch = s->cfg.max_slots;
  // one lane by default: at the serving mix's load two or three lanes kept the
  // same request rate with higher latency (a batch's grid is fixed at launch)
  if (s->cfg.lanes == 0) s->cfg.lanes = 1;
  s->lanes.resize(s->cfg.lanes);
  bool ok = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) == hipSuccess;
  for (Lane& L : s->lanes) {
    ok = ok && hipStreamCreateWithFlags(&L.compute, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&L.done, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc((void**)&L.flags, (size_t)ctx->num_cu * sizeof(int), hipHostMallocCoherent) == hipSuccess;
    if (ok) memset(L.flags, 0, (size_t)ctx->num_cu * sizeof(int));
    for (int i = 0; i < 4 && ok; i++) ok = hipEventCreate(&L.ev[i]) == hipSuccess;
  }
  if (!ok) {
    tsvd_server_destroy(s);
    return fail(ctx, TSVD_ERR_HIP, "server streams/events");
  }
  if (hipMalloc((void**)&s->pool, (size_t)cfg->hbm_budget) != hipSuccess) {
    (void)hipGetLastError();
    s->pool = nullptr;
    tsvd_server_destroy(s);
    return fail(ctx, TSVD_ERR_OUT_OF_MEMORY, "server pool of %lld bytes", (long long)cfg->hbm_budget);
  }
  // tables region: 1/16 of the budget within [16 MiB, 512 MiB] (at most half)
  size_t tb = std::min<size_t>(std::max<size_t>((size_t)cfg->hbm_budget / 16, (size_t)16 << 20), (size_t)512 << 20);
  tb = std::min(tb, (size_t)cfg->hbm_budget / 2) & ~(size_t)255;
  s->tables.init(s->pool, tb);
  s->arena.init(s->pool + tb, (size_t)cfg->hbm_budget - tb);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return TSVD_OK;
}

tsvd_status tsvd_server_submit(tsvd_server* s, const tsvd_problem* p, int32_t loc, uint64_t* ticket) {
  if (!s || !p || !ticket) return TSVD_ERR_INVALID_ARG;
  if (loc != TSVD_LOC_DEVICE && loc != TSVD_LOC_PINNED_HOST) return TSVD_ERR_INVALID_ARG;
  if (loc == TSVD_LOC_PINNED_HOST) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p->A) != hipSuccess || attr.type != hipMemoryTypeHost) {
      (void)hipGetLastError();
      std::lock_guard<std::mutex> g(s->mu);
      s->error = "PINNED_HOST A must be page-locked host memory";
      return TSVD_ERR_INVALID_ARG;
    }
  }
  Request* r = new Request();
  r->prob = *p;
  r->loc = loc;
  const int64_t mn = std::min(p->m, p->n);
  const int k = p->opts.k == -1 ? (int)mn : p->opts.k;
  if (p->opts.fixed_iters && k > 0 && k <= mn) {
    r->fixed.assign(p->opts.fixed_iters, p->opts.fixed_iters + k);
    r->prob.opts.fixed_iters = r->fixed.data();
  }
  // argument checks now, so that bad requests fail at submission
  {
    BatchPlan one;
    tsvd_problem q = r->prob;
    if (loc == TSVD_LOC_PINNED_HOST) q.A = (const void*)16;  // any aligned non-null stand-in for the check
    std::lock_guard<std::mutex> g(s->mu);
    const tsvd_status st = batch_plan(s->ctx, 1, &q, one);
    if (st != TSVD_OK) {
      s->error = s->ctx->last_error;
      delete r;
      return st;
    }
  }
  r->iters.assign(k, 0);
  r->lambda.assign(k, 0.0);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(s->mu);
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->waiting.push_back(r->ticket);
    s->submitted++;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return TSVD_OK;
}

static void copy_out(Request* r, tsvd_info* info) {
  if (!info) return;
  int32_t* it = info->iters;
  double* la = info->lambda;
  *info = r->info;
  info->iters = it;
  info->lambda = la;
  if (it) memcpy(it, r->iters.data(), r->iters.size() * 4);
  if (la) memcpy(la, r->lambda.data(), r->lambda.size() * 8);
}

tsvd_status tsvd_server_poll(tsvd_server* s, uint64_t ticket, int32_t* done, tsvd_info* info, int32_t* status) {
  if (!s || !done) return TSVD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return TSVD_ERR_INVALID_ARG;
  Request* r = it->second;
  *done = r->state == DONE ? 1 : 0;
  if (!*done) return TSVD_OK;
  copy_out(r, info);
  if (status) *status = r->status;
  s->reqs.erase(it);
  delete r;
  return TSVD_OK;
}

tsvd_status tsvd_server_wait(tsvd_server* s, uint64_t ticket, tsvd_info* info) {
  if (!s) return TSVD_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return TSVD_ERR_INVALID_ARG;
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->state == DONE; });
  copy_out(r, info);
  const tsvd_status st = r->status;
  s->reqs.erase(ticket);
  delete r;
  return st;
}

tsvd_status tsvd_server_get_stats(tsvd_server* s, tsvd_server_stats* out) {
  if (!s || !out) return TSVD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->rejected = s->rejected;
  out->batches = s->batches;
  out->mean_batch = s->batches ? (double)s->batched_problems / s->batches : 0.0;
  out->peak_bytes = s->peak_bytes;
  out->in_flight = s->in_flight;
  out->waiting = (int64_t)s->waiting.size();
  out->lanes_busy_max = s->lanes_busy_max;
  out->overlapped = s->overlapped;
  std::vector<double> v = s->latencies_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {  // nearest-rank percentile
      size_t i = (size_t)ceil(q * v.size());
      if (i < 1) i = 1;
      return v[std::min(i, v.size()) - 1];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / v.size();
    out->max_ms = v.back();
  }
  return TSVD_OK;
}

const char* tsvd_server_last_error(const tsvd_server* s) { return s ? s->error.c_str() : "null server"; }

void tsvd_server_destroy(tsvd_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);
  for (Lane& L : s->lanes)
    if (L.compute) (void)hipStreamSynchronize(L.compute);
  if (s->copy) (void)hipStreamSynchronize(s->copy);
  for (auto& kv : s->reqs) {
    if (kv.second->copied) (void)hipEventDestroy(kv.second->copied);
    delete kv.second;
  }
  if (s->pool) (void)hipFree(s->pool);
  for (Lane& L : s->lanes) {
    if (L.hpin) (void)hipHostFree(L.hpin);
    if (L.flags) (void)hipHostFree(L.flags);
    if (L.done) (void)hipEventDestroy(L.done);
    for (int i = 0; i < 4; i++)
      if (L.ev[i]) (void)hipEventDestroy(L.ev[i]);
    if (L.compute) (void)hipStreamDestroy(L.compute);
  }
  if (s->copy) (void)hipStreamDestroy(s->copy);
  delete s;
}

}  // extern "C"
