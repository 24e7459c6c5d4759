// server.cpp -- continuous-batching alignment server on one device.
//
// Callers submit single-pair requests (sequences in host memory, copied at
// submit) and poll for completions.  One worker thread owns the device side:
//   * S slots, each a HIP stream (default priority) with a completion event
//     and a pinned host staging buffer that grows on demand and is reused;
//   * one device arena of the configured budget, reserved at creation and
//     carved per micro-batch (sequences, workspace with traceback codes,
//     results, CIGAR words).  A micro-batch is admitted when a slot is free
//     and the arena has a block for its footprint; otherwise it waits for a
//     running micro-batch to retire and release its block.
// Whenever a slot is free the worker takes the oldest pending request whose
// class (scoring and parameters) holds fewer slots than its quota, and every
// later pending request of that class (up to the configured pair and cell
// caps), plans them as one batch with the same
// planner and kernels as aln_execute, and enqueues upload, kernels and result
// download on the slot's stream.  Requests arriving while other micro-batches
// run join the next one; micro-batches on different streams overlap on the
// device.  Each pair's result depends only on the pair (the kernels are
// schedule-independent), so it is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "arena.h"
#include "runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0, tag = 0;
  int32_t scoring_id = 0;
  aln_params p{};
  std::vector<uint8_t> q, r;
  double t_submit = 0.0;
};

struct Done {
  aln_completion c;
  std::vector<uint32_t> cigar;
};

// Byte layout of one micro-batch, identical in the device block and (for the
// input section) in the slot's pinned staging buffer.
struct Layout {
  uint64_t q = 0, r = 0, q_off = 0, q_len = 0, r_off = 0, r_len = 0, in_end = 0;
  uint64_t ws = 0, res = 0, cig = 0, total = 0;  // device block
  uint64_t up = 0, pres = 0, pcig = 0, pinned = 0; // pinned buffer
};

Layout layout_for(const aln_plan *pl, uint64_t q_bytes, uint64_t r_bytes) {
  using alnrt::align_up;
  const uint64_t n = (uint64_t)pl->n;
  Layout L;
  L.q = 0;
  L.r = align_up(q_bytes);
  L.q_off = L.r + align_up(r_bytes);
  L.q_len = L.q_off + align_up(8 * n);
  L.r_off = L.q_len + align_up(4 * n);
  L.r_len = L.r_off + align_up(8 * n);
  L.in_end = L.r_len + align_up(4 * n);
  L.ws = L.in_end;
  L.res = L.ws + align_up(pl->ws_bytes);
  L.cig = L.res + align_up(sizeof(aln_result) * n);
  L.total = L.cig + align_up(4 * pl->cigar_words);
  L.up = L.in_end;
  L.pres = L.up + align_up(pl->upload_bytes);
  L.pcig = L.pres + align_up(sizeof(aln_result) * n);
  L.pinned = L.pcig + align_up(4 * pl->cigar_words);
  return L;
}

bool same_class(const Request &a, const Request &b) {
  return a.scoring_id == b.scoring_id && a.p.mode == b.p.mode && a.p.prune == b.p.prune &&
         a.p.band_w == b.p.band_w && a.p.xdrop == b.p.xdrop && a.p.width == b.p.width &&
         (a.p.want_cigar != 0) == (b.p.want_cigar != 0);
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  uint8_t *pinned = nullptr;
  uint64_t pinned_cap = 0;
  bool busy = false;
  std::vector<Request> reqs;
  aln_plan *plan = nullptr;
  Layout L;
  uint64_t arena_off = 0;
  uint64_t batch_id = 0;
  double t_launch = 0.0;
};

} // namespace

struct aln_server {
  aln_ctx *ctx = nullptr;   // worker's context: own device copies of the scorings
  aln_ctx *vctx = nullptr;  // submit-side context for planning checks (host only)
  aln_server_cfg cfg{};
  int device = 0;
  uint8_t *d_arena = nullptr;
  alnrt::Arena arena;       // worker only
  std::vector<Slot> slots;  // worker only
  std::thread worker;
  Clock::time_point t0;

  std::mutex mu;            // guards everything below
  std::condition_variable cv_work, cv_done;
  std::deque<Request> incoming;
  std::deque<Done> done;
  bool stop = false;
  uint64_t next_id = 1;
  uint64_t outstanding = 0;
  aln_server_stats stats{};
  std::string worker_err;

  std::mutex submit_mu;     // serialises submitters (vctx)
  std::string err;          // last error of an API call

  // worker-local
  std::deque<Request> pending;
  uint64_t next_batch = 1;
  bool waiting = false;

  double now() const {
    return std::chrono::duration<double>(Clock::now() - t0).count();
  }
};

namespace {

aln_status sfail(aln_server *s, aln_status st, const char *msg) {
  if (s) s->err = msg;
  return st;
}

// Deliver completions (worker thread).
void deliver(aln_server *s, std::vector<Done> &out, int64_t cells) {
  std::lock_guard<std::mutex> lk(s->mu);
  for (Done &d : out) s->done.push_back(std::move(d));
  s->stats.completed += out.size();
  s->stats.cells += cells;
  s->outstanding -= out.size();
  s->cv_done.notify_all();
}

void fail_requests(aln_server *s, std::vector<Request> &reqs, aln_status err, uint64_t batch,
                   double t_launch, const char *why) {
  std::vector<Done> out;
  for (Request &r : reqs) {
    Done d;
    memset(&d.c, 0, sizeof d.c);
    d.c.id = r.id;
    d.c.tag = r.tag;
    d.c.error = err;
    d.c.batch_pairs = (int32_t)reqs.size();
    d.c.batch_id = batch;
    d.c.t_submit = r.t_submit;
    d.c.t_launch = t_launch;
    d.c.t_done = s->now();
    out.push_back(std::move(d));
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (why) s->worker_err = why;
  }
  deliver(s, out, 0);
}

void retire(aln_server *s, Slot &sl) {
  const int32_t n = (int32_t)sl.reqs.size();
  const aln_result *res = reinterpret_cast<const aln_result *>(sl.pinned + sl.L.pres);
  const uint32_t *words = reinterpret_cast<const uint32_t *>(sl.pinned + sl.L.pcig);
  const double t = s->now();
  std::vector<Done> out(n);
  int64_t cells = 0;
  for (int32_t k = 0; k < n; ++k) {
    Done &d = out[k];
    memset(&d.c, 0, sizeof d.c);
    d.c.id = sl.reqs[k].id;
    d.c.tag = sl.reqs[k].tag;
    d.c.result = res[k];
    d.c.error = ALN_OK;
    d.c.batch_pairs = n;
    d.c.batch_id = sl.batch_id;
    d.c.t_submit = sl.reqs[k].t_submit;
    d.c.t_launch = sl.t_launch;
    d.c.t_done = t;
    cells += res[k].cells;
    const int32_t len = res[k].cigar_len;
    const int64_t off = res[k].cigar_off;
    if (len > 0 && off >= 0 && (uint64_t)(off + len) <= sl.plan->cigar_words)
      d.cigar.assign(words + off, words + off + len);
    d.c.result.cigar_off = 0;
  }
  s->arena.release(sl.arena_off);
  aln_plan_destroy(sl.plan);
  sl.plan = nullptr;
  sl.reqs.clear();
  sl.busy = false;
  deliver(s, out, cells);
}

// Try to start a micro-batch on `sl`.  Returns 1 when launched, 0 when the
// head batch must wait for memory, -1 when requests were completed with an
// error instead.
int launch_next(aln_server *s, Slot &sl, size_t head_idx, bool any_busy) {
  const Request &head = s->pending[head_idx];
  std::vector<size_t> pick;
  int64_t cells = 0;
  const size_t scan =
      std::min<size_t>(s->pending.size(), head_idx + 4 * (size_t)s->cfg.max_batch_pairs + 64);
  for (size_t k = head_idx; k < scan && (int32_t)pick.size() < s->cfg.max_batch_pairs; ++k) {
    const Request &r = s->pending[k];
    if (!same_class(r, head)) continue;
    const int64_t c = (int64_t)r.q.size() * (int64_t)r.r.size();
    if (!pick.empty() && s->cfg.max_batch_cells > 0 && cells + c > s->cfg.max_batch_cells) break;
    pick.push_back(k);
    cells += c;
  }
  aln_plan *pl = nullptr;
  Layout L;
  uint64_t off = 0;
  std::vector<int32_t> ql, rl;
  for (;;) {
    ql.clear();
    rl.clear();
    uint64_t qb = 0, rb = 0;
    for (size_t k : pick) {
      ql.push_back((int32_t)s->pending[k].q.size());
      rl.push_back((int32_t)s->pending[k].r.size());
      qb += s->pending[k].q.size();
      rb += s->pending[k].r.size();
    }
    aln_status st = alnrt::plan_build(s->ctx, head.scoring_id, &head.p, (int32_t)pick.size(),
                                      ql.data(), rl.data(), &pl);
    if (st == ALN_OK) {
      L = layout_for(pl, qb, rb);
      if (s->arena.alloc(L.total, &off)) break;
      aln_plan_destroy(pl);
      pl = nullptr;
    }
    if (pick.size() > 1) { // a smaller batch may plan or fit
      pick.resize(pick.size() / 2);
      continue;
    }
    if (st == ALN_OK && any_busy) { // wait for a running micro-batch to free memory
      if (!s->waiting) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.admission_waits++;
      }
      s->waiting = true;
      return 0;
    }
    // a single request that cannot be planned or placed even in an idle arena
    std::vector<Request> one;
    one.push_back(std::move(s->pending[pick[0]]));
    s->pending.erase(s->pending.begin() + (long)pick[0]);
    fail_requests(s, one, st == ALN_OK ? ALN_E_CAPACITY : st, 0, s->now(),
                  st == ALN_OK ? "request larger than the server's device budget"
                               : s->ctx->err.c_str());
    return -1;
  }
  s->waiting = false;

  // pinned staging: [inputs | task upload | results | CIGAR words]
  if (L.pinned > sl.pinned_cap) {
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    sl.pinned = nullptr;
    sl.pinned_cap = 0;
    const uint64_t cap = std::max<uint64_t>(L.pinned + L.pinned / 4, 1 << 20);
    if (hipHostMalloc((void **)&sl.pinned, cap, hipHostMallocDefault) != hipSuccess) {
      s->arena.release(off);
      aln_plan_destroy(pl);
      std::vector<Request> reqs;
      for (size_t i = pick.size(); i-- > 0;) {
        reqs.push_back(std::move(s->pending[pick[i]]));
        s->pending.erase(s->pending.begin() + (long)pick[i]);
      }
      fail_requests(s, reqs, ALN_E_NOMEM, 0, s->now(), "pinned staging allocation failed");
      return -1;
    }
    sl.pinned_cap = cap;
  }
  // move the picked requests out of the queue, keeping their order
  sl.reqs.clear();
  sl.reqs.reserve(pick.size());
  for (size_t k : pick) sl.reqs.push_back(std::move(s->pending[k]));
  for (size_t i = pick.size(); i-- > 0;) s->pending.erase(s->pending.begin() + (long)pick[i]);

  const int32_t n = (int32_t)sl.reqs.size();
  uint8_t *h = sl.pinned;
  int64_t *h_qoff = reinterpret_cast<int64_t *>(h + L.q_off);
  int32_t *h_qlen = reinterpret_cast<int32_t *>(h + L.q_len);
  int64_t *h_roff = reinterpret_cast<int64_t *>(h + L.r_off);
  int32_t *h_rlen = reinterpret_cast<int32_t *>(h + L.r_len);
  uint64_t qo = 0, ro = 0;
  for (int32_t k = 0; k < n; ++k) {
    const Request &r = sl.reqs[k];
    if (!r.q.empty()) memcpy(h + L.q + qo, r.q.data(), r.q.size());
    if (!r.r.empty()) memcpy(h + L.r + ro, r.r.data(), r.r.size());
    h_qoff[k] = (int64_t)qo;
    h_roff[k] = (int64_t)ro;
    h_qlen[k] = (int32_t)r.q.size();
    h_rlen[k] = (int32_t)r.r.size();
    qo += r.q.size();
    ro += r.r.size();
  }
  pl->pinned = h + L.up;
  pl->own_pinned = false;
  alnrt::plan_stage(pl, pl->pinned);

  uint8_t *d = s->d_arena + off;
  aln_batch b;
  b.n = n;
  b.q = d + L.q;
  b.q_off = reinterpret_cast<const int64_t *>(d + L.q_off);
  b.q_len = reinterpret_cast<const int32_t *>(d + L.q_len);
  b.r = d + L.r;
  b.r_off = reinterpret_cast<const int64_t *>(d + L.r_off);
  b.r_len = reinterpret_cast<const int32_t *>(d + L.r_len);
  aln_result *d_res = reinterpret_cast<aln_result *>(d + L.res);
  uint32_t *d_cig = pl->cigar_words ? reinterpret_cast<uint32_t *>(d + L.cig) : nullptr;

  sl.plan = pl;
  sl.L = L;
  sl.arena_off = off;
  sl.batch_id = s->next_batch++;
  sl.t_launch = s->now();
  aln_status st = ALN_OK;
  hipError_t e = hipMemcpyAsync(d, h, L.in_end, hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess) {
    st = alnrt::plan_run(s->ctx, pl, &b, d + L.ws, d_res, d_cig, sl.stream, false);
    if (st == ALN_OK)
      e = hipMemcpyAsync(h + L.pres, d_res, sizeof(aln_result) * (size_t)n,
                         hipMemcpyDeviceToHost, sl.stream);
    if (st == ALN_OK && e == hipSuccess && d_cig)
      e = hipMemcpyAsync(h + L.pcig, d_cig, 4 * pl->cigar_words, hipMemcpyDeviceToHost,
                         sl.stream);
    if (st == ALN_OK && e == hipSuccess) e = hipEventRecord(sl.ev, sl.stream);
  }
  if (st != ALN_OK || e != hipSuccess) {
    // wait for whatever was enqueued before releasing its memory
    (void)hipStreamSynchronize(sl.stream);
    const std::string why = st != ALN_OK ? s->ctx->err : std::string(hipGetErrorString(e));
    s->arena.release(off);
    aln_plan_destroy(pl);
    sl.plan = nullptr;
    fail_requests(s, sl.reqs, st != ALN_OK ? st : ALN_E_DEVICE, sl.batch_id, sl.t_launch,
                  why.c_str());
    sl.reqs.clear();
    return -1;
  }
  sl.busy = true;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.batches++;
    int32_t inflight = 0;
    for (const Slot &x : s->slots) inflight += x.busy ? 1 : 0;
    s->stats.peak_inflight = std::max(s->stats.peak_inflight, inflight);
    s->stats.peak_arena_bytes = std::max<uint64_t>(s->stats.peak_arena_bytes, s->arena.used());
  }
  return 1;
}

void worker_main(aln_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    while (!s->incoming.empty()) {
      s->pending.push_back(std::move(s->incoming.front()));
      s->incoming.pop_front();
    }
    const bool stopping = s->stop;
    lk.unlock();

    bool progressed = false;
    for (Slot &sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipSuccess) {
        retire(s, sl);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        (void)hipStreamSynchronize(sl.stream);
        s->arena.release(sl.arena_off);
        aln_plan_destroy(sl.plan);
        sl.plan = nullptr;
        sl.busy = false;
        fail_requests(s, sl.reqs, ALN_E_DEVICE, sl.batch_id, sl.t_launch, hipGetErrorString(q));
        sl.reqs.clear();
        progressed = true;
      }
    }
    while (!s->pending.empty()) {
      Slot *free_slot = nullptr;
      bool any_busy = false;
      for (Slot &sl : s->slots) {
        if (sl.busy) any_busy = true;
        else if (!free_slot) free_slot = &sl;
      }
      if (!free_slot) break;
      // oldest pending request whose class is under its stream quota
      size_t h = 0;
      const size_t look = std::min<size_t>(s->pending.size(), 4096);
      for (; h < look; ++h) {
        int32_t held = 0;
        for (const Slot &sl : s->slots)
          if (sl.busy && same_class(sl.reqs.front(), s->pending[h])) ++held;
        if (held < s->cfg.class_streams) break;
      }
      if (h == look) break;
      const int r = launch_next(s, *free_slot, h, any_busy);
      if (r == 0) break;
      progressed = true;
    }
    bool any_busy = false;
    for (const Slot &sl : s->slots) any_busy = any_busy || sl.busy;

    lk.lock();
    if (stopping && s->pending.empty() && s->incoming.empty() && !any_busy) break;
    if (progressed || !s->incoming.empty()) continue;
    if (any_busy) {
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    } else if (s->pending.empty()) {
      s->cv_work.wait(lk, [&] { return s->stop || !s->incoming.empty(); });
    }
  }
}

void destroy_resources(aln_server *s) {
  (void)hipSetDevice(s->device);
  for (Slot &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.plan) aln_plan_destroy(sl.plan);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  s->slots.clear();
  if (s->d_arena) (void)hipFree(s->d_arena);
  s->d_arena = nullptr;
  if (s->vctx) {
    s->vctx->dsc.clear(); // borrowed pointers, owned by s->ctx
    aln_destroy(s->vctx);
  }
  if (s->ctx) aln_destroy(s->ctx);
}

} // namespace

extern "C" {

aln_status aln_server_create(aln_ctx *ctx, const aln_server_cfg *cfg, aln_server **out) {
  if (!ctx || !cfg || !out) return ALN_E_INVAL;
  *out = nullptr;
  if (cfg->streams < 1 || cfg->streams > 16)
    return alnrt::fail(ctx, ALN_E_INVAL, "streams must lie in 1..16");
  if (cfg->max_batch_pairs < 1)
    return alnrt::fail(ctx, ALN_E_INVAL, "max_batch_pairs must be >= 1");
  if (cfg->max_batch_cells < 0)
    return alnrt::fail(ctx, ALN_E_INVAL, "max_batch_cells must be >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess)
    return alnrt::fail(ctx, ALN_E_DEVICE, "hipSetDevice failed");
  uint64_t budget = cfg->hbm_budget;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
      return alnrt::fail(ctx, ALN_E_DEVICE, "hipMemGetInfo failed");
    budget = (uint64_t)free_b / 2;
  }
  if (budget < (1u << 20)) return alnrt::fail(ctx, ALN_E_INVAL, "hbm_budget below 1 MiB");

  aln_server *s = new (std::nothrow) aln_server;
  if (!s) return alnrt::fail(ctx, ALN_E_NOMEM, "server allocation");
  s->cfg = *cfg;
  s->cfg.hbm_budget = budget;
  if (s->cfg.class_streams <= 0) s->cfg.class_streams = std::max(1, cfg->streams / 4);
  s->cfg.class_streams = std::min(s->cfg.class_streams, cfg->streams);
  s->device = ctx->device;
  s->t0 = Clock::now();
  aln_status st = aln_create(&s->ctx, ctx->device);
  if (st == ALN_OK) st = aln_create(&s->vctx, ctx->device);
  // the worker gets its own device copies of every scoring set so far
  for (size_t k = 0; st == ALN_OK && k < ctx->hsc.size(); ++k) {
    alnk::DevScoring *d = nullptr;
    if (hipMalloc(&d, sizeof(alnk::DevScoring)) != hipSuccess ||
        hipMemcpy(d, &ctx->hsc[k], sizeof(alnk::DevScoring), hipMemcpyHostToDevice) !=
            hipSuccess) {
      if (d) (void)hipFree(d);
      st = ALN_E_DEVICE;
      break;
    }
    s->ctx->dsc.push_back(d);
    s->ctx->hsc.push_back(ctx->hsc[k]);
    s->vctx->dsc.push_back(d);
    s->vctx->hsc.push_back(ctx->hsc[k]);
  }
  if (st == ALN_OK && hipMalloc((void **)&s->d_arena, budget) != hipSuccess) st = ALN_E_NOMEM;
  if (st == ALN_OK) {
    s->arena.reset(budget, alnrt::kAlign);
    s->slots.resize((size_t)cfg->streams);
    for (Slot &sl : s->slots) {
      if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
        st = ALN_E_DEVICE;
        break;
      }
    }
  }
  if (st != ALN_OK) {
    destroy_resources(s);
    delete s;
    return alnrt::fail(ctx, st, "server set-up failed (device budget %llu bytes)",
                       (unsigned long long)budget);
  }
  s->stats.arena_bytes = s->arena.size();
  s->stats.streams = cfg->streams;
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    destroy_resources(s);
    delete s;
    return alnrt::fail(ctx, ALN_E_NOMEM, "worker thread");
  }
  *out = s;
  return ALN_OK;
}

void aln_server_destroy(aln_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  destroy_resources(s);
  delete s;
}

aln_status aln_server_submit(aln_server *s, const aln_request *rq, uint64_t *id) {
  if (!s || !rq) return ALN_E_INVAL;
  std::lock_guard<std::mutex> sub(s->submit_mu);
  if (rq->q_len < 0 || rq->r_len < 0 || (rq->q_len > 0 && !rq->q) || (rq->r_len > 0 && !rq->r))
    return sfail(s, ALN_E_INVAL, "bad sequence pointer or length");
  if (rq->scoring_id < 0 || rq->scoring_id >= (int32_t)s->vctx->hsc.size())
    return sfail(s, ALN_E_INVAL, "unknown scoring id (set scorings before creating the server)");
  // plan the request alone: rejects what the kernels cannot run and sizes it
  aln_plan *pl = nullptr;
  aln_status st = alnrt::plan_build(s->vctx, rq->scoring_id, &rq->params, 1, &rq->q_len,
                                    &rq->r_len, &pl);
  if (st != ALN_OK) return sfail(s, st, s->vctx->err.c_str());
  const Layout L = layout_for(pl, (uint64_t)rq->q_len, (uint64_t)rq->r_len);
  aln_plan_destroy(pl);
  if (s->arena.round_up(L.total) > s->cfg.hbm_budget / alnrt::kAlign * alnrt::kAlign)
    return sfail(s, ALN_E_CAPACITY, "request footprint exceeds the server's device budget");
  Request r;
  r.tag = rq->tag;
  r.scoring_id = rq->scoring_id;
  r.p = rq->params;
  r.q.assign(rq->q, rq->q + rq->q_len);
  r.r.assign(rq->r, rq->r + rq->r_len);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r.id = s->next_id++;
    r.t_submit = s->now();
    if (id) *id = r.id;
    s->incoming.push_back(std::move(r));
    s->stats.submitted++;
    s->outstanding++;
  }
  s->cv_work.notify_one();
  return ALN_OK;
}

int32_t aln_server_poll(aln_server *s, aln_completion *out, int32_t max, uint32_t *cigar,
                        uint64_t cigar_cap, uint64_t *cigar_used, int32_t wait_us) {
  if (!s || max < 0 || (max > 0 && !out)) return ALN_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->done.empty(); });
  int32_t k = 0;
  uint64_t used = 0;
  while (k < max && !s->done.empty()) {
    Done &d = s->done.front();
    if (!d.cigar.empty()) {
      if (!cigar || used + d.cigar.size() > cigar_cap) {
        if (k == 0) {
          s->err = "CIGAR buffer too small for the next completion (" +
                   std::to_string(d.cigar.size()) + " words)";
          return ALN_E_CAPACITY;
        }
        break;
      }
      memcpy(cigar + used, d.cigar.data(), 4 * d.cigar.size());
      d.c.result.cigar_off = (int64_t)used;
      used += d.cigar.size();
    }
    out[k++] = d.c;
    s->done.pop_front();
  }
  if (cigar_used) *cigar_used = used;
  return k;
}

aln_status aln_server_drain(aln_server *s, int32_t timeout_ms) {
  if (!s) return ALN_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto pred = [&] { return s->outstanding == 0; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, pred);
    return ALN_OK;
  }
  if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
    s->err = "drain timed out";
    return ALN_E_CAPACITY;
  }
  return ALN_OK;
}

double aln_server_clock(const aln_server *s) { return s ? s->now() : 0.0; }

aln_status aln_server_get_stats(aln_server *s, aln_server_stats *st) {
  if (!s || !st) return ALN_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  return ALN_OK;
}

const char *aln_server_last_error(aln_server *s) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->err.empty() && !s->worker_err.empty()) return s->worker_err.c_str();
  return s->err.c_str();
}

} // extern "C"
