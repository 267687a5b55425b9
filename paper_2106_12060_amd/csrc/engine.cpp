// Serving engine: continuous batching of CCA / FDA solves on one device.
//
// One device pool (a single allocation, carved first-fit) holds every
// admitted request's workspace and staged copies for the life of its solve.
// Worker slots each own a host thread and a HIP stream of default priority;
// an idle slot takes the head of the FIFO queue as soon as the head's
// footprint fits in the pool, so solves that arrive while others run start
// when a slot and memory free up, and admitted solves overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace srp;

namespace {

constexpr int kMaxSlots = 16;
constexpr size_t kAlign = 256;

size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, cap) with coalescing of neighbouring holes.
class PoolMap {
 public:
  void reset(size_t cap) {
    cap_ = cap;
    holes_.clear();
    if (cap) holes_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = holes_.begin(); it != holes_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rem = it->second - bytes;
      holes_.erase(it);
      if (rem) holes_[o + bytes] = rem;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = holes_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != holes_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      holes_.erase(nx);
    }
    if (it != holes_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        holes_.erase(it);
      }
    }
    used_ -= bytes;
  }
  size_t cap() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> holes_;
};

struct Job {
  uint64_t ticket = 0;
  srp_request req{};
  size_t footprint = 0;
  double t_submit = 0.0;
};

// Staged copies a request needs in front of its solve workspace.
size_t staged_bytes(const srp_request& q) {
  if (q.stage == SRP_STAGE_NONE) return 0;
  size_t b = bytes_of<uint16_t>((size_t)q.n * q.dx) + bytes_of<uint16_t>((size_t)q.n * q.dy);
  if (q.stage == SRP_STAGE_BF16_FP8)
    b += bytes_of<uint8_t>((size_t)q.n * q.dx) + bytes_of<uint8_t>((size_t)q.n * q.dy) + bytes_of<double>(q.dx) +
         bytes_of<double>(q.dy);
  return b;
}

bool sizes_ok(const srp_request& q) {
  if (q.n < 1 || q.n >= (int64_t(1) << 31) || q.k < 1 || q.sketch_size < 1 || q.dx < 1 || q.dy < 1) return false;
  // a sketch narrower than a view keeps that view's metric in Woodbury form, which needs lambda > 0
  if (q.problem == SRP_PROBLEM_CCA)
    return (q.sketch_size >= q.dx || q.lambda_x > 0.0) && (q.sketch_size >= q.dy || q.lambda_y > 0.0);
  if (q.problem == SRP_PROBLEM_LDA)
    return q.dy >= 2 && (q.sketch_size >= q.dx || q.lambda_x > 0.0) && q.stage == SRP_STAGE_NONE;
  return false;
}

size_t footprint(const srp_request& q) {
  if (!sizes_ok(q)) return 0;
  if (q.problem == SRP_PROBLEM_LDA)
    return lda_ws_bytes(q.n, q.dx, q.dy, q.k, q.sketch_size, q.dtype, q.opt.sketch);
  int skin = q.dtype;
  if (q.stage == SRP_STAGE_BF16_FP8) skin = SRP_FP8E4M3;
  else if (q.stage == SRP_STAGE_NONE && q.opt.sketch_x) skin = q.opt.sketch_dtype;
  size_t ws = cca_ws_bytes(q.n, q.dx, q.dy, q.k, q.sketch_size, q.dtype, q.opt.sketch, skin);
  if (q.stage == SRP_STAGE_BF16_FP8) ws = std::max(ws, stage_fp8_ws_bytes(std::max(q.dx, q.dy)));
  return staged_bytes(q) + ws;
}

}  // namespace

struct srp_engine {
  int device = 0;
  char* pool_mem = nullptr;
  PoolMap pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> queue;
  std::unordered_set<uint64_t> in_flight;
  std::unordered_map<uint64_t, srp_result> done;
  uint64_t next_ticket = 1;
  bool stop = false;
  int running = 0, peak_running = 0;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  // grouped ticks (SRP_ENGINE_GROUPED): one group per (k bound, size
  // class), so that the solves ticking together have passes of similar
  // length (a tick waits for its slowest member's pass)
  static constexpr int kSizeClasses = 5;
  TickGroup* groups[2][kSizeClasses] = {};
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Stages (if asked) and solves one admitted request inside its pool block.
int run_job(srp_engine* e, const Job& job, char* block, hipStream_t st, srp_result& r) {
  const srp_request& q = job.req;
  srp_options opt = q.opt;
  Arena ar{block, job.footprint, 0};
  if (q.problem == SRP_PROBLEM_CCA && q.stage != SRP_STAGE_NONE) {
    SRP_REQUIRE(q.dtype == SRP_F32, "staging needs F32 data");
    SRP_REQUIRE(q.X && q.Y, "null pointer argument");
    uint16_t* xb = ar.take<uint16_t>((size_t)q.n * q.dx);
    uint16_t* yb = ar.take<uint16_t>((size_t)q.n * q.dy);
    SRP_REQUIRE(xb && yb, "engine block too small for the staged copies");
    SRP_TRY(stage_bf16_run((const float*)q.X, q.n, q.dx, xb, st));
    SRP_TRY(stage_bf16_run((const float*)q.Y, q.n, q.dy, yb, st));
    opt.lowp_x = xb;
    opt.lowp_y = yb;
    if (q.stage == SRP_STAGE_BF16_FP8) {
      uint8_t* cx = ar.take<uint8_t>((size_t)q.n * q.dx);
      uint8_t* cy = ar.take<uint8_t>((size_t)q.n * q.dy);
      double* sx = ar.take<double>(q.dx);
      double* sy = ar.take<double>(q.dy);
      SRP_REQUIRE(cx && cy && sx && sy, "engine block too small for the staged copies");
      // the column-maximum scratch lives where the solve's workspace will
      // be; the solve runs after it on the same stream
      Arena s1{ar.base + ar.used, ar.cap - ar.used, 0};
      SRP_TRY(stage_fp8_run(q.X, SRP_F32, q.n, q.dx, cx, sx, s1, st));
      Arena s2{ar.base + ar.used, ar.cap - ar.used, 0};
      SRP_TRY(stage_fp8_run(q.Y, SRP_F32, q.n, q.dy, cy, sy, s2, st));
      opt.sketch_x = cx;
      opt.sketch_y = cy;
      opt.sketch_dtype = SRP_FP8E4M3;
      opt.sketch_scale_x = sx;
      opt.sketch_scale_y = sy;
    }
  }
  SolveCtx ctx;
  ctx.side = nullptr;   // one stream per slot: both views in order on it
  ctx.ws = ar.base + ar.used;
  ctx.ws_bytes = ar.cap - ar.used;
  {
    // size class from the data read per pass, log4 steps from 2^20 elements
    const double elems = (double)q.n * (q.dx + (q.problem == SRP_PROBLEM_CCA ? q.dy : 0));
    int c = 0;
    for (double t = double(1 << 20); elems >= t && c < srp_engine::kSizeClasses - 1; t *= 4.0) ++c;
    ctx.group[0] = e->groups[0][c];
    ctx.group[1] = e->groups[1][c];
  }
  if (q.problem == SRP_PROBLEM_CCA)
    return cca_solve_impl(q.X, q.Y, q.n, q.dx, q.dy, q.k, q.lambda_x, q.lambda_y, q.sketch_size, q.tol, q.dtype,
                          &opt, st, q.U, q.V, q.sigma, &r.info, &ctx);
  return lda_solve_impl(q.X, (const int32_t*)q.Y, q.n, q.dx, q.dy, q.k, q.lambda_x, q.sketch_size, q.tol, q.dtype,
                        &opt, st, q.U, q.sigma, &r.info, &ctx);
}

void worker(srp_engine* e, int slot) {
  (void)hipSetDevice(e->device);
  hipStream_t st = e->streams[slot];
  std::unique_lock<std::mutex> lk(e->mu);
  for (;;) {
    Job job;
    size_t off = 0;
    bool got = false;
    for (;;) {
      if (!e->queue.empty() && e->pool.alloc(e->queue.front().footprint, &off)) {
        job = e->queue.front();
        e->queue.pop_front();
        got = true;
        break;
      }
      if (e->queue.empty() && e->stop) break;
      e->cv_work.wait(lk);
    }
    if (!got) return;
    ++e->running;
    e->peak_running = std::max(e->peak_running, e->running);
    srp_result r;
    memset(&r, 0, sizeof(r));
    r.slot = slot;
    r.t_submit_ms = job.t_submit;
    r.t_start_ms = e->now_ms();
    r.footprint_bytes = job.footprint;
    lk.unlock();
    clear_error();
    int rc = run_job(e, job, e->pool_mem + off, st, r);
    // outputs are complete once the stream drains (the solve synchronises
    // it on success; an early error return may leave work queued)
    (void)hipStreamSynchronize(st);
    r.status = rc;
    r.info.status = rc;
    if (rc != SRP_OK) snprintf(r.message, sizeof(r.message), "%s", last_error());
    r.t_done_ms = e->now_ms();
    lk.lock();
    e->pool.release(off, job.footprint);
    --e->running;
    e->in_flight.erase(job.ticket);
    e->done[job.ticket] = r;
    e->cv_done.notify_all();
    e->cv_work.notify_all();
  }
}

int take_result(srp_engine* e, uint64_t ticket, srp_result* out) {
  auto it = e->done.find(ticket);
  const int rc = it->second.status;
  if (out) *out = it->second;
  e->done.erase(it);
  return rc;
}

}  // namespace

extern "C" {

size_t srp_request_footprint(const srp_request* req) { return req ? footprint(*req) : 0; }

int srp_engine_create(int device, size_t hbm_budget_bytes, int max_slots, srp_engine** out) {
  return srp_engine_create2(device, hbm_budget_bytes, max_slots, 0, out);
}

int srp_engine_create2(int device, size_t hbm_budget_bytes, int max_slots, int flags, srp_engine** out) {
  clear_error();
  SRP_REQUIRE(out, "null pointer argument");
  *out = nullptr;
  SRP_REQUIRE(max_slots >= 1 && max_slots <= kMaxSlots, "max_slots must be in [1, %d]", kMaxSlots);
  SRP_REQUIRE((flags & ~SRP_ENGINE_GROUPED) == 0, "unknown engine flags %d", flags);
  SRP_REQUIRE(hbm_budget_bytes >= kAlign, "hbm_budget_bytes too small");
  int prev = 0;
  SRP_HIP(hipGetDevice(&prev));
  SRP_HIP(hipSetDevice(device));
  auto* e = new srp_engine();
  e->device = device;
  e->t0 = std::chrono::steady_clock::now();
  hipError_t he = hipMalloc((void**)&e->pool_mem, align_up(hbm_budget_bytes));
  if (he != hipSuccess) {
    set_error("engine pool of %zu bytes: %s", hbm_budget_bytes, hipGetErrorString(he));
    delete e;
    (void)hipSetDevice(prev);
    return he == hipErrorOutOfMemory ? SRP_ENOMEM : SRP_EDEVICE;
  }
  e->pool.reset(align_up(hbm_budget_bytes) & ~(kAlign - 1));
  e->streams.assign(max_slots, nullptr);
  for (int i = 0; i < max_slots; ++i) {
    he = hipStreamCreateWithFlags(&e->streams[i], hipStreamNonBlocking);
    if (he != hipSuccess) {
      set_error("engine stream: %s", hipGetErrorString(he));
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(e->streams[j]);
      (void)hipFree(e->pool_mem);
      delete e;
      (void)hipSetDevice(prev);
      return SRP_EDEVICE;
    }
  }
  if (flags & SRP_ENGINE_GROUPED) {
    for (int g = 0; g < 2 * srp_engine::kSizeClasses; ++g) {
      int rc = SRP_OK;
      TickGroup*& slot = e->groups[g / srp_engine::kSizeClasses][g % srp_engine::kSizeClasses];
      slot = tick_group_create(g < srp_engine::kSizeClasses ? 16 : 32, &rc);
      if (!slot) {
        for (auto& row : e->groups)
          for (auto& t : row) {
            tick_group_destroy(t);
            t = nullptr;
          }
        for (auto st : e->streams) (void)hipStreamDestroy(st);
        (void)hipFree(e->pool_mem);
        delete e;
        (void)hipSetDevice(prev);
        return rc;
      }
    }
  }
  for (int i = 0; i < max_slots; ++i) e->workers.emplace_back(worker, e, i);
  (void)hipSetDevice(prev);
  *out = e;
  return SRP_OK;
}

int srp_engine_submit(srp_engine* e, const srp_request* req, uint64_t* ticket) {
  clear_error();
  SRP_REQUIRE(e && req && ticket, "null pointer argument");
  SRP_REQUIRE(req->X && req->Y && req->U && req->sigma && (req->problem == SRP_PROBLEM_LDA || req->V),
              "null pointer argument");
  const size_t fp = footprint(*req);
  SRP_REQUIRE(fp > 0, "invalid request sizes");
  std::lock_guard<std::mutex> lk(e->mu);
  if (e->stop) {
    set_error("engine is shutting down");
    return SRP_EBUSY;
  }
  if (align_up(fp) > e->pool.cap()) {
    set_error("request needs %zu bytes; the engine pool holds %zu", fp, e->pool.cap());
    return SRP_EREJECTED;
  }
  Job j;
  j.ticket = e->next_ticket++;
  j.req = *req;
  j.footprint = fp;
  j.t_submit = e->now_ms();
  e->queue.push_back(j);
  e->in_flight.insert(j.ticket);
  *ticket = j.ticket;
  e->cv_work.notify_all();
  return SRP_OK;
}

int srp_engine_poll(srp_engine* e, uint64_t ticket, srp_result* out) {
  clear_error();
  SRP_REQUIRE(e, "null pointer argument");
  std::lock_guard<std::mutex> lk(e->mu);
  if (e->done.count(ticket)) return take_result(e, ticket, out);
  if (e->in_flight.count(ticket)) return SRP_PENDING;
  set_error("unknown ticket %llu", (unsigned long long)ticket);
  return SRP_EINVAL;
}

int srp_engine_wait(srp_engine* e, uint64_t ticket, srp_result* out) {
  clear_error();
  SRP_REQUIRE(e, "null pointer argument");
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv_done.wait(lk, [&] { return e->done.count(ticket) || !e->in_flight.count(ticket); });
  if (e->done.count(ticket)) return take_result(e, ticket, out);
  set_error("unknown ticket %llu", (unsigned long long)ticket);
  return SRP_EINVAL;
}

int srp_engine_stats(srp_engine* e, int* queued, int* running, int* peak_running, size_t* pool_used,
                     size_t* pool_peak) {
  clear_error();
  SRP_REQUIRE(e, "null pointer argument");
  std::lock_guard<std::mutex> lk(e->mu);
  if (queued) *queued = (int)e->queue.size();
  if (running) *running = e->running;
  if (peak_running) *peak_running = e->peak_running;
  if (pool_used) *pool_used = e->pool.used();
  if (pool_peak) *pool_peak = e->pool.peak();
  return SRP_OK;
}

int srp_engine_ticks(srp_engine* e, uint64_t* ticks) {
  clear_error();
  SRP_REQUIRE(e && ticks, "null pointer argument");
  uint64_t t = 0;
  for (auto& row : e->groups)
    for (auto g : row) t += tick_group_ticks(g);
  *ticks = t;
  return SRP_OK;
}

int srp_engine_destroy(srp_engine* e) {
  clear_error();
  if (!e) return SRP_OK;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->stop = true;
    e->cv_work.notify_all();
  }
  for (auto& t : e->workers) t.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(e->device);
  for (auto& row : e->groups)
    for (auto g : row) tick_group_destroy(g);
  for (auto s : e->streams) (void)hipStreamDestroy(s);
  (void)hipFree(e->pool_mem);
  (void)hipSetDevice(prev);
  delete e;
  return SRP_OK;
}

}  // extern "C"
