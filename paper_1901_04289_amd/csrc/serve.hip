// Request loop: jobs (dot products and matrix products over device-resident
// operands) are validated and admitted by their workspace footprint against
// an HBM budget, queued, and run by worker slots.  Each slot owns a HIP
// stream and a workspace of its own, so requests on different slots
// overlap on the device; a slot that finds several dot jobs at the head of
// the queue runs them together as one persistent batch launch.  Tickets
// carry submit, start and completion times for latency reporting.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

using namespace arbgpu_impl;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr size_t kDotFootprint = 1 << 16;   // staging of one dot task list entry
constexpr int kMaxDotGroup = 4096;          // dot jobs taken together by one slot
constexpr size_t kKeepTickets = 1 << 20;    // completed tickets remembered

}  // namespace

namespace arbgpu_impl {

struct Server {
  arbgpu_ctx *owner = nullptr;
  int nslots = 0;
  size_t budget = 0, reserved = 0;
  std::vector<arbgpu_ctx *> slot_ctx;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  struct Item {
    uint64_t ticket;
    arbgpu_job job;
    size_t footprint;
  };
  std::deque<Item> queue;
  struct Ticket {
    int state = 0;   // 0 queued, 1 running, 2 done
    int rc = ARBGPU_OK;
    std::string err;
    int64_t t_submit = 0, t_start = 0, t_end = 0;
  };
  std::unordered_map<uint64_t, Ticket> tickets;
  std::deque<uint64_t> done_order;
  uint64_t next_ticket = 1;
  bool stop = false;

  void worker(int k) {
    arbgpu_ctx *c = slot_ctx[k];
    hipStream_t s = streams[k];
    (void)hipSetDevice(c->device);
    for (;;) {
      std::vector<Item> take;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        if (queue.empty()) return;   // stop requested and nothing left
        take.push_back(queue.front());
        queue.pop_front();
        if (take[0].job.kind == ARBGPU_JOB_DOT)
          while (!queue.empty() && queue.front().job.kind == ARBGPU_JOB_DOT && (int)take.size() < kMaxDotGroup) {
            take.push_back(queue.front());
            queue.pop_front();
          }
        const int64_t t = now_ns();
        for (auto &it : take) {
          Ticket &tk = tickets[it.ticket];
          tk.state = 1;
          tk.t_start = t;
        }
      }
      int rc;
      if (take[0].job.kind == ARBGPU_JOB_DOT) {
        std::vector<arbgpu_dot_job> dots;
        for (auto &it : take) dots.push_back(it.job.dot);
        std::lock_guard<std::mutex> lk(c->mu);
        ctx_use_stream(c, s);
        rc = dot_batch_run(c, dots.data(), (int64_t)dots.size(), s);
      } else {
        const arbgpu_job &j = take[0].job;
        rc = arbgpu_mat_mul(c, &j.C, &j.A, &j.B, j.p, j.flags, s);
        if (rc == ARBGPU_OK) {
          hipError_t e = hipStreamSynchronize(s);
          if (e != hipSuccess) rc = set_error(c, ARBGPU_EDEVICE, "request: %s", hipGetErrorString(e));
        }
      }
      // the slot keeps its workspace (at most its share of the budget) for
      // the next request
      std::string err = rc ? c->err : std::string();
      {
        std::lock_guard<std::mutex> lk(mu);
        const int64_t t = now_ns();
        for (auto &it : take) {
          Ticket &tk = tickets[it.ticket];
          tk.state = 2;
          tk.rc = rc;
          tk.err = err;
          tk.t_end = t;
          reserved -= it.footprint;
          done_order.push_back(it.ticket);
        }
        while (done_order.size() > kKeepTickets) {
          tickets.erase(done_order.front());
          done_order.pop_front();
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }

  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_work.notify_all();
    for (auto &t : threads)
      if (t.joinable()) t.join();
    for (auto s : streams) (void)hipStreamDestroy(s);
    for (auto c : slot_ctx) arbgpu_destroy(c);
  }
};

void server_delete(Server *s) { delete s; }

}  // namespace arbgpu_impl

namespace {

int start_server(arbgpu_ctx *ctx, int slots, size_t budget) {
  if (ctx->device < 0) return set_error(ctx, ARBGPU_EDEVICE, "host-only context cannot launch work");
  Server *sv = new (std::nothrow) Server;
  if (!sv) return ARBGPU_ENOMEM;
  sv->owner = ctx;
  sv->nslots = slots;
  sv->budget = budget;
  hipError_t e = hipSetDevice(ctx->device);
  // every slot holds at most its share of the budget as workspace
  for (int k = 0; k < slots && e == hipSuccess; ++k) {
    arbgpu_ctx *c = nullptr;
    if (arbgpu_init(&c, ctx->device, budget / (size_t)slots, nullptr) != ARBGPU_OK) {
      e = hipErrorOutOfMemory;
      break;
    }
    c->tune = ctx->tune;
    sv->slot_ctx.push_back(c);
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) sv->streams.push_back(s);
  }
  if (e != hipSuccess) {
    delete sv;
    return set_error(ctx, ARBGPU_EDEVICE, "request loop start: %s", hipGetErrorString(e));
  }
  for (int k = 0; k < slots; ++k) sv->threads.emplace_back([sv, k] { sv->worker(k); });
  ctx->server = sv;
  return ARBGPU_OK;
}

}  // namespace

extern "C" {

int arbgpu_serve_config(arbgpu_ctx *ctx, int slots, size_t budget_bytes) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (slots < 1 || slots > 16) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_serve_config: slots must be 1..16");
  if (ctx->server) {
    std::lock_guard<std::mutex> sl(ctx->server->mu);
    if (!ctx->server->queue.empty() || ctx->server->reserved)
      return set_error(ctx, ARBGPU_EINVAL, "arbgpu_serve_config: requests are in flight");
  }
  if (ctx->server) {
    server_delete(ctx->server);
    ctx->server = nullptr;
  }
  return start_server(ctx, slots, budget_bytes ? budget_bytes : ctx->budget / 2);
}

int arbgpu_submit(arbgpu_ctx *ctx, const arbgpu_job *jobs, int64_t njobs, uint64_t *tickets) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (njobs < 0 || (njobs > 0 && (!jobs || !tickets))) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_submit: bad arguments");
  std::vector<size_t> fp((size_t)njobs);
  size_t need = 0;
  for (int64_t i = 0; i < njobs; ++i) {
    const arbgpu_job &j = jobs[i];
    int rc;
    if (j.kind == ARBGPU_JOB_DOT) {
      DotParams prm[2];
      int nt;
      LimbShape sh;
      rc = dot_tasks(ctx, j.dot, "arbgpu_submit", prm, &nt, &sh);
      fp[i] = kDotFootprint;
    } else if (j.kind == ARBGPU_JOB_MATMUL) {
      rc = mat_mul_check(ctx, &j.C, &j.A, &j.B, j.p, j.flags);
      fp[i] = rc ? 0 : mat_mul_footprint(&j.A, &j.B, j.p, j.flags);
    } else {
      rc = set_error(ctx, ARBGPU_EINVAL, "unknown job kind %d", j.kind);
    }
    if (rc) {
      ctx->err = "job " + std::to_string(i) + ": " + ctx->err;
      return rc;
    }
    need += fp[i];
  }
  if (!ctx->server) {
    const int rc = start_server(ctx, 4, ctx->budget / 2);
    if (rc) return rc;
  }
  Server *sv = ctx->server;
  {
    std::lock_guard<std::mutex> sl(sv->mu);
    const size_t share = sv->budget / (size_t)sv->nslots;
    for (int64_t i = 0; i < njobs; ++i)
      if (fp[i] > share)
        return set_error(ctx, ARBGPU_ENOMEM, "arbgpu_submit: job %lld needs %zu bytes of workspace, a slot holds %zu",
                         (long long)i, fp[i], share);
    if (need > sv->budget)
      return set_error(ctx, ARBGPU_ENOMEM, "arbgpu_submit: %zu bytes of workspace exceed the budget %zu", need,
                       sv->budget);
    if (sv->reserved + need > sv->budget)
      return set_error(ctx, ARBGPU_EAGAIN, "arbgpu_submit: %zu bytes in flight, %zu more do not fit in %zu",
                       sv->reserved, need, sv->budget);
    const int64_t t = now_ns();
    for (int64_t i = 0; i < njobs; ++i) {
      const uint64_t id = sv->next_ticket++;
      Server::Ticket tk;
      tk.t_submit = t;
      sv->tickets[id] = tk;
      sv->queue.push_back(Server::Item{id, jobs[i], fp[i]});
      sv->reserved += fp[i];
      tickets[i] = id;
    }
  }
  sv->cv_work.notify_all();
  return ARBGPU_OK;
}

int arbgpu_serve_reserve(arbgpu_ctx *ctx, const arbgpu_job *jobs, int64_t njobs) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (njobs < 0 || (njobs > 0 && !jobs)) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_serve_reserve: bad arguments");
  size_t sz[WS_COUNT] = {0};
  for (int64_t i = 0; i < njobs; ++i) {
    const arbgpu_job &j = jobs[i];
    size_t js[WS_COUNT] = {0};
    if (j.kind == ARBGPU_JOB_MATMUL) {
      const int rc = mat_mul_check(ctx, &j.C, &j.A, &j.B, j.p, j.flags);
      if (rc) return rc;
      mat_mul_ws_sizes(&j.A, &j.B, j.p, j.flags, js);
    } else if (j.kind == ARBGPU_JOB_DOT) {
      js[WS_BATCH] = dot_batch_ws(2 * (int64_t)kMaxDotGroup);
    } else {
      return set_error(ctx, ARBGPU_EINVAL, "arbgpu_serve_reserve: unknown job kind %d", j.kind);
    }
    for (int k = 0; k < WS_COUNT; ++k) sz[k] = std::max(sz[k], js[k]);
  }
  if (!ctx->server) {
    const int rc = start_server(ctx, 4, ctx->budget / 2);
    if (rc) return rc;
  }
  for (arbgpu_ctx *c : ctx->server->slot_ctx) {
    std::lock_guard<std::mutex> cl(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipSetDevice");
    const int rc = ws_reserve(c, sz);
    if (rc) return set_error(ctx, rc, "arbgpu_serve_reserve: %s", c->err.c_str());
  }
  return ARBGPU_OK;
}

int arbgpu_workspace_info(arbgpu_ctx *ctx, int64_t *allocs, int64_t *bytes) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  int64_t n = 0, held = 0;
  auto add = [&](arbgpu_ctx *c) {
    n += c->allocs;
    for (auto &b : c->ws)
      if (b.owned) held += (int64_t)b.size;
  };
  add(ctx);
  if (ctx->server)
    for (arbgpu_ctx *c : ctx->server->slot_ctx) {
      std::lock_guard<std::mutex> cl(c->mu);
      add(c);
    }
  if (allocs) *allocs = n;
  if (bytes) *bytes = held;
  return ARBGPU_OK;
}

int arbgpu_poll(arbgpu_ctx *ctx, uint64_t ticket, int64_t timeout_us) {
  if (!ctx) return ARBGPU_EINVAL;
  Server *sv;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    sv = ctx->server;
  }
  if (!sv) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_poll: no request was submitted");
  std::unique_lock<std::mutex> sl(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return ARBGPU_EINVAL;
  if (timeout_us > 0)
    sv->cv_done.wait_for(sl, std::chrono::microseconds(timeout_us), [&] {
      auto jt = sv->tickets.find(ticket);
      return jt == sv->tickets.end() || jt->second.state == 2;
    });
  it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return ARBGPU_EINVAL;
  if (it->second.state != 2) return ARBGPU_NOTREADY;
  const int rc = it->second.rc;
  const std::string err = it->second.err;
  sl.unlock();
  if (rc != ARBGPU_OK) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err = err;
  }
  return rc;
}

int arbgpu_ticket_times(arbgpu_ctx *ctx, uint64_t ticket, int64_t times_ns[3]) {
  if (!ctx || !times_ns) return ARBGPU_EINVAL;
  Server *sv;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    sv = ctx->server;
  }
  if (!sv) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> sl(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return ARBGPU_EINVAL;
  times_ns[0] = it->second.t_submit;
  times_ns[1] = it->second.t_start;
  times_ns[2] = it->second.t_end;
  return ARBGPU_OK;
}

}  // extern "C"
