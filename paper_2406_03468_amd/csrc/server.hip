// Serving runtime: a FIFO of independent least-squares requests drained by worker slots.
//
// Each slot is a host thread with its own fs_context (own HIP stream, grow-only workspace), so the
// passes over A of different requests overlap on the GPU (a request with small n does not fill the
// GPU on its own).  The cooperative QR/SVD kernels of different slots run concurrently when their
// grids fit on the GPU together: each reserves its work-groups from a device-wide budget of num_cu
// (CoopBudget), so two grids never hold parts of the GPU while waiting for each other.  Admission is
// by workspace footprint: each slot owns hbm_budget / max_slots bytes and a request needing more is
// refused at submission.
#include <math.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "context.hpp"

namespace {

struct Ticket {
  fs_request req{};
  fs_options opts{};
  bool has_opts = false;
  int state = 0;  // 0 queued, 1 running, 2 done
  fs_status result = FS_OK;
  fs_info info{};
  double t_submit = -1, t_start = -1, t_finish = -1;
};

}  // namespace

struct fs_server_s {
  int device = 0;
  size_t slot_budget = 0;
  std::vector<fs_context> slots;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex mu;                 // queue + tickets
  std::condition_variable cv;    // work available / shutdown
  std::condition_variable done_cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  bool shutdown = false;
  CoopBudget coop;               // work-groups of cooperative grids, device-wide
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void worker(int slot) {
    fs_context ctx = slots[slot];
    (void)hipSetDevice(device);
    for (;;) {
      uint64_t id = 0;
      fs_request req;
      fs_options opts;
      bool has_opts = false;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return shutdown || !queue.empty(); });
        if (queue.empty()) return;  // shutdown with nothing left
        id = queue.front();
        queue.pop_front();
        Ticket& t = tickets[id];
        t.state = 1;
        t.t_start = now();
        req = t.req;
        opts = t.opts;
        has_opts = t.has_opts;
      }
      fs_info info{};
      const fs_options* op = has_opts ? &opts : nullptr;
      fs_status r = (req.method == FS_METHOD_SPIR)
                        ? spir_solve(ctx, req.m, req.n, req.A, req.lda, req.b, req.x, op, &info)
                        : (req.method == FS_METHOD_SPIR_LSQR)
                              ? spir_lsqr_solve(ctx, req.m, req.n, req.A, req.lda, req.b, req.x, op, &info)
                              : fossils_solve(ctx, req.m, req.n, req.A, req.lda, req.b, req.x, op, &info);
      {
        std::lock_guard<std::mutex> lk(mu);
        Ticket& t = tickets[id];
        t.result = r;
        t.info = info;
        t.state = 2;
        t.t_finish = now();
      }
      done_cv.notify_all();
    }
  }
};

extern "C" {

fs_status fs_server_create(fs_context ctx, size_t hbm_budget, int32_t max_slots, fs_server* out) {
  if (!ctx || !out) return FS_ERR_INVALID_ARG;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 16 || hbm_budget == 0) return FS_ERR_INVALID_ARG;
  FS_HIP(hipSetDevice(ctx->device));
  fs_server srv = new fs_server_s();
  srv->device = ctx->device;
  srv->slot_budget = hbm_budget / (size_t)max_slots;
  srv->coop.total = srv->coop.avail = ctx->num_cu;
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);  // default priority
    fs_context c = nullptr;
    fs_status s = (e == hipSuccess) ? fs_context_create(ctx->device, st, &c) : FS_ERR_DEVICE;
    if (s != FS_OK) {
      if (e == hipSuccess) (void)hipStreamDestroy(st);
      for (size_t j = 0; j < srv->slots.size(); ++j) {
        fs_context_destroy(srv->slots[j]);
        (void)hipStreamDestroy(srv->streams[j]);
      }
      delete srv;
      return s;
    }
    c->coop_budget = &srv->coop;
    srv->slots.push_back(c);
    srv->streams.push_back(st);
  }
  for (int i = 0; i < max_slots; ++i) srv->workers.emplace_back([srv, i] { srv->worker(i); });
  *out = srv;
  return FS_OK;
}

fs_status fs_server_destroy(fs_server srv) {
  if (!srv) return FS_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->shutdown = true;
  }
  srv->cv.notify_all();
  for (auto& w : srv->workers) w.join();
  for (size_t j = 0; j < srv->slots.size(); ++j) {
    fs_context_destroy(srv->slots[j]);
    (void)hipStreamDestroy(srv->streams[j]);
  }
  delete srv;
  return FS_OK;
}

fs_status batched_submit(fs_server srv, const fs_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) return FS_ERR_INVALID_ARG;
  if (req->method != FS_METHOD_FOSSILS && req->method != FS_METHOD_SPIR && req->method != FS_METHOD_SPIR_LSQR)
    return FS_ERR_INVALID_ARG;
  FS_TRY(fs_validate_problem(req->m, req->n, req->A, req->lda, req->b, req->x));
  fs_options o;
  if (req->opts) o = *req->opts;
  else FS_TRY(fs_options_default(req->m, req->n, &o));
  FS_TRY(fs_validate_options(req->m, req->n, o));
  // With several slots the GPU is already shared between solves: the SVD beside the first step
  // only adds contention there (C5 stream, 8 slots: 251 solves/s in the serial order, 233 with it).
  if (srv->slots.size() > 1) o.overlap_svd = 0;
  if (fs_solve_footprint(req->m, req->n, &o) > srv->slot_budget) return FS_ERR_TOO_LARGE;
  Ticket t;
  t.req = *req;
  t.req.opts = nullptr;
  t.opts = o;
  t.has_opts = true;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->shutdown) return FS_ERR_INVALID_ARG;
    t.t_submit = srv->now();
    const uint64_t id = srv->next_ticket++;
    srv->tickets.emplace(id, t);
    srv->queue.push_back(id);
    *ticket = id;
  }
  srv->cv.notify_one();
  return FS_OK;
}

fs_status batched_poll(fs_server srv, uint64_t ticket, int32_t* done, fs_status* result, fs_info* info) {
  if (!srv || !done) return FS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return FS_ERR_UNKNOWN_TICKET;
  *done = (it->second.state == 2) ? 1 : 0;
  if (*done) {
    if (result) *result = it->second.result;
    if (info) *info = it->second.info;
  }
  return FS_OK;
}

fs_status fs_server_wait(fs_server srv, uint64_t ticket) {
  if (!srv) return FS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return FS_ERR_UNKNOWN_TICKET;
  srv->done_cv.wait(lk, [&] { return srv->tickets[ticket].state == 2; });
  return FS_OK;
}

fs_status fs_server_ticket_times(fs_server srv, uint64_t ticket, double* submit_s, double* start_s, double* finish_s) {
  if (!srv) return FS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return FS_ERR_UNKNOWN_TICKET;
  if (submit_s) *submit_s = it->second.t_submit;
  if (start_s) *start_s = it->second.t_start;
  if (finish_s) *finish_s = it->second.t_finish;
  return FS_OK;
}

}  // extern "C"
