// Serving runtime: a FIFO of independent least-squares requests drained by worker slots
// (continuous batching).
//
// Each slot is a host thread with its own fs_context (own HIP stream, grow-only workspace), so the
// passes over A of different requests overlap on the GPU (a request with small n does not fill the
// GPU on its own).  The cooperative QR/SVD kernels of different slots run concurrently when their
// grids fit on the GPU together: each reserves its work-groups from a device-wide budget of num_cu
// (CoopBudget), so two grids never hold parts of the GPU while waiting for each other.
//
// Admission is against one device-wide ledger of workspace bytes (hbm_budget).  The ledger charges
// every slot for the workspace it holds (kept between requests, so a slot that serves the same shape
// again allocates nothing) plus, while it runs a request, the growth that request may still need
// (its footprint minus what the slot holds).  A free slot takes the head of the queue once that
// growth fits; otherwise it first gives its own workspace back, then waits, and every idle slot
// gives its workspace back while the head waits.  A request larger than the whole budget is refused
// at submission (FS_ERR_TOO_LARGE); any other is admitted as memory frees up, in arrival order.
#include <math.h>

#include <algorithm>
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
  size_t footprint = 0;
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream: the inputs are ready after it
  int state = 0;               // 0 queued, 1 running, 2 done
  fs_status result = FS_OK;
  fs_info info{};
  double t_submit = -1, t_start = -1, t_finish = -1;
};

}  // namespace

struct fs_server_s {
  int device = 0;
  int num_cu = 0;
  size_t budget = 0;  // workspace bytes of all slots together
  size_t used = 0;    // charged: every slot's resident workspace + running requests' remaining growth
  size_t peak = 0;
  std::vector<size_t> resident;  // per slot: workspace bytes held
  bool pressure = false;         // the queue head waits for memory
  std::vector<fs_context> slots;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex mu;                 // queue, tickets and ledger
  std::condition_variable cv;    // work or memory available / shutdown / pressure
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

  // frees slot s's workspace (its stream is idle) and takes it off the ledger; mu is released meanwhile
  void give_back(int s, std::unique_lock<std::mutex>& lk) {
    lk.unlock();
    (void)fs_context_trim(slots[s]);
    size_t left = 0;
    (void)fs_context_workspace(slots[s], &left);
    lk.lock();
    used -= resident[s] - left;
    resident[s] = left;
    cv.notify_all();
  }

  void worker(int slot) {
    fs_context ctx = slots[slot];
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      if (queue.empty()) {
        if (shutdown) return;
        if (pressure && resident[slot] > 0) {
          give_back(slot, lk);
          continue;
        }
        cv.wait(lk);
        continue;
      }
      const uint64_t id = queue.front();
      Ticket& head = tickets[id];
      const size_t grow = head.footprint > resident[slot] ? head.footprint - resident[slot] : 0;
      if (used + grow > budget) {
        if (resident[slot] > 0) {  // this slot's cache may be what is missing
          give_back(slot, lk);
          continue;
        }
        pressure = true;
        cv.notify_all();  // idle slots give their workspace back
        cv.wait(lk);
        continue;
      }
      queue.pop_front();
      pressure = false;
      used += grow;
      peak = std::max(peak, used);
      head.state = 1;
      head.t_start = now();
      const fs_request req = head.req;
      const fs_options opts = head.opts;
      const hipEvent_t ready = head.ready;
      head.ready = nullptr;
      const size_t held = resident[slot];
      lk.unlock();
      cv.notify_all();  // the next request may fit as well

      fs_info info{};
      fs_status r = FS_OK;
      if (ready) {
        // the caller's work on its stream before the submission (filling A, b) precedes the solve
        if (hipStreamWaitEvent(streams[slot], ready, 0) != hipSuccess) r = FS_ERR_DEVICE;
        (void)hipEventDestroy(ready);
      }
      if (r == FS_OK) {
        r = (req.method == FS_METHOD_SPIR)
                ? spir_solve(ctx, req.m, req.n, req.A, req.lda, req.b, req.x, &opts, &info)
                : (req.method == FS_METHOD_SPIR_LSQR)
                      ? spir_lsqr_solve(ctx, req.m, req.n, req.A, req.lda, req.b, req.x, &opts, &info)
                      : fossils_solve(ctx, req.m, req.n, req.A, req.lda, req.b, req.x, &opts, &info);
      }
      size_t now_held = 0;
      (void)fs_context_workspace(ctx, &now_held);

      lk.lock();
      // the reservation becomes the slot's actual workspace (at most held + grow: the footprint
      // bounds every buffer a solve sizes)
      used = used - grow - held + now_held;
      resident[slot] = now_held;
      Ticket& t = tickets[id];
      t.result = r;
      t.info = info;
      t.state = 2;
      t.t_finish = now();
      done_cv.notify_all();
      cv.notify_all();
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
  srv->num_cu = ctx->num_cu;
  srv->budget = hbm_budget;
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
  srv->resident.assign(max_slots, 0);
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
  for (auto& kv : srv->tickets)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
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
  const size_t need = fs_solve_footprint_cu(req->m, req->n, o, srv->num_cu);
  if (need > srv->budget) return FS_ERR_TOO_LARGE;
  Ticket t;
  t.req = *req;
  t.req.opts = nullptr;
  t.opts = o;
  t.footprint = need;
  FS_HIP(hipSetDevice(srv->device));
  FS_HIP(hipEventCreateWithFlags(&t.ready, hipEventDisableTiming));
  const hipError_t e = hipEventRecord(t.ready, (hipStream_t)req->stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(t.ready);
    fs_set_last_hip_error(e, "hipEventRecord on the submitter's stream", __FILE__, __LINE__);
    return FS_ERR_DEVICE;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->shutdown) {
      (void)hipEventDestroy(t.ready);
      return FS_ERR_INVALID_ARG;
    }
    t.t_submit = srv->now();
    const uint64_t id = srv->next_ticket++;
    srv->tickets.emplace(id, t);
    srv->queue.push_back(id);
    *ticket = id;
  }
  srv->cv.notify_all();
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
  const Ticket& t = it->second;  // (element references survive rehashing by later submissions)
  srv->done_cv.wait(lk, [&] { return t.state == 2; });
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

fs_status fs_server_memory(fs_server srv, size_t* used, size_t* peak, size_t* budget) {
  if (!srv) return FS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (used) *used = srv->used;
  if (peak) *peak = srv->peak;
  if (budget) *budget = srv->budget;
  return FS_OK;
}

fs_status fs_server_request_footprint(fs_server srv, int64_t m, int32_t n, const fs_options* opts, size_t* bytes) {
  if (!srv || !bytes) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < n) return FS_ERR_SHAPE;
  fs_options o;
  if (opts) o = *opts;
  else FS_TRY(fs_options_default(m, n, &o));
  if (srv->slots.size() > 1) o.overlap_svd = 0;
  *bytes = fs_solve_footprint_cu(m, n, o, srv->num_cu);
  return FS_OK;
}

}  // extern "C"
