// fossils_solve_batched: FOSSILS (Algorithm 4, P = V Sigma^{-1}) or SPIR (Algorithm 3 with the same
// preconditioner), each problem's choice, for many independent problems of uneven m and n in one call.
//
//   setup      each problem's sketch, QR of the sketch, SVD of R, sketch-and-solve start x_0 and column
//              scaling, in problem order on kSetupSlots helper contexts (own stream and scratch each, host
//              threads), whose cooperative QR / SVD grids reserve work-groups from one budget so that grids
//              running together always fit on the GPU; results go to the problem's slice of the batch
//              workspace;
//   refinement once every setup is done, the two refinement steps of all problems in lockstep on the
//              caller's stream: each phase of an inner iteration is one launch for the whole batch -- the
//              passes over A as one work-list of (problem, row tiles) per tile
//              configuration, the products with V Sigma^{-1} and the heavy-ball / CG and KW steps with one
//              work-group (or a slice of the grid) per problem.  A problem whose rule has stopped it skips
//              the kernels of the following iterations (its stop flag), and the host polls all flags once
//              per kw_every iterations.
// Problems outside the batched envelope -- n above 1024 (narrower tiles than the batched pass is built
// for), a numerically rank-deficient sketch (truncated preconditioner), b = 0 -- are finished by
// fossils_solve / spir_solve on the caller's context with the caller's options.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/fossils.h"
#include "common.hpp"
#include "context.hpp"
#include "internal.hpp"
#include "state.hpp"

namespace {

constexpr int kSetupSlots = 32;
constexpr double U_ROUND = FS_U_ROUND;

struct ProbLayout {
  size_t off_V, off_sigma, off_dinv, off_cn2, off_vec, off_gpart, off_part, off_pr2, off_state;
  size_t bytes;
  int H = 0, L = 0, G = 0;
  bool vec = false;  // 16-byte loads of A and b
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// per-problem slice of the batch workspace
ProbLayout layout(int n, int G, int H, int L) {
  ProbLayout p;
  size_t o = 0;
  const size_t N = (size_t)n;
  auto take = [&](size_t& off, size_t bytes) {
    off = o;
    o += align256(bytes);
  };
  take(p.off_V, 8 * N * N);
  take(p.off_sigma, 8 * N);
  take(p.off_dinv, 8 * N);
  take(p.off_cn2, 8 * (N + 1));
  take(p.off_vec, 8 * 12 * N);
  take(p.off_gpart, 8 * N * ((N + 63) / 64 + 1));
  take(p.off_part, 8 * (size_t)G * N);
  take(p.off_pr2, 8 * ((size_t)G + 64));
  take(p.off_state, sizeof(DevState) + 64);
  p.bytes = o;
  p.H = H;
  p.L = L;
  p.G = G;
  return p;
}

}  // namespace

struct BatchHelpers {
  std::vector<fs_context> ctx;
  std::vector<hipStream_t> streams;
  std::vector<BatchReport*> report;  // pinned host copy of each helper's last setup report
};

namespace {

// Waits for the work enqueued on s so far, sleeping between polls: the setup threads outnumber the host
// cores, and a spinning wait would hold a core that another thread needs to launch its work.
hipError_t sync_sleep(hipStream_t s, hipEvent_t ev) {
  hipError_t e = hipEventRecord(ev, s);
  if (e != hipSuccess) return e;
  // short waits: polls that only yield the core; longer ones: 20 us sleeps between polls
  for (int polls = 0; (e = hipEventQuery(ev)) == hipErrorNotReady; ++polls) {
    if (polls < 64) std::this_thread::yield();
    else std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  return e;
}

// Work-group reservations of the setup's grid-synchronizing kernels (see CoopBudget).
int coop_acquire(CoopBudget& b, int need) {
  need = std::max(1, std::min(need, b.total));
  std::unique_lock<std::mutex> lk(b.mu);
  b.cv.wait(lk, [&] { return b.avail >= need; });
  b.avail -= need;
  return need;
}

void coop_give_back(CoopBudget& b, int n) {
  {
    std::lock_guard<std::mutex> lk(b.mu);
    b.avail += n;
  }
  b.cv.notify_all();
}

}  // namespace

void fs_batch_helpers_destroy(fs_context c) {
  if (!c->batch) return;
  for (size_t i = 0; i < c->batch->ctx.size(); ++i) {
    fs_context_destroy(c->batch->ctx[i]);
    (void)hipStreamDestroy(c->batch->streams[i]);
  }
  for (BatchReport* r : c->batch->report)
    if (r) (void)hipHostFree(r);
  delete c->batch;
  c->batch = nullptr;
}

namespace {

fs_status solve_batched(fs_context ctx, int32_t count, const fs_problem* probs, const fs_options* opts_in,
                        fs_info* infos, fs_status* statuses) {
  if (!ctx || !probs || count < 1 || !statuses) return FS_ERR_INVALID_ARG;
  if (count > 65535) return FS_ERR_TOO_LARGE;
  // ---- validation and per-problem options (every field from opts_in except d = 12 n)
  std::vector<fs_options> opt(count);
  std::vector<int> batched(count, 0);
  for (int i = 0; i < count; ++i) {
    const fs_problem& P = probs[i];
    statuses[i] = fs_validate_problem(P.m, P.n, P.A, P.lda, P.b, P.x);
    if (statuses[i] != FS_OK) continue;
    if (P.method != FS_METHOD_FOSSILS && P.method != FS_METHOD_SPIR) {
      statuses[i] = FS_ERR_UNSUPPORTED;
      continue;
    }
    fs_options o;
    statuses[i] = fs_options_default(P.m, P.n, &o);
    if (statuses[i] != FS_OK) continue;
    if (opts_in) {
      const int32_t d = o.d;
      o = *opts_in;
      o.d = d;
      if (o.zeta > o.d) o.zeta = o.d;
    }
    o.precision = FS_FP64;
    o.precond = FS_PRECOND_SVD;
    o.fixed_q = 0;
    o.steps = 2;
    o.init = FS_INIT_SKETCH;
    o.overlap_svd = 0;
    o.graph_sweeps = 0;
    statuses[i] = fs_validate_options(P.m, P.n, o);
    if (statuses[i] != FS_OK) continue;
    opt[i] = o;
    // (tile heights 64 / 32 / 16 only, and 32-bit lane offsets inside a column slot)
    const PassConfig pc = fs_pass_config(P.m, P.n, 256);
    const int hres = (pc.H == 32 && P.n > 256) ? 16 : pc.H;  // the residual pass's tile height
    const int64_t cpr = hres ? 512 / (hres / 2) : 0;
    batched[i] = (P.n <= 1024 && pc.H >= 16 && (cpr * P.lda + pc.H) * 8 < (int64_t(1) << 32)) ? 1 : 0;
  }
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  hipStream_t s = ctx->stream;
  if (infos) memset(infos, 0, sizeof(fs_info) * (size_t)count);

  // ---- work-group slices of the batched passes.  The problems are grouped by pass instantiation (tile
  // height H, column slots L, load width); each group's passes are one launch, and the groups' launches
  // follow each other, so each group's grid is sized to fill the GPU (about two work-groups per CU, the
  // pass holding a CU's registers), shared out in proportion to each problem's m n in multiples of 8
  std::vector<int> idx;  // batched problems
  for (int i = 0; i < count; ++i)
    if (batched[i]) idx.push_back(i);
  const int nb = (int)idx.size();
  std::vector<ProbLayout> lay(count);
  std::vector<PassConfig> pcs(count);
  std::vector<int> keyv(count, 0);
  std::map<int, double> group_work;
  for (int i : idx) {
    pcs[i] = fs_pass_config(probs[i].m, probs[i].n, ctx->num_cu);
    const int cpr = 512 / (pcs[i].H / 2);
    const int L = (probs[i].n + cpr - 1) / cpr;
    const bool vec = ((probs[i].lda & 1) == 0) && ((reinterpret_cast<uintptr_t>(probs[i].A) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(probs[i].b) & 15) == 0);
    keyv[i] = (pcs[i].H * 64 + L) * 2 + (vec ? 1 : 0);
    group_work[keyv[i]] += (double)probs[i].m * probs[i].n;
  }
  size_t total = 0;
  for (int i : idx) {
    const int key = keyv[i];
    const double share = 2.0 * ctx->num_cu * ((double)probs[i].m * probs[i].n) / std::max(group_work[key], 1.0);
    int G = (int)std::min<double>(pcs[i].G, std::max(8.0, ceil(share / 8.0) * 8.0));
    G = std::max(8, G / 8 * 8);
    lay[i] = layout(probs[i].n, G, pcs[i].H, (key / 2) % 64);
    lay[i].vec = (key & 1) != 0;
    total += lay[i].bytes;
  }
  // descriptors: the problems' vectors, three pass work-lists (normal, residual, step heads) and the
  // gathered states
  const size_t nb1 = (size_t)std::max(nb, 1);
  const size_t vec_desc = align256(sizeof(BatchVec) * nb1), pass_desc = align256(sizeof(BatchPass) * nb1);
  const size_t desc_bytes = vec_desc + 3 * pass_desc + align256(sizeof(DevState) * nb1);
  FS_TRY(fs_grow(ctx->ws.batch, total + desc_bytes + 256));
  unsigned char* base = (unsigned char*)ctx->ws.batch.p;
  std::vector<size_t> start(count, 0);
  {
    size_t o = 0;
    for (int i : idx) {
      start[i] = o;
      o += lay[i].bytes;
    }
  }
  auto ptr = [&](int i, size_t off) { return (double*)(base + start[i] + off); };
  auto state_of = [&](int i) { return (DevState*)(base + start[i] + lay[i].off_state); };

  // ---- setup on the helper contexts (host threads), in problem order; the main thread refines a wave of
  // problems once all of its setups are complete
  if (!ctx->batch) {
    // all helpers or none: a partial set is torn down again
    ctx->batch = new BatchHelpers();
    fs_status r = FS_OK;
    for (int k = 0; k < kSetupSlots && r == FS_OK; ++k) {
      hipStream_t st = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e != hipSuccess) {
        fs_set_last_hip_error(e, "hipStreamCreateWithFlags", __FILE__, __LINE__);
        r = FS_ERR_DEVICE;
        break;
      }
      fs_context c = nullptr;
      r = fs_context_create(ctx->device, st, &c);
      if (r != FS_OK) {
        (void)hipStreamDestroy(st);
        break;
      }
      ctx->batch->ctx.push_back(c);
      ctx->batch->streams.push_back(st);
      BatchReport* rep = nullptr;
      e = hipHostMalloc((void**)&rep, sizeof(BatchReport), hipHostMallocDefault);
      ctx->batch->report.push_back(e == hipSuccess ? rep : nullptr);
      if (e != hipSuccess) {
        fs_set_last_hip_error(e, "hipHostMalloc", __FILE__, __LINE__);
        r = FS_ERR_NOMEM;
      }
    }
    if (r != FS_OK) {
      fs_batch_helpers_destroy(ctx);
      return r;
    }
  }
  CoopBudget budget;
  budget.total = budget.avail = ctx->num_cu;
  std::vector<int> fallback(count, 0);  // finished by fossils_solve below
  std::vector<DevState> hst(count);
  std::vector<double> setup_ms(count, 0.0);
  std::vector<int> sweeps(count, 0);
  std::mutex mu;
  std::condition_variable cv;
  std::vector<char> ready(count, 0);
  std::atomic<bool> quit{false};
  auto setup_one = [&](fs_context h, BatchReport* rep, int i) {
    Workspace& W = h->ws;
    hipStream_t hs = h->stream;
    const fs_problem& P = probs[i];
    const fs_options& o = opt[i];
    const int n = P.n, d = o.d, kk = n + 1;
    const bool i16 = fs_idx16_ok(d);
    auto fail = [&](fs_status st) { statuses[i] = st; };
    if (fs_grow(W.idx, (size_t)P.m * o.zeta * (i16 ? 2 : 4)) != FS_OK || fs_grow(W.Y, 8 * (size_t)d * kk) != FS_OK ||
        fs_grow(W.qrwork, fs_qr_work_bytes(d, kk, h->num_cu)) != FS_OK ||
        fs_grow(W.svdwork, fs_svd_work_bytes(n)) != FS_OK || fs_grow(W.trsv, fs_trsv_flow_bytes(n)) != FS_OK ||
        fs_grow(W.state, sizeof(BatchReport)) != FS_OK) {
      fail(FS_ERR_NOMEM);
      return;
    }
    DevState* st = state_of(i);
    double* V = ptr(i, lay[i].off_V);
    double* sigma = ptr(i, lay[i].off_sigma);
    double* dinv = ptr(i, lay[i].off_dinv);
    double* cn2 = ptr(i, lay[i].off_cn2);
    double* vec = ptr(i, lay[i].off_vec);  // x, x0, ...
    double* Y = (double*)W.Y.p;
    const double eta = ((o.eta > 0) ? o.eta : sqrt((double)n / d)) * o.eta_factor;
    const double beta0 = eta * eta;  // eq:optimal-coeffs
    hipEvent_t e0 = h->ev[0], e1 = h->ev[1];
    hipError_t e = hipEventRecord(e0, hs);
    if (e == hipSuccess) e = fs_vec_state_init(st, (1.0 - beta0) * (1.0 - beta0), beta0, o.max_inner, hs);
    if (e == hipSuccess) e = fs_trsv_flow_reset(n, W.trsv.p, hs);
    // sketch of [A b] with the column norms (Alg 4, first statement), QR of the sketch, SVD of R
    if (e == hipSuccess) e = fs_launch_sketch_indices(P.m, d, o.zeta, o.seed, 0, P.m, W.idx.p, i16, hs);
    if (e == hipSuccess)
      e = fs_launch_sketch_apply(P.A, P.lda, P.m, n, P.b, P.m, 1, W.idx.p, i16, d, o.zeta, Y, d, cn2,
                                 o.column_scaling != 0, true, h->lds_bytes, hs);
    if (e == hipSuccess) e = fs_vec_scaling(n, cn2, o.column_scaling != 0, dinv, st, hs);
    int* sw = (int*)((char*)st + sizeof(DevState));
    // grid-synchronizing kernels: work-groups reserved against the other setup streams, the QR's and the
    // (smaller, longer-running) SVD's one after the other, each held until its kernel has completed
    auto reserved = [&](int need, auto&& launch) -> hipError_t {
      const int q = coop_acquire(budget, need);
      hipError_t el = launch();
      hipError_t es = sync_sleep(hs, h->ev[2]);
      if (es != hipSuccess) (void)hipStreamSynchronize(hs);
      coop_give_back(budget, q);
      return el != hipSuccess ? el : es;
    };
    if (e == hipSuccess)
      e = reserved(fs_qr_grid_size(d, h->num_cu), [&] { return fs_launch_qr(Y, d, d, kk, W.qrwork.p, h->num_cu, hs); });
    if (e == hipSuccess)
      e = reserved(fs_svd_grid_size(n, h->num_cu, false), [&] {
        hipError_t es = fs_launch_svd_full(Y, d, n, sigma, V, n, nullptr, n, W.svdwork.p, h->num_cu, o.max_sweeps, sw,
                                           hs);
        return es == hipSuccess ? fs_vec_sigma_stats(n, sigma, o.tau_factor, st, hs) : es;
      });
    // x_0 = R^{-1} t (eq:sketch-and-solve-2.3), kept as x and x0; theta^2 and ||b||^2
    if (e == hipSuccess)
      e = fs_launch_trsv_flow(Y, d, n, false, Y + (int64_t)n * d, vec, nullptr, nullptr, nullptr, W.trsv.p, hs);
    if (e == hipSuccess) e = fs_vec_mul(n, vec, nullptr, vec + n, nullptr, hs);
    if (e == hipSuccess) e = fs_b_prep(cn2, n, st, hs);
    // one read-back (pinned): the state, the barrier and flag words, the NaN / overflow marks
    BatchReport* rep_dev = (BatchReport*)W.state.p;
    if (e == hipSuccess)
      e = fs_b_report(st, sw, fs_qr_err_word(W.qrwork.p, d, kk, h->num_cu), fs_svd_err_word(W.svdwork.p, n),
                      fs_trsv_flow_err_word(n, W.trsv.p), cn2, n, rep_dev, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(rep, rep_dev, sizeof(BatchReport), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipEventRecord(e1, hs);
    if (e == hipSuccess) e = sync_sleep(hs, h->ev[2]);
    if (e != hipSuccess) (void)hipStreamSynchronize(hs);  // (the workspace is reused by the next problem)
    if (e != hipSuccess) {
      fs_set_last_hip_error(e, "batched setup", __FILE__, __LINE__);
      fail(FS_ERR_DEVICE);
      return;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    setup_ms[i] = ms;
    hst[i] = rep->st;
    sweeps[i] = rep->sweeps;
    if (rep->err) {
      fs_set_last_hip_error(hipErrorLaunchTimeOut, "a grid barrier or block flag of the setup gave up waiting",
                            __FILE__, __LINE__);
      fail(FS_ERR_DEVICE);
      return;
    }
    // the sketch marks a column holding NaN or Inf with a NaN norm; an infinite norm means overflow
    if (rep->nan) fail(FS_ERR_NONFINITE);
    else if (rep->inf) fail(FS_ERR_TOO_LARGE);
    else if (rep->b2 == 0.0 || !(hst[i].condest <= 1.0 / (o.tau_factor * U_ROUND))) fallback[i] = 1;
  };
  const int nthreads = std::min(kSetupSlots, std::max(nb, 1));
  struct Joiner {  // the setup threads are joined on every exit path (they use this frame's state)
    std::vector<std::thread> th;
    std::atomic<bool>* quit;
    ~Joiner() {
      quit->store(true);
      for (auto& t : th)
        if (t.joinable()) t.join();
    }
  } joiner{{}, &quit};
  for (int k = 0; k < nthreads; ++k)
    joiner.th.emplace_back([&, k]() {
      fs_context h = ctx->batch->ctx[k];
      (void)hipSetDevice(h->device);
      for (int q = k; q < nb; q += nthreads) {
        const int i = idx[q];
        if (!quit.load()) setup_one(h, ctx->batch->report[k], i);
        {
          std::lock_guard<std::mutex> lk(mu);
          ready[i] = 1;
        }
        cv.notify_all();
      }
    });

  // ---- lockstep refinement of one wave of set-up problems (act) on the caller's stream
  BatchVec* dbv = (BatchVec*)(base + total);
  BatchPass* dln = (BatchPass*)(base + total + vec_desc);
  BatchPass* dlr = (BatchPass*)(base + total + vec_desc + pass_desc);
  BatchPass* dlh = (BatchPass*)(base + total + vec_desc + 2 * pass_desc);
  DevState* dst = (DevState*)(base + total + vec_desc + 3 * pass_desc);
  hipEvent_t* ev = ctx->ev;
  auto refine = [&](const std::vector<int>& act) -> fs_status {
    const int na = (int)act.size();
    if (na == 0) return FS_OK;
    FS_HIP(hipEventRecord(ev[0], s));
    int max_n = 1;
    std::vector<BatchVec> bv(na);
    std::vector<int> keys;  // distinct (H, L, vec) keys
    auto key_of = [&](int i) { return (lay[i].H * 64 + lay[i].L) * 2 + (lay[i].vec ? 1 : 0); };
    for (int a = 0; a < na; ++a) {
      const int i = act[a];
      const int n = probs[i].n;
      max_n = std::max(max_n, n);
      double* vec = ptr(i, lay[i].off_vec);
      BatchVec& b = bv[a];
      b.n = n;
      b.done = 0;
      b.V = ptr(i, lay[i].off_V);
      b.sigma = ptr(i, lay[i].off_sigma);
      b.dinv = ptr(i, lay[i].off_dinv);
      b.x = vec;
      b.x0 = vec + n;
      b.c = vec + 2 * n;
      b.dy = vec + 3 * n;
      b.dy_old = vec + 4 * n;
      b.zs = vec + 5 * n;
      b.v = vec + 6 * n;
      b.u = vec + 7 * n;
      b.g = vec + 8 * n;
      b.xh = vec + 9 * n;
      b.w = vec + 10 * n;
      b.gpart = ptr(i, lay[i].off_gpart);
      b.x_out = probs[i].x;
      b.st = state_of(i);
      b.spir = probs[i].method == FS_METHOD_SPIR ? 1 : 0;
      b.res = vec + 11 * n;
      b.p = vec + 4 * n;  // (SPIR has no dy_old)
      if (std::find(keys.begin(), keys.end(), key_of(i)) == keys.end()) keys.push_back(key_of(i));
    }
    // pass work-lists: per (H, L, vec) group, the normal pass (v = D^{-1} A^T A zs), the residual pass
    // (g = D^{-1} A^T (b - A zs), ||b - A zs||^2 into the state) and the step heads (the residual pass
    // for every problem: its stop flag is still set from the previous step); each problem's
    // work-groups consecutive
    struct Group {
      int H, L;
      bool vec;
      int count, total;
      size_t first;  // index of the group's first entry in the lists
    };
    std::vector<Group> groups;
    std::vector<BatchPass> lnorm, lres, lhead;
    for (int key : keys) {
      Group g{key / 128, (key / 2) % 64, (key & 1) != 0, 0, 0, lnorm.size()};
      for (int a = 0; a < na; ++a) {
        const int i = act[a];
        if (key_of(i) != key) continue;
        BatchPass p{};
        p.A = probs[i].A;
        p.lda = probs[i].lda;
        p.m = probs[i].m;
        p.n = probs[i].n;
        p.zs = bv[a].zs;
        p.b = probs[i].b;
        p.partial = ptr(i, lay[i].off_part);
        p.partial_r2 = ptr(i, lay[i].off_pr2);
        p.stop = &bv[a].st->stop;
        p.wg0 = g.total;
        p.G = lay[i].G;
        p.out = bv[a].v;
        p.out_scale = bv[a].dinv;
        p.r2_out = nullptr;
        lnorm.push_back(p);
        p.out = bv[a].g;
        p.r2_out = &bv[a].st->r2;
        lres.push_back(p);
        p.stop = nullptr;
        lhead.push_back(p);
        g.total += lay[i].G;
        ++g.count;
      }
      groups.push_back(g);
    }
    std::vector<DevState> pst(na);
    FS_HIP(hipMemcpyAsync(dbv, bv.data(), sizeof(BatchVec) * na, hipMemcpyHostToDevice, s));
    FS_HIP(hipMemcpyAsync(dln, lnorm.data(), sizeof(BatchPass) * na, hipMemcpyHostToDevice, s));
    FS_HIP(hipMemcpyAsync(dlr, lres.data(), sizeof(BatchPass) * na, hipMemcpyHostToDevice, s));
    FS_HIP(hipMemcpyAsync(dlh, lhead.data(), sizeof(BatchPass) * na, hipMemcpyHostToDevice, s));
    auto read_states = [&]() -> fs_status {
      FS_K(fs_b_gather(dbv, na, dst, s));
      FS_HIP(hipMemcpyAsync(pst.data(), dst, sizeof(DevState) * na, hipMemcpyDeviceToHost, s));
      FS_HIP(hipStreamSynchronize(s));
      return FS_OK;
    };
    auto passes = [&](const BatchPass* list, bool resid) -> fs_status {
      for (const Group& g : groups)
        FS_K(fs_launch_pass_batched(list + g.first, g.count, g.H, g.L, g.vec, resid, g.total, max_n, s));
      return FS_OK;
    };
    const fs_options& o0 = opt[act[0]];  // shared fields (every problem has the caller's options)
    std::vector<int> iters0(na, 0), iters1(na, 0), conv(na, 0);
    std::vector<double> cn0(na, 0.0), cn1(na, 0.0);
    for (int step = 0; step < 2; ++step) {
      // head: zs = D^{-1} x, g = D^{-1} A^T (b - A zs), c = Sigma^{-1} V^T g, dy = dy_old = c
      FS_K(fs_b_vec(dbv, na, BatchOp::SCALE, 0, 0, 0, s));
      FS_TRY(passes(dlh, true));
      if (step == 0) FS_K(fs_b_vec(dbv, na, BatchOp::FIRST_THRESHOLD, 0, o0.gamma, o0.rho, s));
      FS_K(fs_b_gemv_PT(dbv, na, max_n, 0, s));
      FS_K(fs_b_vec(dbv, na, BatchOp::STEP_INIT, 0, 0, 0, s));
      bool all_stopped = false;
      const int cap = o0.max_inner;
      for (int j = 0; j < cap && !all_stopped; ++j) {
        FS_K(fs_b_gemv_P(dbv, na, max_n, 0, s));    // zs = D^{-1} V Sigma^{-1} dy (SPIR: p)
        FS_TRY(passes(dln, false));                // v = D^{-1} A^T A zs
        FS_K(fs_b_gemv_PT(dbv, na, max_n, 1, s));   // u = Sigma^{-1} V^T v
        FS_K(fs_b_vec(dbv, na, BatchOp::UPDATE, step == 0 ? 1 : 0, 0, 0, s));  // heavy ball or CG
        if (step == 1 && j % o0.kw_every == 0) {  // sketched KW at x_hat = x + P dy (second-step rule)
          FS_K(fs_b_gemv_P(dbv, na, max_n, 1, s));
          FS_K(fs_b_vec(dbv, na, BatchOp::XH_NORM, 0, 0, 0, s));
          FS_K(fs_b_vec(dbv, na, BatchOp::SCALE, 1, 0, 0, s));
          FS_TRY(passes(dlr, true));
          FS_K(fs_b_gemv_PT(dbv, na, max_n, 2, s));
          FS_K(fs_b_vec(dbv, na, BatchOp::KW, 0, 0, 0, s));
        }
        if (((j + 1) % o0.kw_every) == 0 || j == cap - 1) {
          FS_TRY(read_states());
          all_stopped = true;
          for (int a = 0; a < na; ++a) all_stopped &= pst[a].stop != 0;
        }
      }
      FS_K(fs_b_gemv_P(dbv, na, max_n, 2, s));  // x = x + P dy
      FS_TRY(read_states());
      for (int a = 0; a < na; ++a) {
        (step == 0 ? iters0 : iters1)[a] = pst[a].iters;
        (step == 0 ? cn0 : cn1)[a] = sqrt(pst[a].cnorm2);
        if (step == 1) conv[a] = pst[a].converged;
      }
    }
    FS_K(fs_b_vec(dbv, na, BatchOp::FINAL, 0, 0, 0, s));
    FS_HIP(hipEventRecord(ev[1], s));
    FS_HIP(hipStreamSynchronize(s));
    float loop_ms = 0.f;
    (void)hipEventElapsedTime(&loop_ms, ev[0], ev[1]);
    for (int a = 0; a < na; ++a) {
      const int i = act[a];
      const DevState& h = hst[i];
      if (!conv[a]) statuses[i] = FS_WARN_NOT_CONVERGED;
      if (infos) {
        fs_info& f = infos[i];
        f.iters[0] = iters0[a];
        f.iters[1] = iters1[a];
        f.flags = conv[a] ? 0 : FS_FLAG_NOT_CONVERGED;
        f.rank = probs[i].n;
        f.be_sk = pst[a].be_sk;
        f.normest = h.normest;
        f.condest = h.condest;
        f.cnorm[0] = cn0[a];
        f.cnorm[1] = cn1[a];
        f.kw_evals = pst[a].kw_evals;
        f.svd_sweeps = sweeps[i];
        f.phase_ms[0] = setup_ms[i];  // setup (sketch, QR, SVD, x_0) of this problem
        f.phase_ms[4] = loop_ms;      // the lockstep refinement of its wave
      }
    }
    return FS_OK;
  };
  // one wave after every setup: a refinement beside setup kernels runs its passes on the compute units
  // they leave free (a pass work-group needs most of a compute unit's registers), measured 3x slower than
  // alone, which costs more than the overlap gains
  const int wave = std::max(nb, 1);
  for (int w0 = 0; w0 < nb; w0 += wave) {
    const int w1 = std::min(nb, w0 + wave);
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        for (int q = w0; q < w1; ++q)
          if (!ready[idx[q]]) return false;
        return true;
      });
    }
    std::vector<int> act;
    for (int q = w0; q < w1; ++q)
      if (statuses[idx[q]] == FS_OK && !fallback[idx[q]]) act.push_back(idx[q]);
    FS_TRY(refine(act));
  }
  for (auto& t : joiner.th) t.join();

  // ---- problems outside the batched envelope, one by one on the caller's context
  for (int i = 0; i < count; ++i) {
    if (statuses[i] < 0 && statuses[i] != FS_ERR_NOMEM) continue;
    if (batched[i] && !fallback[i] && statuses[i] != FS_ERR_NOMEM) continue;
    const fs_problem& P = probs[i];
    fs_options o = opt[i];
    o.overlap_svd = opts_in ? opts_in->overlap_svd : 1;
    fs_info f{};
    statuses[i] = (P.method == FS_METHOD_SPIR ? spir_solve : fossils_solve)(ctx, P.m, P.n, P.A, P.lda, P.b, P.x, &o,
                                                                           &f);
    if (infos) infos[i] = f;
  }
  fs_status result = FS_OK;
  for (int i = 0; i < count; ++i) {
    if (statuses[i] < 0) return statuses[i];
    if (statuses[i] > result) result = statuses[i];
  }
  return result;
}

}  // namespace

// (every C++ exception stops at the C boundary: allocation or thread creation failures become FS_ERR_NOMEM,
// after the setup threads started so far have been joined)
extern "C" fs_status fossils_solve_batched(fs_context ctx, int32_t count, const fs_problem* probs,
                                           const fs_options* opts, fs_info* infos, fs_status* statuses) {
  try {
    return solve_batched(ctx, count, probs, opts, infos, statuses);
  } catch (...) {
    fs_set_last_hip_error(hipErrorOutOfMemory, "host allocation or thread creation in fossils_solve_batched",
                          __FILE__, __LINE__);
    return FS_ERR_NOMEM;
  }
}
