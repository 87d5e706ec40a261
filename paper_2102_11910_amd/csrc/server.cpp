// Request server for independent solves: callers queue requests from any
// thread; one worker thread solves them in arrival order as batches of up to
// max_slots problems and records each request's completion.  It keeps
// kServerSets workspace sets, each with its own stream: a batch goes to a
// free set, so batches of different requests run on the device at the same
// time (a small batch is not held behind a large one).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gpf_internal.h"

using Clock = std::chrono::steady_clock;

namespace {

// Device bytes of a server plan on an n x n grid (LGF table, FP32 and FP64
// spectra, the plan's own workspace), rounded up.
size_t plan_bytes(int n) {
  const size_t c = (size_t)(n + 1) * (n + 1);
  return 20 * c + 44 * (size_t)n * n + (1u << 20);
}

// Device bytes of one problem workspace, rounded up: per cell the source
// fields and half spectra of both precisions and the tiles' halo slots
// (46 B) and the first convolution's band buffer (at most n rows of FP64
// complex: 16 B); per vortex the rank and the 32-byte record (36 B) and the
// window slots of split tiles (at most 2 / 512 of a 9800-byte window:
// 39 B); per surface point the Schur right-hand sides, products and f
// (80 B).
size_t slot_bytes(int n, int nv, int ns) {
  const size_t cap = nv > 1024 ? (size_t)nv : 1024;
  return 62 * (size_t)(n + 1) * n + 75 * cap + 80 * (size_t)ns + (1u << 20);
}

constexpr int kServerSets = 3;

bool same_grid(const gpf_grid &a, const gpf_grid &b) {
  return a.n == b.n && a.dx == b.dx && a.x0 == b.x0 && a.y0 == b.y0;
}

}  // namespace

struct gpf_server {
  struct Req {
    unsigned long long id;
    gpf_plan *plan;
    const gpf_body *body;
    gpf_inputs in;
    gpf_outputs out;
    Clock::time_point t0;
  };
  struct State {
    bool done = false;
    gpf_status st = GPF_OK;
    double latency = 0.0;
  };

  gpf_ctx *ctx = nullptr;
  size_t budget = 0;
  int max_slots = 0;
  unsigned flags = 0;

  std::mutex plan_mu;                                  // plans, bytes, high-water marks
  std::vector<std::pair<gpf_grid, gpf_plan *>> plans;
  size_t plans_total = 0;
  int n_hw = 0, nv_hw = 0, ns_hw = 0;

  std::mutex mu;                                       // queue, states, in-flight sets
  std::condition_variable cv_work, cv_done;
  std::deque<Req> queue;
  std::unordered_map<unsigned long long, State> states;
  unsigned long long next_id = 1;
  bool stop = false;

  gpf_batch *batch[kServerSets] = {};
  hipStream_t stream[kServerSets] = {};
  hipEvent_t ev[kServerSets] = {};
  std::vector<Req> inflight[kServerSets];
  bool busy[kServerSets] = {};
  unsigned long long batches = 0;   // dispatched batches
  int max_busy = 0;                 // most batches in flight at once
  std::thread worker;

  void run();
  void retire(int k);
  void finish(const std::vector<Req> &rs, gpf_status st);
  gpf_status dispatch(int k, std::vector<Req> &rs);
  ~gpf_server();
};

void gpf_server::finish(const std::vector<Req> &rs, gpf_status st) {
  const auto now = Clock::now();
  for (const Req &r : rs) {
    State &s = states[r.id];
    s.done = true;
    s.st = st;
    s.latency = std::chrono::duration<double>(now - r.t0).count();
  }
  cv_done.notify_all();
}

void gpf_server::retire(int k) {
  finish(inflight[k], GPF_OK);
  inflight[k].clear();
  busy[k] = false;
}

// Solve one batch on the stream of workspace set k (called without the lock
// held).  A batch that the library refuses is retried request by request, so
// that one bad request fails alone.
gpf_status gpf_server::dispatch(int k, std::vector<Req> &rs) {
  const int m = (int)rs.size();
  {
    // the set's workspaces go straight to the admitted high-water sizes
    // (what admission budgets for every slot), so that they grow, and
    // synchronise the device, rarely instead of with each new largest request
    std::lock_guard<std::mutex> lk(plan_mu);
    batch[k]->hw_n = std::max(batch[k]->hw_n, n_hw);
    batch[k]->hw_nv = std::max(batch[k]->hw_nv, nv_hw);
    batch[k]->hw_ns = std::max(batch[k]->hw_ns, ns_hw);
  }
  std::vector<gpf_plan *> pl(m);
  std::vector<const gpf_body *> bo(m);
  std::vector<gpf_inputs> in(m);
  std::vector<gpf_outputs> out(m);
  for (int i = 0; i < m; ++i) {
    pl[i] = rs[i].plan;
    bo[i] = rs[i].body;
    in[i] = rs[i].in;
    out[i] = rs[i].out;
  }
  gpf_status st = gpf_solve_batched(batch[k], m, pl.data(), bo.data(), in.data(), out.data(), stream[k]);
  if (st == GPF_OK) return GPF_OK;
  std::vector<Req> ok;
  for (int i = 0; i < m; ++i) {
    const gpf_status s1 = gpf_solve_batched(batch[k], 1, &pl[i], &bo[i], &in[i], &out[i], stream[k]);
    if (s1 == GPF_OK) {
      ok.push_back(rs[i]);
    } else {
      std::lock_guard<std::mutex> lk(mu);
      finish({rs[i]}, s1);
    }
  }
  rs.swap(ok);
  return GPF_OK;
}

void gpf_server::run() {
  if (hipSetDevice(ctx->device) != hipSuccess) return;
  std::unique_lock<std::mutex> lk(mu);
  int next = 0;   // first workspace set to try (round robin)
  for (;;) {
    int nbusy = 0;
    for (int k = 0; k < kServerSets; ++k) {
      if (busy[k] && hipEventQuery(ev[k]) == hipSuccess) retire(k);
      nbusy += busy[k] ? 1 : 0;
    }
    int k = -1;
    for (int q = 0; q < kServerSets && k < 0; ++q)
      if (!busy[(next + q) % kServerSets]) k = (next + q) % kServerSets;
    if (!queue.empty() && k >= 0) {
      std::vector<Req> rs;
      while (!queue.empty() && (int)rs.size() < max_slots) {
        rs.push_back(queue.front());
        queue.pop_front();
      }
      lk.unlock();
      dispatch(k, rs);
      const bool any = !rs.empty();
      const hipError_t e = any ? hipEventRecord(ev[k], stream[k]) : hipSuccess;
      lk.lock();
      if (!any) continue;
      if (e != hipSuccess) {
        finish(rs, GPF_E_DEVICE);
        continue;
      }
      inflight[k] = std::move(rs);
      busy[k] = true;
      ++batches;
      max_busy = std::max(max_busy, nbusy + 1);
      next = (k + 1) % kServerSets;
      continue;
    }
    if (stop && queue.empty() && nbusy == 0) break;
    if (nbusy > 0)
      cv_work.wait_for(lk, std::chrono::microseconds(20));   // poll the in-flight batches
    else
      cv_work.wait(lk);
  }
}

gpf_server::~gpf_server() {
  for (int k = 0; k < kServerSets; ++k) {
    if (ev[k]) (void)hipEventDestroy(ev[k]);
    gpf_batch_destroy(batch[k]);
    if (stream[k]) (void)hipStreamDestroy(stream[k]);
  }
  for (auto &p : plans) gpf_plan_destroy(p.second);
}

extern "C" {

gpf_status gpf_server_create(gpf_ctx *ctx, size_t hbm_budget_bytes, int max_slots,
                             unsigned plan_flags, gpf_server **out) {
  if (!ctx || !out || max_slots < 1 || max_slots > 256 || hbm_budget_bytes == 0)
    return gpf::fail(GPF_E_INVALID, "gpf_server_create: bad arguments");
  *out = nullptr;
  if (plan_flags & ~(unsigned)(GPF_FP64 | GPF_CONV1_FP64 | GPF_POLICY_AUTO))
    return gpf::fail(GPF_E_INVALID, "gpf_server_create: unknown plan flag");
  GPF_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<gpf_server> s(new gpf_server);
  s->ctx = ctx;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->flags = plan_flags;
  for (int k = 0; k < kServerSets; ++k) {
    GPF_TRY(gpf_batch_create(ctx, max_slots, &s->batch[k]));
    s->batch[k]->hw_all = true;   // slots at the admitted high-water sizes
    // merged batches on the set's stream alone: the three sets already run
    // side by side, and side streams inside a small batch cost more than
    // they overlap (serving mix at 0.8 of saturation: p50 0.66-0.71 ms
    // against 0.82-0.85 with them; saturated rate and p99 the same)
    s->batch[k]->merge = 2;
    GPF_HIP(hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming));
    GPF_HIP(hipStreamCreateWithFlags(&s->stream[k], hipStreamNonBlocking));
  }
  gpf_server *raw = s.get();
  s->worker = std::thread([raw] { raw->run(); });
  *out = s.release();
  return GPF_OK;
}

gpf_status gpf_server_plan(gpf_server *srv, const gpf_grid *grid, gpf_plan **out) {
  if (!srv || !grid || !out) return gpf::fail(GPF_E_INVALID, "gpf_server_plan: null argument");
  std::lock_guard<std::mutex> lk(srv->plan_mu);
  for (auto &p : srv->plans)
    if (same_grid(p.first, *grid)) {
      *out = p.second;
      return GPF_OK;
    }
  const size_t need = srv->plans_total + plan_bytes(grid->n) +
                      kServerSets * (size_t)srv->max_slots *
                          slot_bytes(std::max(srv->n_hw, grid->n), srv->nv_hw, srv->ns_hw);
  if (need > srv->budget)
    return gpf::fail(GPF_E_NOMEM, "gpf_server_plan: the plan would exceed the server's HBM budget");
  gpf_plan *p = nullptr;
  GPF_TRY(gpf_plan_create(srv->ctx, grid, srv->flags, &p));
  srv->plans.emplace_back(*grid, p);
  srv->plans_total += plan_bytes(grid->n);
  *out = p;
  return GPF_OK;
}

gpf_status gpf_server_submit(gpf_server *srv, const gpf_grid *grid, const gpf_body *body,
                             const gpf_inputs *in, const gpf_outputs *out,
                             unsigned long long *request_id) {
  if (!srv || !grid || !in || !out || !request_id)
    return gpf::fail(GPF_E_INVALID, "gpf_server_submit: null argument");
  if (in->mode != GPF_NOBODY && !body)
    return gpf::fail(GPF_E_INVALID, "gpf_server_submit: this mode needs a body");
  gpf_plan *plan = nullptr;
  GPF_TRY(gpf_server_plan(srv, grid, &plan));
  if (body && body->plan != plan)
    return gpf::fail(GPF_E_INVALID, "gpf_server_submit: body not created on the server plan of this grid");
  {
    // admission: every workspace set at the high-water sizes must fit
    std::lock_guard<std::mutex> lk(srv->plan_mu);
    const int n = std::max(srv->n_hw, grid->n);
    const int nv = std::max(srv->nv_hw, in->nv);
    const int ns = std::max(srv->ns_hw, body ? body->ns : 0);
    if (srv->plans_total + kServerSets * (size_t)srv->max_slots * slot_bytes(n, nv, ns) > srv->budget)
      return gpf::fail(GPF_E_NOMEM, "gpf_server_submit: request exceeds the server's HBM budget");
    srv->n_hw = n;
    srv->nv_hw = nv;
    srv->ns_hw = ns;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return gpf::fail(GPF_E_INVALID, "gpf_server_submit: server is shutting down");
  if ((int)srv->queue.size() >= 64 * srv->max_slots)
    return gpf::fail(GPF_E_BUSY, "gpf_server_submit: queue full");
  gpf_server::Req r{srv->next_id++, plan, in->mode == GPF_NOBODY ? nullptr : body, *in, *out,
                    Clock::now()};
  srv->states[r.id] = gpf_server::State{};
  srv->queue.push_back(r);
  *request_id = r.id;
  srv->cv_work.notify_one();
  return GPF_OK;
}

gpf_status gpf_server_poll(gpf_server *srv, unsigned long long request_id, int *done,
                           double *latency_s) {
  if (!srv || !done) return gpf::fail(GPF_E_INVALID, "gpf_server_poll: null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->states.find(request_id);
  if (it == srv->states.end()) return gpf::fail(GPF_E_INVALID, "gpf_server_poll: unknown request");
  *done = it->second.done ? 1 : 0;
  if (!it->second.done) return GPF_OK;
  if (latency_s) *latency_s = it->second.latency;
  const gpf_status st = it->second.st;
  srv->states.erase(it);
  if (st != GPF_OK) return gpf::fail(st, "gpf_server_poll: the request failed to launch");
  return GPF_OK;
}

gpf_status gpf_server_wait(gpf_server *srv, unsigned long long request_id, double *latency_s) {
  if (!srv) return gpf::fail(GPF_E_INVALID, "gpf_server_wait: null argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->states.find(request_id);
  if (it == srv->states.end()) return gpf::fail(GPF_E_INVALID, "gpf_server_wait: unknown request");
  // another thread may poll the same id to completion and erase it: stop
  // waiting when the entry is gone (never re-insert it)
  srv->cv_done.wait(lk, [&] {
    auto jt = srv->states.find(request_id);
    return jt == srv->states.end() || jt->second.done;
  });
  it = srv->states.find(request_id);
  if (it == srv->states.end())
    return gpf::fail(GPF_E_INVALID, "gpf_server_wait: the request was collected by another caller");
  if (latency_s) *latency_s = it->second.latency;
  const gpf_status st = it->second.st;
  srv->states.erase(it);
  if (st != GPF_OK) return gpf::fail(st, "gpf_server_wait: the request failed to launch");
  return GPF_OK;
}

void gpf_server_destroy(gpf_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  for (int k = 0; k < kServerSets; ++k)
    if (srv->stream[k]) (void)hipStreamSynchronize(srv->stream[k]);
  delete srv;
}

gpf_status gpf_server_stats(gpf_server *srv, unsigned long long *batches, int *max_inflight) {
  if (!srv) return gpf::fail(GPF_E_INVALID, "gpf_server_stats: null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (batches) *batches = srv->batches;
  if (max_inflight) *max_inflight = srv->max_busy;
  return GPF_OK;
}

}  // extern "C"
