// Serving form: a continuous-batching request loop on one GPU.
//
// Requests (fit + predict of one problem) are queued in arrival order.  A
// request is admitted when a worker slot is free and its HBM estimate fits
// into the budget next to the requests already running; a finished request
// frees its slot and its share of the budget at once, so waiting requests
// join while others are still on the GPU.  Each slot is a host thread with
// its own HIP stream; the kernels of different requests overlap on the
// device.  Every request runs on its own model (B, D, mode, CG and Lanczos
// state stay resident for the request's life), and no result depends on
// what else runs: each kernel's arithmetic is fixed by its own inputs, so a
// request's results in the mix equal its results alone.
//
// Deadlock freedom of the sync-free solves under concurrency: each model's
// solves use at most CUs / slots work streams, so the streams of all solves
// in flight together never exceed the CU count and each keeps a resident
// wave.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "vl_internal.h"
#include "vl_laplace.h"
#include "vl_ops.h"

namespace vl {

Model* model_of(vl_model* h);

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
  int64_t ticket = 0;
  vl_request req{};
  double bytes = 0.0;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  bool done = false;
  vl_status status = VL_OK;
  double nll = 0.0;
  vl_stats st{};
};

struct Server {
  int slots = 1;
  double budget = 0.0, in_use = 0.0;
  vl_opts opts{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Job>> queue;    // waiting, arrival order
  std::deque<std::shared_ptr<Job>> ready;    // admitted, not yet taken by a slot
  std::map<int64_t, std::shared_ptr<Job>> jobs;
  int64_t next_ticket = 1;
  int running = 0;
  bool stop = false;
  double peak_in_use = 0.0;
  int peak_running = 0;
  int waiters = 0;                           // threads inside vl_server_wait
  std::vector<std::thread> workers;
};

// Device bytes one request holds while it runs: the model (coordinates,
// neighbours, B, B^T, D, level and head schedules, neighbour-search grid,
// the grouped B and B^T, the dense inverse of the leading block), the block
// CG state for the probes and for one prediction tile, and the prediction
// factor.
double request_bytes(const vl_request& r, const vl_opts& o) {
  const double n = static_cast<double>(r.n), m = r.m, np = static_cast<double>(r.n_p);
  const int tile = (o.pred_tile > 0 && o.pred_tile < o.num_pred_samples) ? o.pred_tile
                                                                          : o.num_pred_samples;
  const double t = std::max(o.num_probes, tile);
  const double kd = std::min(n, static_cast<double>(kDenseRows));
  const double model = n * (16.0 + m * 12.0 + m * 16.0 + 8.0 * 8.0 + 64.0) +
                       n * (16.0 * m + 64.0 * (m + 1)) + 16.0 * kd * kd + 64.0 * 1048576.0;
  const double cg = 10.0 * n * t * 8.0;
  const double pred = np * (m * 12.0 + 40.0);
  return model + cg + pred;
}

// Admit waiting requests in arrival order while a slot and the budget allow
// (the head of the queue is never overtaken).  Caller holds the lock.
static void admit(Server& S) {
  while (!S.queue.empty() && S.running + static_cast<int>(S.ready.size()) < S.slots) {
    auto& j = S.queue.front();
    const bool alone = S.running == 0 && S.ready.empty();
    if (!alone && S.in_use + j->bytes > S.budget) break;
    S.in_use += j->bytes;
    S.peak_in_use = std::max(S.peak_in_use, S.in_use);
    S.ready.push_back(j);
    S.queue.pop_front();
  }
  S.cv_work.notify_all();
}

static Status run_request(Job& J, const vl_opts& o, hipStream_t stream, int max_streams) {
  const vl_request& r = J.req;
  vl_model* h = nullptr;
  double theta[2] = {r.theta[0], r.theta[1]};
  auto code = [](vl_status s, const char* what) {
    return s == VL_OK ? Status::ok() : Status::make(s, std::string(what) + ": " + vl_last_error());
  };
  VL_TRY(code(vl_build_vecchia(r.coords, r.n, r.m, r.cov, theta, stream, 0, &h), "build"));
  model_of(h)->max_streams = max_streams;
  vl_opts oo = o;
  oo.seed = r.seed;
  // A loop that stops at its cap still writes its outputs: the request then
  // completes with VL_ERR_NO_CONVERGENCE and hit_cap set.
  Status s = [&]() -> Status {
    vl_stats st{};
    const double aux = r.aux;
    bool capped = false;
    vl_status c = vl_find_mode(h, r.y, r.F, r.lik, &aux, &oo, nullptr, &st);
    if (c != VL_OK && c != VL_ERR_NO_CONVERGENCE) return code(c, "mode");
    capped |= (c == VL_ERR_NO_CONVERGENCE) || st.hit_cap;
    J.st.newton_iters = st.newton_iters;
    J.st.cg_iters_total = st.cg_iters_total;
    c = vl_neg_log_marglik(h, &oo, &J.nll, nullptr, &st);
    if (c != VL_OK && c != VL_ERR_NO_CONVERGENCE) return code(c, "likelihood");
    capped |= (c == VL_ERR_NO_CONVERGENCE) || st.hit_cap;
    J.st.cg_iters_max = st.cg_iters_max;
    if (r.n_p > 0) {
      c = vl_predict(h, r.coords_p, r.n_p, r.Fp, &oo, r.mean_out, r.var_out, &st);
      if (c != VL_OK && c != VL_ERR_NO_CONVERGENCE) return code(c, "predict");
      capped |= (c == VL_ERR_NO_CONVERGENCE) || st.hit_cap;
    }
    J.st.hit_cap = capped ? 1 : 0;
    if (capped) return Status::make(VL_ERR_NO_CONVERGENCE, "a loop stopped at its cap");
    return Status::ok();
  }();
  vl_free(h);
  return s;
}

static void worker_loop(Server* S, int slot) {
  (void)slot;
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
  int dev_cus = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int max_streams = std::max(1, dev_cus / std::max(1, S->slots));
  for (;;) {
    std::shared_ptr<Job> J;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->ready.empty(); });
      if (S->stop && S->ready.empty()) break;
      J = S->ready.front();
      S->ready.pop_front();
      ++S->running;
      S->peak_running = std::max(S->peak_running, S->running);
      J->t_start = now_s();
    }
    Status st = run_request(*J, S->opts, stream, max_streams);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      J->status = st.good() ? VL_OK : st.code;
      J->t_done = now_s();
      J->st.t_ms = 1e3 * (J->t_done - J->t_submit);
      J->done = true;
      --S->running;
      S->in_use -= J->bytes;
      admit(*S);
    }
    S->cv_done.notify_all();
  }
  if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace vl

struct vl_server : public vl::Server {};

extern "C" {

vl_status vl_server_create(int slots, double hbm_budget_bytes, const vl_opts* o,
                           vl_server** out) {
  if (!out || !o || slots < 1 || slots > 64 || !(hbm_budget_bytes > 0.0))
    return vl::report(vl::Status::invalid("bad server arguments"));
  auto* S = new (std::nothrow) vl_server();
  if (!S) return vl::report(vl::Status::make(VL_ERR_OOM, "host allocation failed"));
  S->slots = slots;
  S->budget = hbm_budget_bytes;
  S->opts = *o;
  S->opts.replay_cg_iters = nullptr;  // requests run with their own tolerances
  S->opts.replay_len = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete S;
    return vl::report(vl::Status::make(VL_ERR_HIP, "no device"));
  }
  for (int k = 0; k < slots; ++k)
    S->workers.emplace_back([S, k, dev] {
      (void)hipSetDevice(dev);
      vl::worker_loop(S, k);
    });
  *out = S;
  return VL_OK;
}

vl_status vl_server_submit(vl_server* S, const vl_request* r, int64_t* ticket) {
  if (!S || !r || !ticket || !r->coords || !r->y || r->n < 1)
    return vl::report(vl::Status::invalid("bad request"));
  if (r->n_p > 0 && (!r->coords_p || !r->mean_out))
    return vl::report(vl::Status::invalid("prediction outputs missing"));
  auto J = std::make_shared<vl::Job>();
  J->req = *r;
  J->bytes = vl::request_bytes(*r, S->opts);
  J->t_submit = vl::now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return vl::report(vl::Status::make(VL_ERR_STATE, "server stopped"));
    J->ticket = S->next_ticket++;
    S->jobs[J->ticket] = J;
    S->queue.push_back(J);
    vl::admit(*S);
  }
  *ticket = J->ticket;
  return VL_OK;
}

vl_status vl_server_wait(vl_server* S, int64_t ticket, double* nll_out, vl_stats* st,
                         double* queue_ms) {
  if (!S) return vl::report(vl::Status::invalid("null server"));
  std::shared_ptr<vl::Job> J;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return vl::report(vl::Status::invalid("unknown ticket"));
    J = it->second;
    ++S->waiters;
    S->cv_done.wait(lk, [&] { return J->done; });
    S->jobs.erase(ticket);
    --S->waiters;
  }
  S->cv_done.notify_all();  // vl_server_free may wait for the last waiter
  if (nll_out) *nll_out = J->nll;
  if (st) *st = J->st;
  if (queue_ms) *queue_ms = 1e3 * (J->t_start - J->t_submit);
  if (J->status != VL_OK) return J->status;
  return VL_OK;
}

vl_status vl_server_info(vl_server* S, double* peak_bytes, int* peak_running) {
  if (!S) return vl::report(vl::Status::invalid("null server"));
  std::lock_guard<std::mutex> lk(S->mu);
  if (peak_bytes) *peak_bytes = S->peak_in_use;
  if (peak_running) *peak_running = S->peak_running;
  return VL_OK;
}

double vl_request_bytes(const vl_request* r, const vl_opts* o) {
  if (!r || !o) return -1.0;
  return vl::request_bytes(*r, *o);
}

void vl_server_free(vl_server* S) {
  if (!S) return;
  {
    // requests still waiting for admission are dropped: they complete with
    // VL_ERR_STATE, which wakes any thread waiting for them
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (auto& j : S->queue) {
      j->status = VL_ERR_STATE;
      j->t_start = j->t_done = vl::now_s();
      j->done = true;
    }
    S->queue.clear();
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  for (auto& t : S->workers) t.join();
  {
    // the server outlives every vl_server_wait that is still returning
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->waiters == 0; });
  }
  delete S;
}

}  // extern "C"
