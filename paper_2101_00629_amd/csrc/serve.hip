// Continuous-batching server for K-L solve requests on one GPU.
//
// Requests (problem descriptor, M, tolerance, arrival time) queue in arrival
// order.  A pool of worker threads (one per slot) serves them: a worker takes
// the head request once it has arrived and a contiguous range of its device
// footprint (problem set-up + eigensolver workspace) is free in the server's
// arena, and drives that solve on its own stream with the whole Krylov state
// on the device, every buffer laid out inside the range.  Solves therefore
// progress independently, and their small kernels (transfers,
// orthogonalisation, the one-workgroup Rayleigh-Ritz eigensolves) overlap on
// the device.  Finished solves return their range at once, so waiting
// requests join while others run.  The arena and the dispatcher's launch
// lists are allocated when the server is created: serving itself allocates
// and frees no device memory (hipFree would also synchronise the device).
//
// Kernel products: a product too small to fill the chip on its own is handed
// to a dispatcher thread, which merges all pending products into shared
// persistent launches (one per block size and precision) over a combined work
// list; it launches as soon as every running solve is waiting for its product,
// or after a short gathering window.  Larger products launch directly on
// their own stream.  Every product keeps its own split-K partition, fixed by
// its own shape, and every reduction has a fixed order, and the direct /
// batched choice depends only on the request's own size: a request's result
// is bitwise the same whether it runs alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "eigrun.hpp"

namespace ka {

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(KA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

namespace {

using Clock = std::chrono::steady_clock;

// work items at which a single product fills the chip without batching
constexpr int64_t kDirectItems = 2048;
// longest wait for other solves to reach their kernel product
constexpr double kGatherSeconds = 150e-6;
constexpr int kRing = 8;   // device job/item buffers in flight

// First-fit ranges of the server's device arena (offsets and lengths in
// bytes, multiples of 256), adjacent free ranges merged.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void give(size_t off, size_t bytes) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Request {
  int64_t id = 0;
  ka_desc desc;
  int M = 0;
  double tol = 0.0;
  int maxit = 0;
  double arrival = 0.0;
  uint64_t tag = 0;
  double* lambda_host = nullptr;
  size_t bytes = 0;           // arena range (ka_request_bytes rounded up to 256)
  size_t offset = 0;          // start of the range once admitted
  std::vector<double> geo_knots, geo_ctrl;   // KA_NURBS: copies that desc points to
};

struct BatchDone {
  hipEvent_t ev = nullptr;   // recorded after the batch's launches
  int refs = 0;              // members that have not yet queued their wait
};

struct PendingGamma {
  GammaJob job;
  int b = 16, precision = KA_FP32;
  int64_t items = 0;
  hipEvent_t ready = nullptr;     // recorded on the requester's stream
  BatchDone* done = nullptr;      // set by the dispatcher
  bool launched = false;
  int status = KA_OK;
};

struct Server {
  size_t budget = 0;
  int max_slots = 1;
  char* arena_base = nullptr;   // hbm_budget bytes of device memory
  Arena arena;                  // its free ranges (mu)
  // shared state (mu)
  std::mutex mu;
  std::condition_variable cv;          // queue / completion changes
  std::condition_variable cv_gamma;    // dispatcher wake-up and launch notices
  size_t used = 0;
  int64_t next_id = 0;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<ka_result> done;
  int in_flight = 0;        // requests taken by workers and not finished
  int solving = 0;          // workers inside their iteration loop
  std::vector<PendingGamma*> pending;
  bool stop = false;
  // dispatcher
  hipStream_t stream = nullptr;
  hipEvent_t ring_ev[kRing] = {};
  GammaJob* jobs_dev[kRing] = {};     // launch lists, sized at creation: a batch holds at most one
  GammaItem* items_dev[kRing] = {};   // product per slot, each of fewer than kDirectItems items
  size_t jobs_cap = 0, items_cap = 0;
  std::vector<GammaJob> jobs_host[kRing];      // copy sources, alive until the slot's event completes
  std::vector<GammaItem> items_host[kRing];
  int ring_pos = 0;
  // clock and statistics
  Clock::time_point t0;
  bool started = false;
  int batches = 0;
  double batch_items = 0.0;
  int max_active = 0;
  int direct_launches = 0;
};

double now_s(const Server* S) { return std::chrono::duration<double>(Clock::now() - S->t0).count(); }

int64_t work_items(const GammaLaunch& a, int b) {
  const int64_t rpb = gamma_rows_per_block(b);
  return ((a.nr + rpb - 1) / rpb) * a.nsplit;
}

// ---- dispatcher -------------------------------------------------------------
int launch_batch(Server* S, std::vector<PendingGamma*>& batch, hipEvent_t done_ev) {
  const int slot = S->ring_pos;
  S->ring_pos = (S->ring_pos + 1) % kRing;
  // the device buffers of this slot may still be read by an older batch
  HIP_TRY(hipEventSynchronize(S->ring_ev[slot]));
  size_t ni = 0;
  for (auto* p : batch) ni += (size_t)p->items;
  if (batch.size() > S->jobs_cap || ni > S->items_cap)
    return fail(KA_ERR_STATE, "batched product exceeds the server's launch lists");
  std::map<std::pair<int, int>, std::vector<PendingGamma*>> groups;
  for (auto* p : batch) groups[{p->b, p->precision}].push_back(p);
  std::vector<GammaJob>& jobs = S->jobs_host[slot];
  std::vector<GammaItem>& items = S->items_host[slot];
  jobs.clear();
  items.clear();
  std::vector<std::tuple<int, int, size_t, size_t, size_t, size_t>> launches;   // b, prec, j0, j1, i0, i1
  for (auto& g : groups) {
    const size_t j0 = jobs.size(), i0 = items.size();
    for (auto* p : g.second) {
      const int jl = (int)(jobs.size() - j0);
      jobs.push_back(p->job);
      const int64_t rpb = gamma_rows_per_block(p->b);
      const int64_t rblocks = (p->job.a.nr + rpb - 1) / rpb;
      for (int sp = 0; sp < p->job.a.nsplit; ++sp)
        for (int64_t rb = 0; rb < rblocks; ++rb) items.push_back(GammaItem{jl, (int)rb, sp});
    }
    launches.emplace_back(g.first.first, g.first.second, j0, jobs.size(), i0, items.size());
  }
  for (auto* p : batch) HIP_TRY(hipStreamWaitEvent(S->stream, p->ready, 0));
  HIP_TRY(hipMemcpyAsync(S->jobs_dev[slot], jobs.data(), jobs.size() * sizeof(GammaJob), hipMemcpyHostToDevice,
                         S->stream));
  HIP_TRY(hipMemcpyAsync(S->items_dev[slot], items.data(), items.size() * sizeof(GammaItem), hipMemcpyHostToDevice,
                         S->stream));
  for (auto& L : launches) {
    const int b = std::get<0>(L), prec = std::get<1>(L);
    const size_t j0 = std::get<2>(L), j1 = std::get<3>(L), i0 = std::get<4>(L), i1 = std::get<5>(L);
    if (prec == KA_BF16X3)
      HIP_TRY(launch_gamma_split_jobs(S->jobs_dev[slot] + j0, (int)(j1 - j0), b, S->stream));
    HIP_TRY(launch_gamma_batch(S->jobs_dev[slot] + j0, S->items_dev[slot] + i0, (int)(i1 - i0), b, prec, S->stream));
    for (size_t q = j0; q < j1; ++q) {
      const GammaLaunch& a = jobs[q].a;
      if (a.nsplit > 1) HIP_TRY(launch_gamma_reduce(a.partial, a.nsplit, a.nr * b, a.Z, S->stream));
    }
  }
  HIP_TRY(hipEventRecord(done_ev, S->stream));
  HIP_TRY(hipEventRecord(S->ring_ev[slot], S->stream));
  S->batches++;
  S->batch_items += (double)items.size();
  return KA_OK;
}

void dispatcher_main(Server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv_gamma.wait(lk, [&] { return (S->stop && S->solving == 0) || !S->pending.empty(); });
    if (S->pending.empty()) return;    // stop requested and no solve left
    // gather: until every solving worker waits for its product, or the window closes
    const auto t_first = Clock::now();
    while (!S->stop && (int)S->pending.size() < S->solving &&
           Clock::now() - t_first < std::chrono::duration<double>(kGatherSeconds)) {
      S->cv_gamma.wait_for(lk, std::chrono::duration<double>(kGatherSeconds / 4));
    }
    std::vector<PendingGamma*> batch;
    batch.swap(S->pending);
    lk.unlock();
    BatchDone* bd = new BatchDone();
    bd->refs = (int)batch.size();
    int rc = hipEventCreateWithFlags(&bd->ev, hipEventDisableTiming) == hipSuccess ? KA_OK : KA_ERR_HIP;
    if (rc == KA_OK) rc = launch_batch(S, batch, bd->ev);
    lk.lock();
    for (auto* p : batch) {
      p->done = bd;
      p->status = rc;
      p->launched = true;
    }
    S->cv_gamma.notify_all();
  }
}

// ---- workers -------------------------------------------------------------------
void finish_request(Server* S, const Request& r, int status, double t_admit, EigRun* run) {
  ka_result res;
  std::memset(&res, 0, sizeof(res));
  res.id = r.id;
  res.tag = r.tag;
  res.status = status;
  res.arrival_s = r.arrival;
  res.admit_s = t_admit;
  if (status >= 0 && run) res.status = run->finish(r.lambda_host, nullptr, &res.info);
  res.done_s = now_s(S);
  std::lock_guard<std::mutex> g(S->mu);
  S->done.push_back(res);
}

// One block application's kernel product for the solve on `P`.
int product(Server* S, Problem* P, hipEvent_t ready) {
  GammaLaunch a = gamma_job(P);
  const int64_t items = work_items(a, P->b);
  if (items >= kDirectItems) {
    // fills the chip on its own
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->direct_launches++;
    }
    return gamma_step(P, P->w32b, P->w32a, P->stream);
  }
  PendingGamma pg;
  pg.job.a = a;
  pg.job.kernel = P->d.kernel;
  pg.b = P->b;
  pg.precision = P->d.precision;
  pg.items = items;
  pg.ready = ready;
  HIP_TRY(hipEventRecord(ready, P->stream));
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->pending.push_back(&pg);
    S->cv_gamma.notify_all();
    S->cv_gamma.wait(lk, [&] { return pg.launched; });
  }
  hipError_t e = hipSuccess;
  if (pg.status == KA_OK) {
    e = hipStreamWaitEvent(P->stream, pg.done->ev, 0);
    if (e != hipSuccess) (void)hipEventSynchronize(pg.done->ev);   // the batch still reads this request's buffers
  }
  bool last = false;
  {
    std::lock_guard<std::mutex> g(S->mu);
    last = --pg.done->refs == 0;
  }
  if (last) {
    if (pg.done->ev) (void)hipEventDestroy(pg.done->ev);
    delete pg.done;
  }
  if (pg.status != KA_OK) return pg.status;
  if (e != hipSuccess) return fail(KA_ERR_HIP, "stream wait on the batched product failed");
  P->pairs_total += (double)a.nr * (double)a.nc;
  return KA_OK;
}

void worker_main(Server* S) {
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess)
    return;
  while (true) {
    std::unique_ptr<Request> r;
    double t_admit = 0.0;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (true) {
        if (S->stop) break;
        if (S->queue.empty()) {
          S->cv.wait(lk);
          continue;
        }
        Request* h = S->queue.front().get();
        const double t = now_s(S);
        if (h->arrival > t) {
          S->cv.wait_for(lk, std::chrono::duration<double>(std::min(h->arrival - t, 0.005)));
          continue;
        }
        size_t off = 0;
        if (!S->arena.take(h->bytes, &off)) {
          if (S->in_flight == 0) {
            // the whole arena is free and still too small: reject
            ka_result res;
            std::memset(&res, 0, sizeof(res));
            res.id = h->id;
            res.tag = h->tag;
            res.status = KA_ERR_OOM;
            res.arrival_s = h->arrival;
            res.admit_s = res.done_s = t;
            S->done.push_back(res);
            S->queue.pop_front();
            S->cv.notify_all();
            continue;
          }
          S->cv.wait(lk);     // wait for a range to be returned
          continue;
        }
        r = std::move(S->queue.front());
        S->queue.pop_front();
        r->offset = off;
        S->used += r->bytes;
        S->in_flight++;
        S->max_active = std::max(S->max_active, S->in_flight);
        t_admit = t;
        break;
      }
      if (!r) break;
    }
    // solve, every device buffer inside the request's range of the arena
    Region region;
    region.base = S->arena_base + r->offset;
    region.size = r->bytes;
    Problem* P = nullptr;
    int rc = setup_problem(&r->desc, stream, &P, &region);
    std::unique_ptr<EigRun> run;
    if (rc == KA_OK) {
      run.reset(new EigRun(P, r->M, r->tol, r->maxit));
      rc = run->start();
    }
    bool solving_flag = false;
    if (rc == KA_OK) {
      std::lock_guard<std::mutex> g(S->mu);
      S->solving++;
      solving_flag = true;
    }
    bool done = false;
    while (rc == KA_OK && !done) {
      rc = run->pre_apply();
      if (rc == KA_OK) rc = product(S, P, ready);
      if (rc == KA_OK) rc = run->post_apply(done);
    }
    if (solving_flag) {
      std::lock_guard<std::mutex> g(S->mu);
      S->solving--;
      S->cv_gamma.notify_all();
    }
    finish_request(S, *r, rc, t_admit, rc == KA_OK ? run.get() : nullptr);
    run.reset();
    // the range is reused at once: no work of this request may still be queued
    (void)hipStreamSynchronize(stream);
    if (P) destroy_problem(P);
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->arena.give(r->offset, r->bytes);
      S->used -= r->bytes;
      S->in_flight--;
      S->cv.notify_all();
    }
  }
  (void)hipStreamSynchronize(stream);
  (void)hipEventDestroy(ready);
  (void)hipStreamDestroy(stream);
}

}  // namespace
}  // namespace ka

using namespace ka;

extern "C" {

int ka_request_bytes(const ka_desc* desc, int M, size_t* bytes) {
  if (!desc || !bytes) return fail(KA_ERR_ARG, "NULL argument");
  size_t fp = 0;
  if (int rc = footprint(desc, &fp)) return rc;
  int64_t N = 0;
  if (int rc = desc_sizes(desc, &N, nullptr, nullptr)) return rc;
  if (M < 1 || M > N) return fail(KA_ERR_ARG, "M must be in 1..N");
  *bytes = (fp + eig_workspace_bytes(N, M, desc->block) + 255) / 256 * 256;
  return KA_OK;
}

int ka_server_create(size_t hbm_budget, int max_slots, ka_server** out) {
  if (!out) return fail(KA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 256 || hbm_budget == 0) return fail(KA_ERR_ARG, "need 1 <= max_slots <= 256 and a budget");
  Server* S = new Server();
  S->budget = hbm_budget / 256 * 256;
  S->max_slots = max_slots;
  // all device memory of the server: the arena and the launch lists
  if (hipMalloc((void**)&S->arena_base, S->budget) != hipSuccess) {
    S->arena_base = nullptr;
    ka_server_destroy(reinterpret_cast<ka_server*>(S));
    return fail(KA_ERR_OOM, "server arena allocation failed");
  }
  S->arena.reset(S->budget);
  S->jobs_cap = (size_t)max_slots;
  S->items_cap = (size_t)max_slots * kDirectItems;
  bool ok = true;
  for (int i = 0; i < kRing && ok; ++i)
    ok = hipMalloc((void**)&S->jobs_dev[i], S->jobs_cap * sizeof(GammaJob)) == hipSuccess &&
         hipMalloc((void**)&S->items_dev[i], S->items_cap * sizeof(GammaItem)) == hipSuccess;
  if (!ok) {
    ka_server_destroy(reinterpret_cast<ka_server*>(S));
    return fail(KA_ERR_OOM, "server launch lists allocation failed");
  }
  ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < kRing && ok; ++i) {
    ok = hipEventCreateWithFlags(&S->ring_ev[i], hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipEventRecord(S->ring_ev[i], S->stream) == hipSuccess;
  }
  if (!ok) {
    ka_server_destroy(reinterpret_cast<ka_server*>(S));
    return fail(KA_ERR_HIP, "server stream creation failed");
  }
  S->t0 = Clock::now();
  *out = reinterpret_cast<ka_server*>(S);
  return KA_OK;
}

int ka_server_submit(ka_server* s, const ka_desc* desc, int M, double tol, int maxit, double arrival_s,
                     uint64_t tag, double* lambda_host, int64_t lambda_len, int64_t* req_id) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S || !desc || !lambda_host) return fail(KA_ERR_ARG, "NULL argument");
  size_t need = 0;
  if (int rc = ka_request_bytes(desc, M, &need)) return rc;
  if (lambda_len < lambda_doubles(*desc, M))
    return fail(KA_ERR_ARG, "lambda_host holds " + std::to_string(lambda_len) + " doubles, the request writes " +
                                std::to_string(lambda_doubles(*desc, M)));
  std::unique_ptr<Request> r(new Request());
  r->desc = *desc;
  if (desc->domain == KA_NURBS) {   // validated above: copy the geometry, the caller's arrays are not kept
    size_t nk = 0, nc = 4;
    for (int k = 0; k < 3; ++k) {
      nk += (size_t)desc->geo_nctrl[k] + desc->geo_degree[k] + 1;
      nc *= (size_t)desc->geo_nctrl[k];
    }
    r->geo_knots.assign(desc->geo_knots, desc->geo_knots + nk);
    r->geo_ctrl.assign(desc->geo_ctrl, desc->geo_ctrl + nc);
    r->desc.geo_knots = r->geo_knots.data();
    r->desc.geo_ctrl = r->geo_ctrl.data();
  }
  r->M = M;
  r->tol = tol;
  r->maxit = maxit;
  r->arrival = arrival_s;
  r->tag = tag;
  r->lambda_host = lambda_host;
  r->bytes = need;
  std::lock_guard<std::mutex> g(S->mu);
  r->id = S->next_id++;
  if (req_id) *req_id = r->id;
  auto pos = S->queue.end();       // keep arrival order
  while (pos != S->queue.begin() && (*(pos - 1))->arrival > arrival_s) --pos;
  S->queue.insert(pos, std::move(r));
  S->cv.notify_all();
  return KA_OK;
}

int ka_server_run(ka_server* s, double timeout_s) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S) return fail(KA_ERR_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (!S->started) {
      S->t0 = Clock::now();
      S->started = true;
    }
    S->stop = false;
  }
  std::thread disp(dispatcher_main, S);
  std::vector<std::thread> workers;
  for (int i = 0; i < S->max_slots; ++i) workers.emplace_back(worker_main, S);
  const auto t_end = Clock::now() + std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9);
  int rc = KA_OK;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    while (!(S->queue.empty() && S->in_flight == 0)) {
      if (S->cv.wait_until(lk, t_end) == std::cv_status::timeout && Clock::now() >= t_end) {
        rc = KA_NOT_CONVERGED;
        break;
      }
    }
    S->stop = true;
    S->cv.notify_all();
    S->cv_gamma.notify_all();
  }
  for (auto& w : workers) w.join();
  disp.join();
  (void)hipStreamSynchronize(S->stream);
  return rc;
}

int ka_server_poll(ka_server* s, ka_result* out, int max, int* n) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S || !n || (max > 0 && !out)) return fail(KA_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  const int k = std::min<int>(max, (int)S->done.size());
  for (int i = 0; i < k; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *n = k;
  return KA_OK;
}

int ka_server_stats(ka_server* s, int* batches, double* mean_items, int* max_active, size_t* bytes_in_use) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S) return fail(KA_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  if (batches) *batches = S->batches;
  if (mean_items) *mean_items = S->batches ? S->batch_items / S->batches : 0.0;
  if (max_active) *max_active = S->max_active;
  if (bytes_in_use) *bytes_in_use = S->used;
  return KA_OK;
}

void ka_server_destroy(ka_server* s) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S) return;
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (int i = 0; i < kRing; ++i) {
    if (S->ring_ev[i]) (void)hipEventDestroy(S->ring_ev[i]);
    if (S->jobs_dev[i]) (void)hipFree(S->jobs_dev[i]);
    if (S->items_dev[i]) (void)hipFree(S->items_dev[i]);
  }
  if (S->arena_base) (void)hipFree(S->arena_base);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
