// Continuous-batching server for K-L solve requests on one GPU.
//
// Requests (problem descriptor, M, tolerance, arrival time) queue in arrival
// order.  The serving loop admits a request once it has arrived, a slot is
// free and its device footprint (problem set-up + eigensolver workspace)
// fits the HBM budget; each admitted request keeps its whole Krylov state on
// the device, on its own stream.  Every iteration of the loop advances all
// active solves by one block application of A': their operator steps before
// the kernel product run on their own streams, then the kernel products of
// all of them run as shared persistent launches (one per block size and
// precision) over a combined work list, then each solve finishes its step
// (transfers, orthogonalisation, Rayleigh-Ritz).  Finished solves release
// their memory at once, so newly arrived requests join the running batch.
//
// Each product keeps its own split-K partition, fixed by its own shape, and
// every reduction has a fixed order: a request's result is bitwise the same
// whether it runs alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
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

struct Request {
  int64_t id = 0;
  ka_desc desc;
  int M = 0;
  double tol = 0.0;
  int maxit = 0;
  double arrival = 0.0;
  uint64_t tag = 0;
  double* lambda_host = nullptr;
  size_t bytes = 0;
  // runtime
  hipStream_t stream = nullptr;
  hipEvent_t ev_pre = nullptr;
  Problem* prob = nullptr;
  std::unique_ptr<EigRun> run;
  double t_admit = 0.0;
};

struct Server {
  size_t budget = 0;
  int max_slots = 1;
  size_t used = 0;
  int64_t next_id = 0;
  std::deque<std::unique_ptr<Request>> queue;      // not yet admitted, arrival order
  std::vector<std::unique_ptr<Request>> active;
  std::vector<ka_result> done;
  hipStream_t stream = nullptr;                     // batched kernel products
  hipEvent_t ev_gamma = nullptr;
  GammaJob* jobs_host = nullptr;
  GammaItem* items_host = nullptr;
  GammaJob* jobs_dev = nullptr;
  GammaItem* items_dev = nullptr;
  size_t jobs_cap = 0, items_cap = 0;
  std::chrono::steady_clock::time_point t0;
  bool started = false;
  int batches = 0;
  double batch_items = 0.0;
  int max_active = 0;
};

static double now_s(const Server* S) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
}

static int ensure_capacity(Server* S, size_t njobs, size_t nitems) {
  if (njobs > S->jobs_cap) {
    (void)hipHostFree(S->jobs_host);
    (void)hipFree(S->jobs_dev);
    S->jobs_cap = std::max(njobs, 2 * S->jobs_cap);
    HIP_TRY(hipHostMalloc((void**)&S->jobs_host, S->jobs_cap * sizeof(GammaJob)));
    HIP_TRY(hipMalloc((void**)&S->jobs_dev, S->jobs_cap * sizeof(GammaJob)));
  }
  if (nitems > S->items_cap) {
    (void)hipHostFree(S->items_host);
    (void)hipFree(S->items_dev);
    S->items_cap = std::max(nitems, 2 * S->items_cap);
    HIP_TRY(hipHostMalloc((void**)&S->items_host, S->items_cap * sizeof(GammaItem)));
    HIP_TRY(hipMalloc((void**)&S->items_dev, S->items_cap * sizeof(GammaItem)));
  }
  return KA_OK;
}

static void release(Server* S, Request* r) {
  r->run.reset();
  if (r->prob) destroy_problem(r->prob);
  r->prob = nullptr;
  if (r->ev_pre) (void)hipEventDestroy(r->ev_pre);
  if (r->stream) (void)hipStreamDestroy(r->stream);
  r->ev_pre = nullptr;
  r->stream = nullptr;
  S->used -= r->bytes;
}

static void finish_request(Server* S, Request* r, int status) {
  ka_result res;
  std::memset(&res, 0, sizeof(res));
  res.id = r->id;
  res.tag = r->tag;
  res.status = status;
  res.arrival_s = r->arrival;
  res.admit_s = r->t_admit;
  if (status >= 0 && r->run) {
    const int rc = r->run->finish(r->lambda_host, nullptr, &res.info);
    res.status = rc;
  }
  res.done_s = now_s(S);
  S->done.push_back(res);
  release(S, r);
}

// Admit arrived requests while slots and memory allow (arrival order; the
// head of the queue waits for memory rather than being overtaken).
static int admit(Server* S) {
  const double t = now_s(S);
  while (!S->queue.empty() && (int)S->active.size() < S->max_slots && S->queue.front()->arrival <= t) {
    Request* r = S->queue.front().get();
    if (S->used + r->bytes > S->budget) {
      if (S->active.empty()) {
        // can never fit: reject
        std::unique_ptr<Request> own = std::move(S->queue.front());
        S->queue.pop_front();
        ka_result res;
        std::memset(&res, 0, sizeof(res));
        res.id = own->id;
        res.tag = own->tag;
        res.status = KA_ERR_OOM;
        res.arrival_s = own->arrival;
        res.admit_s = res.done_s = now_s(S);
        S->done.push_back(res);
        continue;
      }
      break;
    }
    std::unique_ptr<Request> own = std::move(S->queue.front());
    S->queue.pop_front();
    S->used += r->bytes;
    r->t_admit = t;
    HIP_TRY(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&r->ev_pre, hipEventDisableTiming));
    int rc = setup_problem(&r->desc, r->stream, &r->prob);
    if (rc == KA_OK) {
      r->run.reset(new EigRun(r->prob, r->M, r->tol, r->maxit));
      rc = r->run->start();
    }
    if (rc != KA_OK) {
      finish_request(S, r, rc);
      continue;
    }
    S->active.push_back(std::move(own));
  }
  S->max_active = std::max(S->max_active, (int)S->active.size());
  return KA_OK;
}

// One iteration: every active solve advances by one block application.
static int step(Server* S) {
  std::vector<Request*> act;
  for (auto& r : S->active) act.push_back(r.get());
  // 1. operator steps before the kernel product, per request stream
  for (Request* r : act) {
    const int rc = r->run->pre_apply();
    if (rc != KA_OK) return rc;
    HIP_TRY(hipEventRecord(r->ev_pre, r->stream));
    HIP_TRY(hipStreamWaitEvent(S->stream, r->ev_pre, 0));
  }
  // 2. shared launches of all kernel products, grouped by (b, precision)
  std::map<std::pair<int, int>, std::vector<Request*>> groups;
  for (Request* r : act) groups[{r->prob->b, r->prob->d.precision}].push_back(r);
  size_t nj = 0, ni = 0;
  for (auto& g : groups)
    for (Request* r : g.second) {
      const GammaLaunch a = gamma_job(r->prob);
      const int64_t rpb = gamma_rows_per_block(r->prob->b);
      ++nj;
      ni += (size_t)((a.nr + rpb - 1) / rpb) * a.nsplit;
    }
  if (int rc = ensure_capacity(S, nj, ni)) return rc;
  size_t j = 0, it = 0;
  for (auto& g : groups) {
    const size_t j0 = j, it0 = it;
    for (Request* r : g.second) {
      GammaJob job;
      job.a = gamma_job(r->prob);
      job.kernel = r->prob->d.kernel;
      S->jobs_host[j] = job;
      const int64_t rpb = gamma_rows_per_block(r->prob->b);
      const int64_t rblocks = (job.a.nr + rpb - 1) / rpb;
      for (int sp = 0; sp < job.a.nsplit; ++sp)
        for (int64_t rb = 0; rb < rblocks; ++rb) S->items_host[it++] = GammaItem{(int)(j - j0), (int)rb, sp};
      ++j;
    }
    HIP_TRY(hipMemcpyAsync(S->jobs_dev + j0, S->jobs_host + j0, (j - j0) * sizeof(GammaJob), hipMemcpyHostToDevice,
                           S->stream));
    HIP_TRY(hipMemcpyAsync(S->items_dev + it0, S->items_host + it0, (it - it0) * sizeof(GammaItem),
                           hipMemcpyHostToDevice, S->stream));
    HIP_TRY(launch_gamma_batch(S->jobs_dev + j0, S->items_dev + it0, (int)(it - it0), g.first.first,
                               g.first.second, S->stream));
    for (size_t q = j0; q < j; ++q) {
      const GammaLaunch& a = S->jobs_host[q].a;
      if (a.nsplit > 1) HIP_TRY(launch_gamma_reduce(a.partial, a.nsplit, a.nr * g.first.first, a.Z, S->stream));
    }
  }
  S->batches++;
  S->batch_items += (double)it;
  for (Request* r : act) r->prob->pairs_total += (double)r->prob->n_rows * (double)r->prob->n_cols;
  HIP_TRY(hipEventRecord(S->ev_gamma, S->stream));
  // the host staging buffers are reused next step: wait for the copies
  // (cheap: the stream only holds this step's copies and launches)
  // 3. the rest of each step, per request stream
  for (Request* r : act) HIP_TRY(hipStreamWaitEvent(r->stream, S->ev_gamma, 0));
  std::vector<std::unique_ptr<Request>> keep;
  for (auto& own : S->active) {
    Request* r = own.get();
    bool done = false;
    const int rc = r->run->post_apply(done);
    if (rc != KA_OK) {
      finish_request(S, r, rc);
      continue;
    }
    if (done) {
      finish_request(S, r, KA_OK);
      continue;
    }
    keep.push_back(std::move(own));
  }
  S->active = std::move(keep);
  HIP_TRY(hipStreamSynchronize(S->stream));
  return KA_OK;
}

}  // namespace ka

using namespace ka;

extern "C" {

int ka_server_create(size_t hbm_budget, int max_slots, ka_server** out) {
  if (!out) return fail(KA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || hbm_budget == 0) return fail(KA_ERR_ARG, "need max_slots >= 1 and a budget");
  Server* S = new Server();
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&S->ev_gamma, hipEventDisableTiming) != hipSuccess) {
    delete S;
    return fail(KA_ERR_HIP, "server stream creation failed");
  }
  S->t0 = std::chrono::steady_clock::now();
  *out = reinterpret_cast<ka_server*>(S);
  return KA_OK;
}

int ka_request_bytes(const ka_desc* desc, int M, size_t* bytes) {
  if (!desc || !bytes) return fail(KA_ERR_ARG, "NULL argument");
  size_t fp = 0;
  if (int rc = footprint(desc, &fp)) return rc;
  int64_t N = 1;
  for (int k = 0; k < 3; ++k) N *= desc->degree[k] + desc->nel[k];
  if (M < 1 || M > N) return fail(KA_ERR_ARG, "M must be in 1..N");
  *bytes = fp + eig_workspace_bytes(N, M, desc->block);
  return KA_OK;
}

int ka_server_submit(ka_server* s, const ka_desc* desc, int M, double tol, int maxit, double arrival_s,
                     uint64_t tag, double* lambda_host, int64_t* req_id) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S || !desc || !lambda_host) return fail(KA_ERR_ARG, "NULL argument");
  size_t need = 0;
  if (int rc = ka_request_bytes(desc, M, &need)) return rc;
  std::unique_ptr<Request> r(new Request());
  r->id = S->next_id++;
  r->desc = *desc;
  r->M = M;
  r->tol = tol;
  r->maxit = maxit;
  r->arrival = arrival_s;
  r->tag = tag;
  r->lambda_host = lambda_host;
  r->bytes = need;
  if (req_id) *req_id = r->id;
  // keep arrival order
  auto pos = S->queue.end();
  while (pos != S->queue.begin() && (*(pos - 1))->arrival > arrival_s) --pos;
  S->queue.insert(pos, std::move(r));
  return KA_OK;
}

int ka_server_run(ka_server* s, double timeout_s) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S) return fail(KA_ERR_ARG, "server is NULL");
  if (!S->started) {
    S->t0 = std::chrono::steady_clock::now();
    S->started = true;
  }
  const double t_end = now_s(S) + (timeout_s > 0 ? timeout_s : 1e300);
  while (!S->queue.empty() || !S->active.empty()) {
    if (now_s(S) > t_end) return KA_NOT_CONVERGED;
    if (int rc = admit(S)) return rc;
    if (S->active.empty()) {
      if (S->queue.empty()) break;
      const double wait = S->queue.front()->arrival - now_s(S);
      if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
      continue;
    }
    if (int rc = step(S)) return rc;
  }
  return KA_OK;
}

int ka_server_poll(ka_server* s, ka_result* out, int max, int* n) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S || !n || (max > 0 && !out)) return fail(KA_ERR_ARG, "NULL argument");
  const int k = std::min<int>(max, (int)S->done.size());
  for (int i = 0; i < k; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *n = k;
  return KA_OK;
}

int ka_server_stats(ka_server* s, int* batches, double* mean_items, int* max_active, size_t* bytes_in_use) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S) return fail(KA_ERR_ARG, "server is NULL");
  if (batches) *batches = S->batches;
  if (mean_items) *mean_items = S->batches ? S->batch_items / S->batches : 0.0;
  if (max_active) *max_active = S->max_active;
  if (bytes_in_use) *bytes_in_use = S->used;
  return KA_OK;
}

void ka_server_destroy(ka_server* s) {
  Server* S = reinterpret_cast<Server*>(s);
  if (!S) return;
  (void)hipDeviceSynchronize();
  for (auto& r : S->active) release(S, r.get());
  S->active.clear();
  S->queue.clear();
  (void)hipHostFree(S->jobs_host);
  (void)hipHostFree(S->items_host);
  (void)hipFree(S->jobs_dev);
  (void)hipFree(S->items_dev);
  if (S->ev_gamma) (void)hipEventDestroy(S->ev_gamma);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
