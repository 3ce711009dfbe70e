// Solve server of the fcgmg library: concurrent finite cell Stokes solves with device-resident
// hierarchies and admission by device-memory footprint (see include/fcgmg.h, fcgmg_server_*).
//
// A client of the library's own C-ABI. Worker threads, one HIP stream each, take requests in
// arrival order; a request whose hierarchy is not resident is admitted once its footprint fits the
// memory budget, after evicting idle hierarchies least recently used first. Without a fixed cache
// policy the server picks the fastest of the three policies of Sec. 3.1.2 whose footprint fits
// (cache_inverse, cache_matrix, cache_none). Requests with the same problem reuse one hierarchy,
// one solve at a time (its level buffers are scratch of the solve).
//
// Continuous batching: a request that the batched cycle takes is only set up by its worker; it then
// joins the running batch of an engine thread, which advances every joined request by one V-cycle
// per step in shared launches (fcgmg_batch.cpp) and retires each as it meets its stopping test.
#include <hip/hip_runtime.h>

#include <algorithm>
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

#include "fcgmg_impl.h"

using namespace fcg;

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// Policies in order of speed (Sec. 3.1.2: cache_inverse fastest, cache_none slowest).
const int kPolicyBySpeed[3] = {FCGMG_CACHE_INVERSE, FCGMG_CACHE_MATRIX, FCGMG_CACHE_NONE};

struct Entry {
  std::string key;          // problem bytes (params with the policy) + obstacles
  fcgmg_h h = nullptr;
  double* b = nullptr;      // right-hand side of the finest level (fcgmg_rhs), computed once
  int64_t ndof = 0;
  int64_t bytes = 0;        // footprint + b
  int policy = 0;
  bool busy = false;
  bool ready = false;       // set-up finished
  uint64_t last_use = 0;
};

struct Request {
  int64_t id = 0;
  fcgmg_params prm{};
  std::vector<double> balls;
  double rtol = 1e-8;
  double* x = nullptr;
  int64_t fp[3] = {-1, -1, -1};  // footprint per policy (-1: not a candidate)
  Clock::time_point t_submit, t_start, t_setup_done, t_done;
  bool done = false;
  fcgmg_request_result res{};
  Entry* entry = nullptr;  // the hierarchy it runs on (batched requests: while in the batch)
  double r0 = 0;           // initial residual norm (batched requests)
};

std::string problem_key(const fcgmg_params& p, const std::vector<double>& balls) {
  std::string k(reinterpret_cast<const char*>(&p), sizeof(p));
  k.append(reinterpret_cast<const char*>(balls.data()), balls.size() * sizeof(double));
  return k;
}

}  // namespace

struct fcgmg_server {
  fcgmg_server_params sp{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::unique_ptr<Entry>> entries;
  // device bytes of the problems (parameters with the policy, and obstacles) seen so far: the host
  // planning behind fcgmg_footprint_bytes takes up to a second on the largest grids, and a stream of
  // requests repeats its problems. At most kFootprintTable entries; a full table starts over.
  static constexpr size_t kFootprintTable = 4096;
  std::map<std::string, int64_t> footprints;
  int64_t in_use = 0;
  int64_t next_id = 1;
  uint64_t tick = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  // continuous batching
  std::deque<Request*> joining;  // set up, waiting to join the batch
  std::condition_variable cv_engine;
  bool engine_stop = false;
  std::thread engine;
  int64_t engine_steps = 0, engine_request_cycles = 0;
  int engine_max_batch = 0;

  // Completion of a request under the lock: results, timings, its hierarchy released.
  void finish_locked(Request* r, int rc) {
    r->t_done = Clock::now();
    r->res.status = rc;
    r->res.t_queue_ms = ms_since(r->t_submit, r->t_start);
    r->res.t_setup_ms = ms_since(r->t_start, r->t_setup_done);
    r->res.t_solve_ms = ms_since(r->t_setup_done, r->t_done);
    r->res.t_total_ms = ms_since(r->t_submit, r->t_done);
    if (Entry* e = r->entry) {
      e->busy = false;
      e->last_use = ++tick;
    }
    r->done = true;
  }

  void engine_loop() {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    fcgmg_batch* bt = nullptr;
    (void)batch_engine_create(&bt);
    std::vector<Request*> active;
    for (;;) {
      std::vector<Request*> join;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_engine.wait(lk, [&] { return !joining.empty() || !active.empty() || engine_stop; });
        if (joining.empty() && active.empty() && engine_stop) break;
        join.assign(joining.begin(), joining.end());
        joining.clear();
      }
      std::vector<Request*> retire;
      std::vector<int> codes;
      auto vecs = [](const std::vector<Request*>& rs, std::vector<fcgmg_ctx*>& hs, std::vector<double*>& xs,
                     std::vector<const double*>& bs) {
        hs.clear();
        xs.clear();
        bs.clear();
        for (Request* r : rs) {
          hs.push_back(r->entry->h);
          xs.push_back(r->x);
          bs.push_back(r->entry->b);
        }
      };
      std::vector<fcgmg_ctx*> hs;
      std::vector<double*> xs;
      std::vector<const double*> bs;
      std::vector<double> nrm;
      if (!join.empty()) {  // initial residual norms of the joining requests
        vecs(join, hs, xs, bs);
        const int rc = batch_engine_step(bt, hs, xs.data(), bs.data(), false, s, nrm);
        for (size_t k = 0; k < join.size(); ++k) {
          Request* r = join[k];
          if (rc != FCGMG_OK || !std::isfinite(nrm[k])) {
            retire.push_back(r);
            codes.push_back(rc != FCGMG_OK ? rc : set_error(FCGMG_E_NAN, "server: non-finite initial residual"));
          } else if (nrm[k] == 0.0) {
            retire.push_back(r);
            codes.push_back(FCGMG_OK);
          } else {
            r->r0 = nrm[k];
            active.push_back(r);
          }
        }
      }
      if (!active.empty()) {  // one V-cycle of every request in the batch
        vecs(active, hs, xs, bs);
        const int rc = batch_engine_step(bt, hs, xs.data(), bs.data(), true, s, nrm);
        std::vector<Request*> keep;
        for (size_t k = 0; k < active.size(); ++k) {
          Request* r = active[k];
          r->res.iters += 1;
          if (rc != FCGMG_OK) {
            retire.push_back(r);
            codes.push_back(rc);
            continue;
          }
          r->res.rel_res = nrm[k] / r->r0;
          if (!std::isfinite(nrm[k])) {
            retire.push_back(r);
            codes.push_back(set_error(FCGMG_E_NAN, "server: non-finite residual"));
          } else if (nrm[k] <= r->rtol * r->r0) {
            retire.push_back(r);
            codes.push_back(FCGMG_OK);
          } else if (r->res.iters >= sp.max_iter) {
            retire.push_back(r);
            codes.push_back(set_error(FCGMG_E_NOCONV, "server: cycle limit reached"));
          } else {
            keep.push_back(r);
          }
        }
        std::lock_guard<std::mutex> lk(mu);
        ++engine_steps;
        engine_request_cycles += (int64_t)active.size();
        engine_max_batch = std::max(engine_max_batch, (int)active.size());
        active.swap(keep);
      }
      if (!retire.empty()) {
        {
          std::lock_guard<std::mutex> lk(mu);
          for (size_t k = 0; k < retire.size(); ++k) finish_locked(retire[k], codes[k]);
        }
        cv_done.notify_all();
        cv_work.notify_all();
      }
    }
    batch_engine_destroy(bt);
    if (s) (void)hipStreamDestroy(s);
  }

  // Pick the entry for `r` under the lock: a resident idle hierarchy of the same problem, or a new
  // one admitted within the budget (evicting idle ones). Returns nullptr when `r` has to wait; sets
  // r->res.status and returns nullptr when it can never be admitted.
  Entry* admit(Request* r, std::vector<Entry*>& evict) {
    for (int k = 0; k < 3; ++k) {
      const int pol = kPolicyBySpeed[k];
      if (r->fp[pol] < 0) continue;
      fcgmg_params p = r->prm;
      p.cache_policy = pol;
      const std::string key = problem_key(p, r->balls);
      for (auto& e : entries)
        if (e->key == key) {
          if (e->busy) return nullptr;  // same problem in use: wait for it
          r->res.cache_hit = 1;
          return e.get();
        }
    }
    int64_t idle = 0;
    for (auto& e : entries)
      if (!e->busy) idle += e->bytes;
    bool any_could_fit = false;
    for (int k = 0; k < 3; ++k) {
      const int pol = kPolicyBySpeed[k];
      if (r->fp[pol] < 0) continue;
      int64_t ndof = 1;
      for (int d = 0; d < r->prm.dim; ++d) ndof *= r->prm.n_cells + 1;
      ndof *= r->prm.dim + 1;
      const int64_t need = r->fp[pol] + ndof * (int64_t)sizeof(double);
      if (need <= sp.hbm_budget) any_could_fit = true;
      if (in_use - idle + need > sp.hbm_budget) continue;  // does not fit even with every idle one evicted
      // evict idle entries, least recently used first, until `need` fits
      std::vector<Entry*> idle_lru;
      for (auto& e : entries)
        if (!e->busy) idle_lru.push_back(e.get());
      std::sort(idle_lru.begin(), idle_lru.end(), [](Entry* a, Entry* b) { return a->last_use < b->last_use; });
      size_t i = 0;
      while (in_use + need > sp.hbm_budget && i < idle_lru.size()) {
        Entry* v = idle_lru[i++];
        in_use -= v->bytes;
        evict.push_back(v);
        auto it = std::find_if(entries.begin(), entries.end(), [&](const std::unique_ptr<Entry>& u) {
          return u.get() == v;
        });
        it->release();  // deleted by the worker, outside the lock
        entries.erase(it);
      }
      auto e = std::make_unique<Entry>();
      fcgmg_params p = r->prm;
      p.cache_policy = pol;
      e->key = problem_key(p, r->balls);
      e->bytes = need;
      e->ndof = ndof;
      e->policy = pol;
      in_use += need;
      Entry* ep = e.get();
      entries.push_back(std::move(e));
      r->res.policy = pol;
      return ep;
    }
    if (!any_could_fit) r->res.status = FCGMG_E_NOMEM;
    return nullptr;
  }

  void worker_loop() {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    for (;;) {
      Request* r = nullptr;
      Entry* e = nullptr;
      std::vector<Entry*> evict;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          for (auto it = pending.begin(); it != pending.end(); ++it) {
            Entry* got = admit(*it, evict);
            if (got || (*it)->res.status != FCGMG_OK) {
              r = *it;
              e = got;
              pending.erase(it);
              break;
            }
          }
          if (r || (stop && pending.empty())) break;
          cv_work.wait(lk);
        }
        if (!r) break;
        if (e) {
          e->busy = true;
          e->last_use = ++tick;
          r->res.policy = e->policy;
        }
      }
      for (Entry* v : evict) {  // outside the lock: frees device memory
        if (v->b) (void)hipFree(v->b);
        if (v->h) fcgmg_destroy(v->h);
        delete v;
      }
      r->t_start = Clock::now();
      int rc = r->res.status;
      if (e && rc == FCGMG_OK) {
        if (!e->ready) {
          fcgmg_params p = r->prm;
          p.cache_policy = r->res.policy;
          rc = fcgmg_setup_hierarchy(&p, r->balls.data(), (int)r->balls.size() / 4, s, &e->h);
          if (rc == FCGMG_OK && hipMalloc((void**)&e->b, e->ndof * sizeof(double)) != hipSuccess)
            rc = set_error(FCGMG_E_NOMEM, "server: right-hand side allocation failed");
          if (rc == FCGMG_OK) rc = fcgmg_rhs(e->h, r->prm.n_levels - 1, e->b, s);
          if (rc == FCGMG_OK) e->ready = true;
        }
        if (rc == FCGMG_OK && hipMemsetAsync(r->x, 0, e->ndof * sizeof(double), s) != hipSuccess)
          rc = set_error(FCGMG_E_HIP, "server: clearing x failed");
        fcgmg_params pr = r->prm;
        pr.cache_policy = e->policy;
        if (rc == FCGMG_OK && sp.continuous_batching && batch_engine_accepts(pr)) {
          // set-up, right-hand side and x = 0 complete before the engine's stream reads them
          if (hipStreamSynchronize(s) != hipSuccess) {
            rc = set_error(FCGMG_E_HIP, "server: stream synchronisation failed");
          } else {
            r->t_setup_done = Clock::now();
            r->res.footprint = e->bytes;
            r->entry = e;
            {
              std::lock_guard<std::mutex> lk(mu);
              joining.push_back(r);
            }
            cv_engine.notify_one();
            continue;  // the engine completes it
          }
        }
        r->t_setup_done = Clock::now();
        if (rc == FCGMG_OK)
          rc = fcgmg_solve(e->h, r->x, e->b, r->rtol, sp.max_iter, &r->res.iters, &r->res.rel_res, nullptr, s);
        if (hipStreamSynchronize(s) != hipSuccess && rc == FCGMG_OK)
          rc = set_error(FCGMG_E_HIP, "server: stream synchronisation failed");
        r->res.footprint = e->bytes;
      } else {
        r->t_setup_done = r->t_start;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        r->entry = e;
        finish_locked(r, rc);
        if (e) {
          if (!e->ready) {  // failed set-up: give its reservation back
            in_use -= e->bytes;
            if (e->h) fcgmg_destroy(e->h);
            if (e->b) (void)hipFree(e->b);
            entries.erase(std::find_if(entries.begin(), entries.end(),
                                       [&](const std::unique_ptr<Entry>& u) { return u.get() == e; }));
          }
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" {

int fcgmg_server_create(const fcgmg_server_params* sp, fcgmg_server_h* out) {
  if (!sp || !out) return set_error(FCGMG_E_ARG, "null argument");
  *out = nullptr;
  if (sp->workers < 1 || sp->workers > 16) return set_error(FCGMG_E_ARG, "workers must be in [1,16]");
  if (sp->hbm_budget < 0 || sp->max_iter < 1) return set_error(FCGMG_E_ARG, "bad budget or max_iter");
  auto* srv = new fcgmg_server();
  srv->sp = *sp;
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return set_error(FCGMG_E_HIP, "no current device");
  }
  if (srv->sp.hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete srv;
      return set_error(FCGMG_E_HIP, "hipMemGetInfo failed");
    }
    srv->sp.hbm_budget = (int64_t)(0.8 * (double)free_b);
  }
  if (sp->continuous_batching != 0 && sp->continuous_batching != 1) {
    delete srv;
    return set_error(FCGMG_E_ARG, "continuous_batching must be 0 or 1");
  }
  for (int i = 0; i < sp->workers; ++i) srv->workers.emplace_back([srv] { srv->worker_loop(); });
  if (sp->continuous_batching) srv->engine = std::thread([srv] { srv->engine_loop(); });
  *out = srv;
  return FCGMG_OK;
}

int fcgmg_server_submit(fcgmg_server_h srv, const fcgmg_params* prm, const double* balls, int n_balls, double rtol,
                        double* x_out, int64_t* request_id) {
  if (!srv || !prm || !x_out || !request_id || !(rtol > 0)) return set_error(FCGMG_E_ARG, "bad argument");
  auto r = std::make_unique<Request>();
  r->t_submit = Clock::now();  // latency counts from the call, footprint planning included
  r->prm = *prm;
  r->balls.assign(balls, balls + 4 * (size_t)std::max(n_balls, 0));
  r->rtol = rtol;
  r->x = x_out;
  // footprints of the candidate policies, computed here (host only) so that admission is cheap;
  // a problem seen before takes its footprints from the server's table
  bool any = false;
  for (int pol = 0; pol < 3; ++pol) {
    if (prm->cache_policy >= 0 && pol != prm->cache_policy) continue;
    if (prm->precision == FCGMG_PREC_MIXED && pol != FCGMG_CACHE_INVERSE) continue;
    fcgmg_params p = *prm;
    p.cache_policy = pol;
    const std::string key = problem_key(p, r->balls);
    int64_t known = -1;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      const auto it = srv->footprints.find(key);
      if (it != srv->footprints.end()) known = it->second;
    }
    if (known < 0) {
      size_t fp = 0;
      const int rc = fcgmg_footprint_bytes(&p, r->balls.data(), n_balls, &fp);
      if (rc != FCGMG_OK) return rc;
      known = (int64_t)fp;
      std::lock_guard<std::mutex> lk(srv->mu);
      if (srv->footprints.size() >= fcgmg_server::kFootprintTable) srv->footprints.clear();
      srv->footprints[key] = known;
    }
    r->fp[pol] = known;
    any = true;
  }
  if (!any) return set_error(FCGMG_E_ARG, "no cache policy applies to this request");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->id = srv->next_id++;
    *request_id = r->id;
    srv->pending.push_back(r.get());
    srv->reqs[r->id] = std::move(r);
  }
  srv->cv_work.notify_one();
  return FCGMG_OK;
}

int fcgmg_server_wait(fcgmg_server_h srv, int64_t request_id, fcgmg_request_result* res) {
  if (!srv || !res) return set_error(FCGMG_E_ARG, "bad argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(request_id);
  if (it == srv->reqs.end()) return set_error(FCGMG_E_ARG, "unknown request id");
  Request* r = it->second.get();
  srv->cv_done.wait(lk, [&] { return r->done; });
  *res = r->res;
  srv->reqs.erase(it);
  return FCGMG_OK;
}

int fcgmg_server_resident_bytes(fcgmg_server_h srv, int64_t* bytes, int* hierarchies) {
  if (!srv || !bytes || !hierarchies) return set_error(FCGMG_E_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *bytes = srv->in_use;
  *hierarchies = (int)srv->entries.size();
  return FCGMG_OK;
}

int fcgmg_server_stats(fcgmg_server_h srv, int64_t* steps, int64_t* request_cycles, int* max_batch) {
  if (!srv || !steps || !request_cycles || !max_batch) return set_error(FCGMG_E_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *steps = srv->engine_steps;
  *request_cycles = srv->engine_request_cycles;
  *max_batch = srv->engine_max_batch;
  return FCGMG_OK;
}

int fcgmg_server_destroy(fcgmg_server_h srv) {
  if (!srv) return FCGMG_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  if (srv->engine.joinable()) {  // the workers have handed over every batched request
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->engine_stop = true;
    }
    srv->cv_engine.notify_all();
    srv->engine.join();
  }
  for (auto& e : srv->entries) {
    if (e->b) (void)hipFree(e->b);
    if (e->h) fcgmg_destroy(e->h);
  }
  delete srv;
  return FCGMG_OK;
}

}  // extern "C"
