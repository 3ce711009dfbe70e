// Batched V-cycles over independent 2D problems (see include/fcgmg.h, fcgmg_batch_*).
//
// Each step of the V-cycle of Sec. 3 (a fused sweep, the residual + restriction, the coarsest solve)
// is one launch over every problem that takes part in it: a job table gives each workgroup its
// problem and level. Problems of different sizes and depths are aligned by their distance from
// their finest level: depth d works on level L_i - 1 - d of problem i. The problems' own cycles are
// unchanged, so each result is the one its hierarchy gives alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fcgmg_impl.h"

using namespace fcg;

namespace {

enum { kFused = 0, kRR = 1, kDense = 2, kNorm = 3 };

// One launch of a batched cycle: its jobs and workgroups in the concatenated tables.
struct LaunchRec {
  int kind;
  int job0, njobs;      // first job in the table of this kind, count
  int block0, nblocks;  // first entry in block_job, count
};

}  // namespace

struct fcgmg_batch {
  std::vector<fcgmg_ctx*> hs;
  // host tables of the current call, then copied into one device buffer
  std::vector<Fused2Job<double>> fj;
  std::vector<RR2Job<double>> rj;
  std::vector<DenseJob> dj;
  std::vector<NormJob> nj;
  std::vector<int> bj;
  std::vector<LaunchRec> launches;
  bool persistent = false;  // fused sweeps as persistent launches (fcgmg_batch_set_persistent)
  char* host_buf = nullptr;  // pinned staging
  char* dev_buf = nullptr;
  size_t buf_cap = 0;
  double* part = nullptr;  // norm partial sums
  double* norms = nullptr;
  double* norms_host = nullptr;
  int part_cap = 0;
  int norm_cap = 0;        // problems that norms / norms_host hold

  void clear() {
    fj.clear();
    rj.clear();
    dj.clear();
    nj.clear();
    bj.clear();
    launches.clear();
  }

  template <class Job>
  void add_launch(int kind, std::vector<Job>& table, const std::vector<std::pair<Job, int>>& jobs) {
    if (jobs.empty()) return;
    LaunchRec L{kind, (int)table.size(), (int)jobs.size(), (int)bj.size(), 0};
    int blk = 0;
    for (size_t j = 0; j < jobs.size(); ++j) {
      Job job = jobs[j].first;
      job.block0 = blk;
      table.push_back(job);
      for (int b = 0; b < jobs[j].second; ++b) bj.push_back((int)j);
      blk += jobs[j].second;
    }
    L.nblocks = blk;
    launches.push_back(L);
  }

  // Copy the tables into the device buffer (one transfer) and run the recorded launches. The host
  // staging buffer is reused, so the previous transfer must be complete: `synced` says the caller
  // has synchronised the stream since the last run; otherwise run waits for it first.
  int run(hipStream_t s, bool synced = false) {
    const size_t o_f = 0, o_r = o_f + fj.size() * sizeof(fj[0]), o_d = o_r + rj.size() * sizeof(rj[0]),
                 o_n = o_d + dj.size() * sizeof(dj[0]), o_b = o_n + nj.size() * sizeof(nj[0]),
                 total = o_b + bj.size() * sizeof(int);
    if (!synced && hipStreamSynchronize(s) != hipSuccess)
      return set_error(FCGMG_E_HIP, "batch: stream synchronisation failed");
    if (total > buf_cap) {
      if (host_buf) (void)hipHostFree(host_buf);
      if (dev_buf) (void)hipFree(dev_buf);
      host_buf = nullptr;
      dev_buf = nullptr;
      buf_cap = std::max(total, 2 * buf_cap);
      if (hipHostMalloc((void**)&host_buf, buf_cap, hipHostMallocDefault) != hipSuccess ||
          hipMalloc((void**)&dev_buf, buf_cap) != hipSuccess) {
        buf_cap = 0;
        return set_error(FCGMG_E_NOMEM, "batch: job table allocation failed");
      }
    }
    std::memcpy(host_buf + o_f, fj.data(), fj.size() * sizeof(fj[0]));
    std::memcpy(host_buf + o_r, rj.data(), rj.size() * sizeof(rj[0]));
    std::memcpy(host_buf + o_d, dj.data(), dj.size() * sizeof(dj[0]));
    std::memcpy(host_buf + o_n, nj.data(), nj.size() * sizeof(nj[0]));
    std::memcpy(host_buf + o_b, bj.data(), bj.size() * sizeof(int));
    if (hipMemcpyAsync(dev_buf, host_buf, total, hipMemcpyHostToDevice, s) != hipSuccess)
      return set_error(FCGMG_E_HIP, "batch: job table copy failed");
    const auto* d_f = reinterpret_cast<const Fused2Job<double>*>(dev_buf + o_f);
    const auto* d_r = reinterpret_cast<const RR2Job<double>*>(dev_buf + o_r);
    const auto* d_d = reinterpret_cast<const DenseJob*>(dev_buf + o_d);
    const auto* d_n = reinterpret_cast<const NormJob*>(dev_buf + o_n);
    const auto* d_b = reinterpret_cast<const int*>(dev_buf + o_b);
    for (const LaunchRec& L : launches) {
      hipError_t e = hipSuccess;
      if (L.kind == kFused)
        e = persistent ? k_batch_fused2_persistent(d_f + L.job0, d_b + L.block0, L.nblocks, s)
                       : k_batch_fused2(d_f + L.job0, d_b + L.block0, L.nblocks, s);
      if (L.kind == kRR) e = k_batch_rr2(d_r + L.job0, d_b + L.block0, L.nblocks, s);
      if (L.kind == kDense) e = k_batch_dense(d_d + L.job0, d_b + L.block0, L.nblocks, s);
      if (L.kind == kNorm) e = k_batch_sumsq(d_n + L.job0, L.njobs, d_b + L.block0, L.nblocks, part, norms, s);
      if (e != hipSuccess) return set_error(FCGMG_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    return FCGMG_OK;
  }

  // Record one V-cycle of the problems in `act` (x, b: their finest-level vectors).
  void record_vcycle(const std::vector<int>& act, double* const* x, const double* const* b) {
    int dmax = 0;
    for (int i : act) dmax = std::max(dmax, (int)hs[i]->lev.size() - 1);
    auto X = [&](int i, int l) -> double* {
      return l == (int)hs[i]->lev.size() - 1 ? x[i] : hs[i]->lev[l].x;
    };
    auto B = [&](int i, int l) -> const double* {
      return l == (int)hs[i]->lev.size() - 1 ? b[i] : hs[i]->lev[l].b;
    };
    auto smooth = [&](int d, int sweeps, bool post) {
      for (int pair = 0; pair < sweeps / 2; ++pair) {
        std::vector<std::pair<Fused2Job<double>, int>> a, c;
        for (int i : act) {
          const int l = (int)hs[i]->lev.size() - 1 - d;
          if (l < 1) continue;
          const Level& L = hs[i]->lev[l];
          int mode = 0;
          const double* xc = nullptr;
          if (pair == 0 && post) {
            mode = 2;
            xc = X(i, l - 1);
          } else if (pair == 0 && d > 0) {
            mode = 1;
          }
          a.push_back({batch_fused2_job(*hs[i], L, X(i, l), B(i, l), L.xalt, mode, xc), batch_fused2_blocks(L)});
          c.push_back({batch_fused2_job(*hs[i], L, L.xalt, B(i, l), X(i, l), 0, nullptr), batch_fused2_blocks(L)});
        }
        add_launch(kFused, fj, a);
        add_launch(kFused, fj, c);
      }
    };
    for (int d = 0; d < dmax; ++d) {
      smooth(d, hs[act[0]]->prm.nu_pre, false);
      std::vector<std::pair<RR2Job<double>, int>> r;
      for (int i : act) {
        const int l = (int)hs[i]->lev.size() - 1 - d;
        if (l < 1) continue;
        const Level& L = hs[i]->lev[l];
        r.push_back({batch_rr2_job(L, X(i, l), B(i, l), hs[i]->lev[l - 1].b), batch_rr2_blocks(L)});
      }
      add_launch(kRR, rj, r);
    }
    std::vector<std::pair<DenseJob, int>> dense;
    for (int i : act) {
      const Ctx& c = *hs[i];
      dense.push_back({DenseJob{c.coarse_inv, B(i, 0), X(i, 0), c.coarse_n, 0}, (c.coarse_n + 3) / 4});
    }
    add_launch(kDense, dj, dense);
    for (int d = dmax - 1; d >= 0; --d) smooth(d, hs[act[0]]->prm.nu_post, true);
  }

  void record_norms(const std::vector<int>& act, double* const* x, const double* const* b) {
    std::vector<std::pair<NormJob, int>> jobs;
    for (int i : act) {
      const Level& L = hs[i]->lev.back();
      NormJob J = batch_norm_job(L, x[i], b[i]);
      J.nblocks = batch_norm_blocks(L);
      jobs.push_back({J, J.nblocks});
    }
    add_launch(kNorm, nj, jobs);
  }

  int ensure_norm_space(int nblocks, int njobs) {
    if (njobs > norm_cap) {
      if (norms) (void)hipFree(norms);
      if (norms_host) (void)hipHostFree(norms_host);
      norms = nullptr;
      norms_host = nullptr;
      norm_cap = 0;
      const int cap = std::max(njobs, 2 * norm_cap);
      if (hipMalloc((void**)&norms, cap * sizeof(double)) != hipSuccess ||
          hipHostMalloc((void**)&norms_host, cap * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return set_error(FCGMG_E_NOMEM, "batch: norm allocation failed");
      norm_cap = cap;
    }
    if (nblocks <= part_cap) return FCGMG_OK;
    if (part) (void)hipFree(part);
    part = nullptr;
    part_cap = 0;
    if (hipMalloc((void**)&part, (size_t)nblocks * sizeof(double)) != hipSuccess)
      return set_error(FCGMG_E_NOMEM, "batch: norm partials allocation failed");
    part_cap = nblocks;
    return FCGMG_OK;
  }

  // Norms of b - L x of the problems in `act` into out (host), one synchronisation.
  int norms_of(const std::vector<int>& act, double* const* x, const double* const* b, hipStream_t s,
               std::vector<double>& out) {
    clear();
    record_norms(act, x, b);
    int rc;
    if ((rc = ensure_norm_space((int)bj.size(), (int)act.size()))) return rc;
    if ((rc = run(s))) return rc;
    if (hipMemcpyAsync(norms_host, norms, act.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(FCGMG_E_HIP, "batch: norm read-back failed");
    out.assign(norms_host, norms_host + act.size());
    for (double& v : out) v = std::sqrt(v);
    return FCGMG_OK;
  }
};

extern "C" {

int fcgmg_batch_create(const fcgmg_h* hs, int count, fcgmg_batch_h* out) {
  if (!hs || !out || count < 1) return set_error(FCGMG_E_ARG, "bad argument");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    const fcgmg_h h = hs[i];
    if (!h) return set_error(FCGMG_E_ARG, "null hierarchy in batch");
    const fcgmg_params& P = h->prm;
    if (P.dim != 2 || P.cache_policy != FCGMG_CACHE_INVERSE || P.precision != FCGMG_PREC_FP64)
      return set_error(FCGMG_E_ARG, "batch: every hierarchy must be 2D, cache_inverse, FP64");
    if (P.nu_pre < 2 || P.nu_pre % 2 || P.nu_post < 2 || P.nu_post % 2 || P.nu_pre != hs[0]->prm.nu_pre ||
        P.nu_post != hs[0]->prm.nu_post)
      return set_error(FCGMG_E_ARG, "batch: nu_pre, nu_post must be equal, even and >= 2 for all problems");
  }
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (hs[i] == hs[j]) return set_error(FCGMG_E_ARG, "batch: a hierarchy appears twice");
  auto* bt = new fcgmg_batch();
  bt->hs.assign(hs, hs + count);
  if (hipMalloc((void**)&bt->norms, count * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&bt->norms_host, count * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    fcgmg_batch_destroy(bt);
    return set_error(FCGMG_E_NOMEM, "batch: allocation failed");
  }
  bt->norm_cap = count;
  *out = bt;
  return FCGMG_OK;
}

int fcgmg_batch_vcycle(fcgmg_batch_h bt, double* const* x, const double* const* b, void* stream) {
  if (!bt || !x || !b) return set_error(FCGMG_E_ARG, "bad argument");
  std::vector<int> act(bt->hs.size());
  for (size_t i = 0; i < act.size(); ++i) act[i] = (int)i;
  bt->clear();
  bt->record_vcycle(act, x, b);
  return bt->run((hipStream_t)stream);
}

int fcgmg_batch_solve(fcgmg_batch_h bt, double* const* x, const double* const* b, double rtol, int max_iter,
                      int* iters, double* rel_res, void* stream) {
  if (!bt || !x || !b || !iters || !rel_res || max_iter < 0 || !(rtol >= 0))
    return set_error(FCGMG_E_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const int count = (int)bt->hs.size();
  std::vector<int> act;
  std::vector<double> r0, rn;
  for (int i = 0; i < count; ++i) act.push_back(i);
  int rc;
  if ((rc = bt->norms_of(act, x, b, s, r0))) return rc;
  std::vector<int> live;
  for (int i = 0; i < count; ++i) {
    iters[i] = 0;
    rel_res[i] = 0;
    if (!std::isfinite(r0[i])) return set_error(FCGMG_E_NAN, "batch: non-finite initial residual");
    if (r0[i] > 0) live.push_back(i);
  }
  for (int it = 1; it <= max_iter && !live.empty(); ++it) {
    bt->clear();
    bt->record_vcycle(live, x, b);
    if ((rc = bt->run(s))) return rc;
    if ((rc = bt->norms_of(live, x, b, s, rn))) return rc;
    std::vector<int> next;
    for (size_t k = 0; k < live.size(); ++k) {
      const int i = live[k];
      iters[i] = it;
      rel_res[i] = rn[k] / r0[i];
      if (!std::isfinite(rn[k])) return set_error(FCGMG_E_NAN, "batch: non-finite residual, problem " + std::to_string(i));
      if (rn[k] > rtol * r0[i]) next.push_back(i);
    }
    live.swap(next);
  }
  if (!live.empty())
    return set_error(FCGMG_E_NOCONV, "batch: " + std::to_string(live.size()) + " problems not converged in " +
                                         std::to_string(max_iter) + " cycles");
  return FCGMG_OK;
}

int fcgmg_batch_set_persistent(fcgmg_batch_h bt, int on) {
  if (!bt || (on != 0 && on != 1)) return set_error(FCGMG_E_ARG, "bad argument");
  bt->persistent = on == 1;
  return FCGMG_OK;
}

int fcgmg_batch_destroy(fcgmg_batch_h bt) {
  if (!bt) return FCGMG_OK;
  if (bt->host_buf) (void)hipHostFree(bt->host_buf);
  if (bt->dev_buf) (void)hipFree(bt->dev_buf);
  if (bt->part) (void)hipFree(bt->part);
  if (bt->norms) (void)hipFree(bt->norms);
  if (bt->norms_host) (void)hipHostFree(bt->norms_host);
  delete bt;
  return FCGMG_OK;
}

}  // extern "C"

namespace fcg {

bool batch_engine_accepts(const fcgmg_params& p) {
  return p.dim == 2 && p.cache_policy == FCGMG_CACHE_INVERSE && p.precision == FCGMG_PREC_FP64 &&
         p.solver == FCGMG_SOLVER_GMG && p.nu_pre == 2 && p.nu_post == 2;
}

int batch_engine_create(fcgmg_batch** out) {
  *out = new fcgmg_batch();
  return FCGMG_OK;
}

int batch_engine_step(fcgmg_batch* bt, const std::vector<fcgmg_ctx*>& hs, double* const* x, const double* const* b,
                      bool cycle, hipStream_t s, std::vector<double>& norms) {
  // the cycle and the norms in one table, one transfer and one synchronisation (the engine
  // synchronises at the end of every step, so the staging buffer is free when the next one starts)
  bt->hs = hs;
  std::vector<int> act(hs.size());
  for (size_t i = 0; i < act.size(); ++i) act[i] = (int)i;
  bt->clear();
  if (cycle) bt->record_vcycle(act, x, b);
  bt->record_norms(act, x, b);
  int rc;
  if ((rc = bt->ensure_norm_space((int)bt->bj.size(), (int)act.size()))) return rc;
  if ((rc = bt->run(s, true))) return rc;
  if (hipMemcpyAsync(bt->norms_host, bt->norms, act.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(FCGMG_E_HIP, "batch: norm read-back failed");
  norms.assign(bt->norms_host, bt->norms_host + act.size());
  for (double& v : norms) v = std::sqrt(v);
  return FCGMG_OK;
}

void batch_engine_destroy(fcgmg_batch* bt) { fcgmg_batch_destroy(bt); }

}  // namespace fcg
