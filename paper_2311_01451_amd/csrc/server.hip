// Continuous-batching solve server (rsrs_server_*).
//
// Factorizations stay resident on the device and are addressed by id.  Two
// worker threads, each with its own HIP stream (default priority), serve two
// queues:
//  * solves: the worker takes the oldest pending request and every other
//    pending request for the same factor, in arrival order, while the batch
//    stays within max_batch_cols columns; their right-hand sides are copied
//    side by side into one N x W block, one apply of the factor (eq. Ainvfact)
//    solves all of them, and the columns are copied back to each caller.
//    Requests that arrive while a batch is on the device wait for the next
//    batch, which takes everything pending (continuous batching).
//  * factorizations: a request (tree, black-box operator, s, seed, options)
//    is admitted when the device bytes it needs (samples, sampling buffers,
//    workspace and stored factor, estimated from the schedule before any
//    allocation) fit in the HBM budget next to what is resident and in
//    flight; it is then sampled and factored on the second stream, so its
//    work overlaps with solve batches on the device, and becomes resident.
//    Requests admitted together (same precision) are factored as one batch
//    of independent problems (rsrs_factor_batched), the factor-side analogue
//    of the solve batches.
// Releasing a factor returns its bytes to the budget once its in-flight
// batch is done.  Every column of a batch is computed by the same kernels,
// per column, as a solve of that request alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "impl.hpp"

namespace rsrs {
rsrs_status apply_factor(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                         int64_t ldf, double* Uout, int64_t ldu, hipStream_t st);
size_t factor_bytes_estimate(const rsrs_tree_t* th, int k, int p, int64_t s, int precision,
                             size_t* stored, bool adaptive);
}  // namespace rsrs

using namespace rsrs;

namespace {

constexpr int kMaxFactorBatch = 64;   // factor requests merged into one batched factorization

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct rsrs_server_s {
  int64_t budget = 0, max_cols = 1024;
  int device = 0;
  hipStream_t s_solve = nullptr, s_factor = nullptr;
  std::mutex mu;
  std::condition_variable cv_solve, cv_factor, cv_done;
  bool stop = false;

  struct Resident {
    rsrs_factor_t* F = nullptr;
    int64_t bytes = 0;
    int inflight = 0;
    bool release_pending = false;
    // refinement of served solves through the operator (mv null: one-shot)
    rsrs_matvec_fn mv = nullptr;
    void* user = nullptr;
    double tol = 0.0;
    int maxit = 0;
  };
  struct Solve {
    int64_t ticket, fid, w;
    const double* F;
    int64_t ldf;
    double* U;
    int64_t ldu;
  };
  struct Fact {
    int64_t ticket;
    const rsrs_tree_t* t;
    rsrs_matvec_fn mv;
    void* user;
    int64_t s;
    uint64_t seed;
    int dtype;
    rsrs_factor_opts o;
    int64_t est;
  };
  struct Ticket {
    int kind = 0;   // 0 solve, 1 factor
    bool done = false;
    rsrs_status st = RSRS_OK;
    std::string msg;
    int64_t result = -1;
    double t_sub = 0.0, t_done = 0.0;
  };
  std::map<int64_t, Resident> res;
  std::deque<Solve> qs;
  std::deque<Fact> qf;
  std::map<int64_t, Ticket> tickets;
  int64_t next_fid = 1, next_ticket = 1;
  int64_t in_use = 0, peak = 0;
  std::vector<double> lat_solve, lat_factor;
  int64_t batches = 0, cols_done = 0, solves_done = 0, factors_done = 0;
  int64_t refined_batches = 0, refine_steps = 0;
  double max_relres = 0.0;
  DevBuf Fb, Ub;
  int64_t batch_bytes = 0;   // Fb + Ub as charged to the budget
  std::thread th_solve, th_factor;

  void use(int64_t d) {
    in_use += d;
    peak = std::max(peak, in_use);
  }
  // Device bytes a resident factor holds while served: the stored factor and
  // its permutation, the solve graphs of every width bucket a batch of up to
  // max_cols columns can use (two tree-ordered blocks of n x bucket elements
  // each, in the factor's type) and, beyond the graph widths, the direct
  // path's two blocks of n x max_cols.
  int64_t resident_bytes(const rsrs_factor_t* F) const {
    const int64_t n = F->n, e = F->esz;
    int64_t plans = 0;
    for (int64_t b = 16; b <= 1024; b *= 2) {
      plans += 2 * n * b * e;
      if (b >= max_cols) break;
    }
    const int64_t direct = max_cols > 1024 ? 2 * n * max_cols * e : 0;
    return F->stored_values * e + n * 8 + plans + direct;
  }
  void free_resident(std::map<int64_t, Resident>::iterator it) {
    delete it->second.F;
    use(-it->second.bytes);
    res.erase(it);
    cv_factor.notify_all();
  }
  void finish(int64_t ticket, rsrs_status st, const std::string& msg, int64_t result, double t) {
    Ticket& k = tickets[ticket];
    k.done = true;
    k.st = st;
    k.msg = msg;
    k.result = result;
    k.t_done = t;
    if (k.kind == 0) {
      lat_solve.push_back(t - k.t_sub);
      ++solves_done;
    } else {
      lat_factor.push_back(t - k.t_sub);
      ++factors_done;
    }
  }

  void solve_loop() {
    (void)hipSetDevice(device);
    for (;;) {
      std::unique_lock<std::mutex> lk(mu);
      cv_solve.wait(lk, [&] { return stop || !qs.empty(); });
      if (qs.empty()) break;   // stop requested and nothing pending
      // the oldest request's factor, then every pending request for it that fits
      const int64_t fid = qs.front().fid;
      std::vector<Solve> batch;
      int64_t W = 0;
      for (auto it = qs.begin(); it != qs.end();) {
        if (it->fid == fid && (batch.empty() || W + it->w <= max_cols)) {
          W += it->w;
          batch.push_back(*it);
          it = qs.erase(it);
        } else {
          ++it;
        }
      }
      auto rit = res.find(fid);
      if (rit == res.end() || rit->second.release_pending) {
        const double t = now_ms();
        for (const auto& r : batch) finish(r.ticket, RSRS_E_INVALID, "unknown or released factor", -1, t);
        cv_done.notify_all();
        continue;
      }
      Resident& R = rit->second;
      ++R.inflight;
      const rsrs_factor_t* F = R.F;
      const rsrs_matvec_fn rmv = R.mv;
      void* ruser = R.user;
      const double rtol = R.tol;
      const int rmaxit = R.maxit;
      lk.unlock();

      const int64_t n = F->n;
      rsrs_status st = Fb.alloc((size_t)n * W * 8);
      if (st == RSRS_OK) st = Ub.alloc((size_t)n * W * 8);
      {
        // the FP64 batch blocks count against the budget at their size
        std::lock_guard<std::mutex> g(mu);
        const int64_t now = (int64_t)(Fb.bytes + Ub.bytes);
        use(now - batch_bytes);
        batch_bytes = now;
      }
      std::string msg;
      double relres = -1.0;
      int iters = 0;
      if (st == RSRS_OK) {
        int64_t c0 = 0;
        for (const auto& r : batch) {
          if (hipMemcpy2DAsync(Fb.as<double>() + c0, (size_t)W * 8, r.F, (size_t)r.ldf * 8,
                               (size_t)r.w * 8, (size_t)n, hipMemcpyDeviceToDevice, s_solve) != hipSuccess)
            st = RSRS_E_HIP;
          c0 += r.w;
        }
      }
      if (st == RSRS_OK) {
        if (rmv)   // refined to the factor's tolerance through the black-box residual
          st = rsrs_solve_refine(F, rmv, ruser, W, Fb.as<double>(), W, Ub.as<double>(), W, rtol, rmaxit, &relres,
                                 &iters, s_solve);
        else
          st = apply_factor(F, 0, 0, W, Fb.as<double>(), W, Ub.as<double>(), W, s_solve);
      }
      if (st == RSRS_OK) {
        int64_t c0 = 0;
        for (const auto& r : batch) {
          if (hipMemcpy2DAsync(r.U, (size_t)r.ldu * 8, Ub.as<double>() + c0, (size_t)W * 8,
                               (size_t)r.w * 8, (size_t)n, hipMemcpyDeviceToDevice, s_solve) != hipSuccess)
            st = RSRS_E_HIP;
          c0 += r.w;
        }
      }
      if (hipStreamSynchronize(s_solve) != hipSuccess && st == RSRS_OK) st = RSRS_E_HIP;
      if (st != RSRS_OK) msg = rsrs_last_error();
      const double t = now_ms();

      lk.lock();
      for (const auto& r : batch) finish(r.ticket, st, msg, -1, t);
      ++batches;
      cols_done += W;
      if (rmv && st == RSRS_OK) {
        ++refined_batches;
        refine_steps += iters;
        max_relres = std::max(max_relres, relres);
      }
      auto it2 = res.find(fid);
      if (it2 != res.end()) {
        --it2->second.inflight;
        if (it2->second.release_pending && it2->second.inflight == 0) free_resident(it2);
      }
      cv_done.notify_all();
    }
  }

  void factor_loop() {
    (void)hipSetDevice(device);
    for (;;) {
      std::unique_lock<std::mutex> lk(mu);
      // device memory the scratch pool keeps from earlier factorizations
      // counts too; it is trimmed when a request would not fit otherwise
      auto admissible = [&] {
        if (budget <= 0) return true;
        const int64_t need = in_use + qf.front().est;
        if (need > budget) return false;
        int64_t cached = (int64_t)pool_cached_device_bytes(device);
        if (need + cached > budget) {
          pool_trim_device(device, (size_t)(budget - need));
          cached = (int64_t)pool_cached_device_bytes(device);
        }
        return need + cached <= budget;
      };
      cv_factor.wait(lk, [&] { return stop || (!qf.empty() && admissible()); });
      if (qf.empty()) break;
      if (!admissible()) {   // shutting down with requests that never fit
        const double t = now_ms();
        while (!qf.empty()) {
          finish(qf.front().ticket, RSRS_E_NOMEM, "server shut down before the request fit the budget", -1, t);
          qf.pop_front();
        }
        cv_done.notify_all();
        break;
      }
      // every queued request that fits next to it (same precision, in order)
      std::vector<Fact> group;
      int64_t charged = 0;
      while (!qf.empty() && (int)group.size() < kMaxFactorBatch &&
             qf.front().o.precision == (group.empty() ? qf.front().o.precision : group[0].o.precision) &&
             (budget <= 0 || in_use + charged + qf.front().est <= budget)) {
        group.push_back(qf.front());
        charged += qf.front().est;
        qf.pop_front();
      }
      use(charged);
      lk.unlock();

      std::vector<rsrs_factor_t*> Fs(group.size(), nullptr);
      std::vector<rsrs_status> sts(group.size(), RSRS_OK);
      std::vector<std::string> msgs(group.size());
      run_group(group, Fs, sts, msgs);
      const double t = now_ms();

      lk.lock();
      use(-charged);
      for (size_t i = 0; i < group.size(); ++i) {
        int64_t fid = -1;
        if (sts[i] == RSRS_OK) {
          rsrs_factor_t* F = Fs[i];
          const int64_t bytes = resident_bytes(F);
          fid = next_fid++;
          res[fid] = Resident{F, bytes, 0, false};
          use(bytes);
        }
        finish(group[i].ticket, sts[i], msgs[i], fid, t);
      }
      cv_done.notify_all();
      cv_factor.notify_all();
    }
  }

  // Samples every request of the group and factors them together
  // (rsrs_factor_batched).  If the batch fails, each request is sampled and
  // factored again on its own, so only the request at fault reports the error.
  void run_group(const std::vector<Fact>& group, std::vector<rsrs_factor_t*>& Fs,
                 std::vector<rsrs_status>& sts, std::vector<std::string>& msgs) {
    const size_t m = group.size();
    std::vector<rsrs_samples_t*> smp(m, nullptr);
    std::vector<const rsrs_tree_t*> trees;
    std::vector<rsrs_samples_t*> ok_smp;
    std::vector<rsrs_factor_opts> opts;
    std::vector<size_t> idx;
    for (size_t i = 0; i < m; ++i) {
      const Fact& r = group[i];
      sts[i] = (r.o.symmetric ? rsrs_sample_symmetric : rsrs_sample)(r.t, r.mv, r.user, r.s, r.seed, r.dtype, s_factor, &smp[i]);
      if (sts[i] != RSRS_OK) {
        msgs[i] = rsrs_last_error();
        continue;
      }
      trees.push_back(r.t);
      ok_smp.push_back(smp[i]);
      opts.push_back(r.o);
      idx.push_back(i);
    }
    if (!idx.empty()) {
      std::vector<rsrs_factor_t*> out(idx.size(), nullptr);
      const rsrs_status st = factor_batch_impl((int64_t)idx.size(), trees.data(), ok_smp.data(), opts.data(),
                                               s_factor, out.data());
      if (st == RSRS_OK) {
        for (size_t j = 0; j < idx.size(); ++j) Fs[idx[j]] = out[j];
      } else if (idx.size() == 1) {
        sts[idx[0]] = st;
        msgs[idx[0]] = rsrs_last_error();
      } else {
        for (size_t j : idx) {
          const Fact& r = group[j];
          rsrs_samples_destroy(smp[j]);
          smp[j] = nullptr;
          sts[j] = (r.o.symmetric ? rsrs_sample_symmetric : rsrs_sample)(r.t, r.mv, r.user, r.s, r.seed, r.dtype, s_factor, &smp[j]);
          if (sts[j] == RSRS_OK) sts[j] = factor_impl(r.t, smp[j], &r.o, s_factor, &Fs[j]);
          if (sts[j] != RSRS_OK) msgs[j] = rsrs_last_error();
        }
      }
    }
    for (auto* x : smp) rsrs_samples_destroy(x);
  }
};

extern "C" {

rsrs_status rsrs_server_create(const rsrs_server_opts* o, rsrs_server_t** out) {
  if (!o || !out || o->max_batch_cols < 1 || o->hbm_budget < 0) {
    set_error("bad server options");
    return RSRS_E_INVALID;
  }
  *out = nullptr;
  auto sv = new rsrs_server_t();
  sv->budget = o->hbm_budget;
  sv->max_cols = o->max_batch_cols;
  if (hipGetDevice(&sv->device) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->s_solve, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->s_factor, hipStreamNonBlocking) != hipSuccess) {
    if (sv->s_solve) (void)hipStreamDestroy(sv->s_solve);
    delete sv;
    set_error("could not create the server streams");
    return RSRS_E_HIP;
  }
  sv->th_solve = std::thread([sv] { sv->solve_loop(); });
  sv->th_factor = std::thread([sv] { sv->factor_loop(); });
  *out = sv;
  return RSRS_OK;
}

void rsrs_server_destroy(rsrs_server_t* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_solve.notify_all();
  sv->cv_factor.notify_all();
  sv->th_solve.join();
  sv->th_factor.join();
  for (auto& kv : sv->res) delete kv.second.F;
  sv->res.clear();
  sv->Fb.release();
  sv->Ub.release();
  (void)hipStreamDestroy(sv->s_solve);
  (void)hipStreamDestroy(sv->s_factor);
  delete sv;
}

rsrs_status rsrs_server_add_factor(rsrs_server_t* sv, rsrs_factor_t* f, int64_t* id) {
  if (!sv || !f || !id) {
    set_error("null argument");
    return RSRS_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  const int64_t bytes = sv->resident_bytes(f);
  if (sv->budget > 0 && sv->in_use + bytes > sv->budget) {
    set_error("factor does not fit in the HBM budget");
    return RSRS_E_NOMEM;
  }
  *id = sv->next_fid++;
  sv->res[*id] = rsrs_server_s::Resident{f, bytes, 0, false};
  sv->use(bytes);
  return RSRS_OK;
}

rsrs_status rsrs_server_set_refine(rsrs_server_t* sv, int64_t id, rsrs_matvec_fn mv, void* user, double tol,
                                   int maxit) {
  if (!sv || (mv && (!(tol > 0.0) || maxit < 0))) {
    set_error("bad refinement settings");
    return RSRS_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->res.find(id);
  if (it == sv->res.end() || it->second.release_pending) {
    set_error("unknown factor id");
    return RSRS_E_INVALID;
  }
  it->second.mv = mv;
  it->second.user = user;
  it->second.tol = tol;
  it->second.maxit = maxit;
  return RSRS_OK;
}

rsrs_status rsrs_server_release_factor(rsrs_server_t* sv, int64_t id) {
  if (!sv) {
    set_error("null server");
    return RSRS_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->res.find(id);
  if (it == sv->res.end() || it->second.release_pending) {
    set_error("unknown factor id");
    return RSRS_E_INVALID;
  }
  if (it->second.inflight > 0) it->second.release_pending = true;
  else sv->free_resident(it);
  return RSRS_OK;
}

rsrs_status rsrs_server_submit_solve(rsrs_server_t* sv, int64_t id, int64_t nrhs, const double* F,
                                     int64_t ldf, double* U, int64_t ldu, int64_t* ticket) {
  if (!sv || !F || !U || !ticket || nrhs < 1 || ldf < nrhs || ldu < nrhs) {
    set_error("bad solve request");
    return RSRS_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->res.find(id);
  if (it == sv->res.end() || it->second.release_pending) {
    set_error("unknown factor id");
    return RSRS_E_INVALID;
  }
  const int64_t t = sv->next_ticket++;
  rsrs_server_s::Ticket k;
  k.kind = 0;
  k.t_sub = now_ms();
  sv->tickets[t] = k;
  sv->qs.push_back(rsrs_server_s::Solve{t, id, nrhs, F, ldf, U, ldu});
  *ticket = t;
  sv->cv_solve.notify_one();
  return RSRS_OK;
}

rsrs_status rsrs_server_submit_factor(rsrs_server_t* sv, const rsrs_tree_t* t, rsrs_matvec_fn mv,
                                      void* user, int64_t s, uint64_t seed, int dtype,
                                      const rsrs_factor_opts* o, int64_t* ticket) {
  if (!sv || !t || !mv || !o || !ticket || s < 1 || o->k < 1) {
    set_error("bad factor request");
    return RSRS_E_INVALID;
  }
  if ((o->precision == RSRS_PREC_F64) != (dtype == RSRS_F64)) {
    set_error("sample dtype does not match the precision");
    return RSRS_E_INVALID;
  }
  const int64_t need = rsrs_samples_required(t, o->k, o->p < 0 ? o->k : o->p);
  if (s < need) {
    set_required_s(need);
    set_error("s = " + std::to_string(s) + " is below the required " + std::to_string(need));
    return RSRS_E_SAMPLES;
  }
  const int64_t esz = dtype == RSRS_F64 ? 8 : 4;
  const int64_t n = t->t.n;
  const int64_t est = 6 * n * round_up(s, 16) * esz + 8 * n +
                      (int64_t)factor_bytes_estimate(t, o->k, o->p, s, o->precision, nullptr, o->rank_tol > 0.0);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->budget > 0 && est > sv->budget) {
    set_error("factorization needs " + std::to_string(est) + " bytes, more than the HBM budget");
    return RSRS_E_NOMEM;
  }
  const int64_t tk = sv->next_ticket++;
  rsrs_server_s::Ticket k;
  k.kind = 1;
  k.t_sub = now_ms();
  sv->tickets[tk] = k;
  sv->qf.push_back(rsrs_server_s::Fact{tk, t, mv, user, s, seed, dtype, *o, est});
  *ticket = tk;
  sv->cv_factor.notify_one();
  return RSRS_OK;
}

rsrs_status rsrs_server_wait(rsrs_server_t* sv, int64_t ticket, double timeout_ms, int64_t* result,
                             double* latency_ms) {
  if (!sv) {
    set_error("null server");
    return RSRS_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) {
    set_error("unknown ticket");
    return RSRS_E_INVALID;
  }
  auto ready = [&] { return sv->tickets[ticket].done; };
  if (timeout_ms < 0) {
    sv->cv_done.wait(lk, ready);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready)) {
    set_error("timed out");
    return RSRS_E_TIMEOUT;
  }
  const rsrs_server_s::Ticket k = sv->tickets[ticket];
  sv->tickets.erase(ticket);
  if (result) *result = k.result;
  if (latency_ms) *latency_ms = k.t_done - k.t_sub;
  if (k.st != RSRS_OK) set_error(k.msg);
  return k.st;
}

rsrs_status rsrs_server_get_stats(rsrs_server_t* sv, int reset, rsrs_server_stats* out) {
  if (!sv || !out) {
    set_error("null argument");
    return RSRS_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  out->solves_done = sv->solves_done;
  out->factors_done = sv->factors_done;
  out->batches = sv->batches;
  out->cols_done = sv->cols_done;
  out->hbm_in_use = sv->in_use;
  out->hbm_peak = sv->peak;
  out->resident_factors = (int64_t)sv->res.size();
  out->queued_solves = (int64_t)sv->qs.size();
  out->queued_factors = (int64_t)sv->qf.size();
  out->solve_p50_ms = percentile(sv->lat_solve, 0.50);
  out->solve_p99_ms = percentile(sv->lat_solve, 0.99);
  out->factor_p50_ms = percentile(sv->lat_factor, 0.50);
  out->refined_batches = sv->refined_batches;
  out->refine_steps = sv->refine_steps;
  out->max_relres = sv->max_relres;
  out->factor_p99_ms = percentile(sv->lat_factor, 0.99);
  if (reset) {
    sv->solves_done = sv->factors_done = sv->batches = sv->cols_done = 0;
    sv->refined_batches = sv->refine_steps = 0;
    sv->max_relres = 0.0;
    sv->lat_solve.clear();
    sv->lat_factor.clear();
    sv->peak = sv->in_use;
  }
  return RSRS_OK;
}

}  // extern "C"
