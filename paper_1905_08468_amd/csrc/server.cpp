// Serving: continuous batching of independent MUFFIN / ADA-PT solves on one
// GPU (the request loop of the C ABI's muffin_server_*).
//
// A worker thread owns a pool of handles.  Requests wait in a FIFO queue and
// are admitted as soon as a slot and their workspace fit; each admitted
// solve iterates in chunks on a stream of its own (chunks end with the
// asynchronous stopping-rule check when the request has one), so the chunks
// of different solves overlap on the device while the worker polls their
// completion events.  A finished solve returns its handle to the pool, idle
// for reuse by a request of the same configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "muffin.h"
#include "internal.hpp"

namespace muffin {
int handle_run_chunk(muffin_handle* h, int iters, bool check);
int handle_chunk_poll(muffin_handle* h, int* done, double* rel);
size_t handle_workspace_bytes(const muffin_config* c);
}  // namespace muffin

namespace {

using Clock = std::chrono::steady_clock;

bool same_config(const muffin_config& a, const muffin_config& b) {
  return a.n == b.n && a.L == b.L && a.n_bases == b.n_bases && a.levels == b.levels &&
         a.mode == b.mode && a.mu == b.mu && a.gamma == b.gamma && a.sigma == b.sigma &&
         a.tau == b.tau && a.tau_rule == b.tau_rule && a.rho == b.rho && a.eps_w == b.eps_w &&
         a.sure == b.sure && a.delta_period == b.delta_period && a.eta_mu == b.eta_mu &&
         a.eta_gamma == b.eta_gamma && a.eps_fd == b.eps_fd && a.sigma_w == b.sigma_w &&
         a.deriv_reset == b.deriv_reset && a.pi_iters == b.pi_iters && a.pi_tol == b.pi_tol &&
         a.stop_rel == b.stop_rel && a.check_every == b.check_every &&
         a.dictionary == b.dictionary && a.visibilities == b.visibilities &&
         a.vis_norm2 == b.vis_norm2 && a.vis_count == b.vis_count;
}

struct Request {
  int64_t ticket = 0;
  muffin_config cfg{};
  const void* dirty = nullptr;
  const void* psf = nullptr;
  const void* delta = nullptr;
  std::vector<double> alpha, beta;
  int32_t max_iters = 0;
  void* sky_out = nullptr;
  size_t bytes = 0;
  int32_t status = MUFFIN_REQ_QUEUED;  // or a negative error code
  bool cancel = false;
  muffin_report rep{};
  Clock::time_point t_submit, t_done;
};

struct PoolEntry {
  muffin_config cfg{};
  muffin_handle* h = nullptr;
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  bool busy = false;
  Clock::time_point last;
};

struct Slot {
  PoolEntry* pe = nullptr;
  Request* r = nullptr;
  int done_iters = 0;
  int chunk_iters = 0;
  bool inflight = false;
};

}  // namespace

struct muffin_server {
  muffin_server_config sc{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_ticket = 1;
  std::vector<std::unique_ptr<PoolEntry>> pool;
  std::vector<Slot> active;  // touched by the worker only
  size_t bytes_in_use = 0;
  int32_t n_active = 0, completed = 0, failed = 0, cancelled = 0;
  bool stop = false;
  std::thread worker;

  void finish(Slot& sl, int32_t status) {
    Request* r = sl.r;
    if (status == MUFFIN_REQ_DONE) {
      int rc = muffin_get_sky(sl.pe->h, r->sky_out);
      if (!rc) rc = muffin_get_report(sl.pe->h, &r->rep);  // synchronises this stream
      if (rc) status = rc;
    }
    std::lock_guard<std::mutex> g(mu);
    r->status = status;
    r->t_done = Clock::now();
    if (status == MUFFIN_REQ_DONE) ++completed;
    else if (status == MUFFIN_REQ_CANCELLED) ++cancelled;
    else ++failed;
    sl.pe->busy = false;
    sl.pe->last = r->t_done;
    --n_active;
    cv_done.notify_all();
  }

  // Releases the least recently used idle handle; false if there is none.
  bool evict_one() {
    int best = -1;
    for (int i = 0; i < (int)pool.size(); ++i)
      if (!pool[i]->busy && (best < 0 || pool[i]->last < pool[best]->last)) best = i;
    if (best < 0) return false;
    PoolEntry* pe = pool[best].get();
    muffin_destroy(pe->h);
    (void)hipStreamDestroy(pe->stream);
    bytes_in_use -= pe->bytes;
    pool.erase(pool.begin() + best);
    return true;
  }

  // Under the lock: moves admissible requests from the queue head to `out`.
  void admit(std::vector<std::pair<Request*, PoolEntry*>>& out) {
    while (!queue.empty() && n_active + (int)out.size() < sc.max_active) {
      Request* r = queue.front();
      if (r->cancel) {
        queue.pop_front();
        r->status = MUFFIN_REQ_CANCELLED;
        r->t_done = Clock::now();
        ++cancelled;
        cv_done.notify_all();
        continue;
      }
      PoolEntry* pe = nullptr;
      for (auto& e : pool)
        if (!e->busy && same_config(e->cfg, r->cfg)) {
          pe = e.get();
          break;
        }
      if (!pe) {
        while (bytes_in_use + r->bytes > sc.hbm_budget && evict_one()) {
        }
        if (bytes_in_use + r->bytes > sc.hbm_budget) break;  // wait for memory
        std::unique_ptr<PoolEntry> e(new PoolEntry());
        e->cfg = r->cfg;
        e->bytes = r->bytes;
        int rc = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) == hipSuccess
                     ? MUFFIN_OK
                     : MUFFIN_E_HIP;
        if (!rc) rc = muffin_create(&e->h, &r->cfg, e->stream);
        if (rc) {
          if (e->stream) (void)hipStreamDestroy(e->stream);
          queue.pop_front();
          r->status = rc;
          r->t_done = Clock::now();
          ++failed;
          cv_done.notify_all();
          continue;
        }
        bytes_in_use += e->bytes;
        pe = e.get();
        pool.push_back(std::move(e));
      }
      pe->busy = true;
      queue.pop_front();
      out.push_back({r, pe});
    }
  }

  void loop() {
    (void)hipSetDevice(device);
    for (;;) {
      std::vector<std::pair<Request*, PoolEntry*>> adm;
      {
        std::lock_guard<std::mutex> g(mu);
        if (stop && queue.empty() && active.empty()) break;
        admit(adm);
        n_active += (int)adm.size();
      }
      bool progress = !adm.empty();
      for (auto& ar : adm) {
        Request* r = ar.first;
        Slot sl;
        sl.pe = ar.second;
        sl.r = r;
        const double* a = r->alpha.empty() ? nullptr : r->alpha.data();
        const double* b = r->beta.empty() ? nullptr : r->beta.data();
        const int rc = muffin_set_problem(sl.pe->h, r->dirty, r->psf, a, b, r->delta);
        if (rc) {
          finish(sl, rc);
          continue;
        }
        {
          std::lock_guard<std::mutex> g(mu);
          r->status = MUFFIN_REQ_RUNNING;
        }
        active.push_back(sl);
      }
      for (size_t i = 0; i < active.size();) {
        Slot& sl = active[i];
        Request* r = sl.r;
        bool cancel;
        {
          std::lock_guard<std::mutex> g(mu);
          cancel = r->cancel;
        }
        bool remove = false;
        if (!sl.inflight) {
          if (cancel) {
            finish(sl, MUFFIN_REQ_CANCELLED);
            remove = true;
          } else {
            const bool check = r->cfg.stop_rel > 0;
            int k = check ? r->cfg.check_every : sc.chunk;
            k = std::min(k, r->max_iters - sl.done_iters);
            const int rc = muffin::handle_run_chunk(sl.pe->h, k, check);
            if (rc) {
              finish(sl, rc);
              remove = true;
            } else {
              sl.inflight = true;
              sl.chunk_iters = k;
              progress = true;
            }
          }
        } else {
          int done = 0;
          double rel = -1;
          const int rc = muffin::handle_chunk_poll(sl.pe->h, &done, &rel);
          if (rc) {
            finish(sl, rc);
            remove = true;
          } else if (done) {
            progress = true;
            sl.inflight = false;
            sl.done_iters += sl.chunk_iters;
            const bool met = r->cfg.stop_rel > 0 && rel >= 0 && rel <= r->cfg.stop_rel;
            if (met || sl.done_iters >= r->max_iters) {
              finish(sl, MUFFIN_REQ_DONE);
              remove = true;
            } else if (cancel) {
              finish(sl, MUFFIN_REQ_CANCELLED);
              remove = true;
            }
          }
        }
        if (remove)
          active.erase(active.begin() + i);
        else
          ++i;
      }
      if (!progress) {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::microseconds(active.empty() ? 2000 : 50));
      }
    }
  }
};

extern "C" {

int muffin_server_default_config(muffin_server_config* sc) {
  if (!sc) return MUFFIN_E_INVAL;
  std::memset(sc, 0, sizeof(*sc));
  sc->hbm_budget = 0;
  sc->max_active = 8;
  sc->max_queue = 4096;
  sc->chunk = 10;
  return MUFFIN_OK;
}

int muffin_server_create(muffin_server** s, const muffin_server_config* sc) {
  if (!s || !sc) return MUFFIN_E_INVAL;
  *s = nullptr;
  if (sc->max_active < 1 || sc->max_active > 64 || sc->max_queue < 1 || sc->chunk < 1)
    return MUFFIN_E_INVAL;
  std::unique_ptr<muffin_server> sv(new (std::nothrow) muffin_server());
  if (!sv) return MUFFIN_E_NOMEM;
  sv->sc = *sc;
  if (hipGetDevice(&sv->device) != hipSuccess) return MUFFIN_E_HIP;
  if (sv->sc.hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return MUFFIN_E_HIP;
    sv->sc.hbm_budget = fr / 100 * 85;
  }
  muffin_server* raw = sv.get();
  try {
    sv->worker = std::thread([raw] { raw->loop(); });
  } catch (...) {
    return MUFFIN_E_NOMEM;
  }
  *s = sv.release();
  return MUFFIN_OK;
}

int muffin_server_submit(muffin_server* s, const muffin_config* cfg, const void* dirty,
                         const void* psf, const double* alpha, const double* beta,
                         const void* delta, int32_t max_iters, void* sky_out, int64_t* ticket) {
  if (!s || !cfg || !dirty || !psf || !sky_out || !ticket || max_iters < 1)
    return MUFFIN_E_INVAL;
  const size_t need = muffin_workspace_bytes(cfg);
  if (need == 0) {
    muffin_handle* probe = nullptr;  // report the validation error itself
    const int rc = muffin_create(&probe, cfg, nullptr);
    if (probe) muffin_destroy(probe);
    return rc ? rc : MUFFIN_E_INVAL;
  }
  if (cfg->sure && !delta) return MUFFIN_E_INVAL;
  if (need > s->sc.hbm_budget) return MUFFIN_E_NOMEM;
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return MUFFIN_E_NOMEM;
  r->cfg = *cfg;
  r->dirty = dirty;
  r->psf = psf;
  r->delta = delta;
  if (alpha) r->alpha.assign(alpha, alpha + (size_t)cfg->n * cfg->n);
  if (beta) r->beta.assign(beta, beta + cfg->L);
  r->max_iters = max_iters;
  r->sky_out = sky_out;
  r->bytes = need;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return MUFFIN_E_STATE;
    if ((int)s->queue.size() >= s->sc.max_queue) return MUFFIN_E_BUSY;
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
  }
  s->cv_work.notify_one();
  return MUFFIN_OK;
}

static int fill_status(const Request* r, int32_t* status, muffin_report* report,
                       double* latency_ms) {
  if (status) *status = r->status;
  const bool ended = r->status != MUFFIN_REQ_QUEUED && r->status != MUFFIN_REQ_RUNNING;
  if (report) {
    if (ended) *report = r->rep;
    else std::memset(report, 0, sizeof(*report));
  }
  if (latency_ms)
    *latency_ms = ended ? std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count()
                        : -1.0;
  return MUFFIN_OK;
}

int muffin_server_poll(muffin_server* s, int64_t ticket, int32_t* status, muffin_report* report,
                       double* latency_ms) {
  if (!s) return MUFFIN_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return MUFFIN_E_INVAL;
  return fill_status(it->second.get(), status, report, latency_ms);
}

int muffin_server_wait(muffin_server* s, int64_t ticket, double timeout_ms, int32_t* status,
                       muffin_report* report, double* latency_ms) {
  if (!s) return MUFFIN_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return MUFFIN_E_INVAL;
  Request* r = it->second.get();
  auto ended = [r] {
    return r->status != MUFFIN_REQ_QUEUED && r->status != MUFFIN_REQ_RUNNING;
  };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, ended);
  else
    s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ended);
  return fill_status(r, status, report, latency_ms);
}

int muffin_server_cancel(muffin_server* s, int64_t ticket) {
  if (!s) return MUFFIN_E_INVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MUFFIN_E_INVAL;
    it->second->cancel = true;
  }
  s->cv_work.notify_one();
  return MUFFIN_OK;
}

int muffin_server_get_stats(muffin_server* s, muffin_server_stats* out) {
  if (!s || !out) return MUFFIN_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->queued = (int32_t)s->queue.size();
  out->active = s->n_active;
  out->completed = s->completed;
  out->failed = s->failed;
  out->cancelled = s->cancelled;
  out->pooled_handles = (int32_t)s->pool.size();
  out->bytes_in_use = s->bytes_in_use;
  out->bytes_budget = s->sc.hbm_budget;
  return MUFFIN_OK;
}

int muffin_server_destroy(muffin_server* s) {
  if (!s) return MUFFIN_E_INVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (auto& kv : s->reqs) kv.second->cancel = true;
  }
  s->cv_work.notify_one();
  if (s->worker.joinable()) s->worker.join();
  for (auto& e : s->pool) {
    muffin_destroy(e->h);
    (void)hipStreamDestroy(e->stream);
  }
  delete s;
  return MUFFIN_OK;
}

}  // extern "C"
