// Multi-start ADA-PT: one cube solved from several initial couples
// theta^(0) = (mu, gamma) at once (the experiment of Section 4.2, which
// follows four starts to a common theta).  Each start is a handle on a
// stream of its own; all starts iterate as one muffin_batch, i.e. one graph
// launch per chunk of every start, so their kernels overlap on the device.
// The set-up of Section 2 (weights, beta_H by power iteration) is computed
// once by the first start and handed to the others.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <new>
#include <vector>

#include "muffin.h"
#include "internal.hpp"

#define RC(expr)              \
  do {                        \
    const int _rc = (expr);   \
    if (_rc) return _rc;      \
  } while (0)

namespace muffin {
void handle_preset_beta_H(muffin_handle* h, double v);
}  // namespace muffin

struct muffin_multistart {
  muffin_config cfg{};
  std::vector<muffin_handle*> hs;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> evs;  // one per start: its stream's tail
  hipStream_t root = nullptr;
  bool own_root = false;
  hipEvent_t root_ev = nullptr;
  muffin_batch* batch = nullptr;

  ~muffin_multistart() {
    if (batch) (void)muffin_batch_destroy(batch);
    for (auto* h : hs)
      if (h) (void)muffin_destroy(h);
    for (auto s : streams)
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    for (auto e : evs)
      if (e) (void)hipEventDestroy(e);
    if (root_ev) (void)hipEventDestroy(root_ev);
    if (own_root && root) {
      (void)hipStreamSynchronize(root);
      (void)hipStreamDestroy(root);
    }
  }
};

extern "C" {

int muffin_multistart_create(muffin_multistart** m, const muffin_config* cfg, int32_t starts,
                             const double* mu0, const double* gamma0, void* stream) {
  if (!m || !cfg || !mu0 || !gamma0 || starts < 1 || starts > 64) return MUFFIN_E_INVAL;
  *m = nullptr;
  for (int i = 0; i < starts; ++i)
    if (!std::isfinite(mu0[i]) || !std::isfinite(gamma0[i]) || mu0[i] < 0 || gamma0[i] < 0)
      return MUFFIN_E_INVAL;
  std::unique_ptr<muffin_multistart> ms(new (std::nothrow) muffin_multistart());
  if (!ms) return MUFFIN_E_NOMEM;
  ms->cfg = *cfg;
  if (stream) {
    ms->root = static_cast<hipStream_t>(stream);
  } else {
    MUFFIN_HIP_CHECK(hipStreamCreateWithFlags(&ms->root, hipStreamNonBlocking));
    ms->own_root = true;
  }
  MUFFIN_HIP_CHECK(hipEventCreateWithFlags(&ms->root_ev, hipEventDisableTiming));
  ms->hs.assign(starts, nullptr);
  ms->streams.assign(starts, nullptr);
  ms->evs.assign(starts, nullptr);
  for (int i = 0; i < starts; ++i) {
    MUFFIN_HIP_CHECK(hipStreamCreateWithFlags(&ms->streams[i], hipStreamNonBlocking));
    MUFFIN_HIP_CHECK(hipEventCreateWithFlags(&ms->evs[i], hipEventDisableTiming));
    muffin_config c = *cfg;
    c.mu = mu0[i];
    c.gamma = gamma0[i];
    const int rc = muffin_create(&ms->hs[i], &c, ms->streams[i]);
    if (rc) return rc;
  }
  *m = ms.release();
  return MUFFIN_OK;
}

int muffin_multistart_set_problem(muffin_multistart* m, const void* dirty, const void* psf,
                                  const double* alpha, const double* beta, const void* delta,
                                  int32_t chunk) {
  if (!m) return MUFFIN_E_INVAL;
  if (m->batch) {
    // a new problem restarts every start: the old graph is dropped
    (void)muffin_batch_destroy(m->batch);
    m->batch = nullptr;
  }
  RC(muffin_set_problem(m->hs[0], dirty, psf, alpha, beta, delta));
  const int n = m->cfg.n, L = m->cfg.L;
  std::vector<double> a((size_t)n * n), b(L);
  RC(muffin_get_weights(m->hs[0], a.data(), b.data()));
  muffin_report r{};
  RC(muffin_get_report(m->hs[0], &r));
  for (size_t i = 1; i < m->hs.size(); ++i) {
    if (r.beta_H > 0) muffin::handle_preset_beta_H(m->hs[i], r.beta_H);
    RC(muffin_set_problem(m->hs[i], dirty, psf, a.data(), b.data(), delta));
  }
  return muffin_batch_create(&m->batch, m->hs.data(), (int32_t)m->hs.size(), chunk, m->root);
}

int muffin_multistart_run(muffin_multistart* m, int32_t chunks) {
  if (!m || chunks < 0) return MUFFIN_E_INVAL;
  if (!m->batch) return MUFFIN_E_STATE;
  if (chunks == 0) return MUFFIN_OK;
  // join: the launch follows whatever was enqueued on the starts' streams
  for (size_t i = 0; i < m->hs.size(); ++i) {
    MUFFIN_HIP_CHECK(hipEventRecord(m->evs[i], m->streams[i]));
    MUFFIN_HIP_CHECK(hipStreamWaitEvent(m->root, m->evs[i], 0));
  }
  RC(muffin_batch_run(m->batch, chunks));
  // fork: later work on a start's stream (sky copies, quality) follows it
  MUFFIN_HIP_CHECK(hipEventRecord(m->root_ev, m->root));
  for (auto s : m->streams) MUFFIN_HIP_CHECK(hipStreamWaitEvent(s, m->root_ev, 0));
  return MUFFIN_OK;
}

int muffin_multistart_quality(muffin_multistart* m, const void* truth, double* snr_db,
                              double* wmse) {
  if (!m || !truth) return MUFFIN_E_INVAL;
  for (size_t i = 0; i < m->hs.size(); ++i)
    RC(muffin_quality(m->hs[i], truth, snr_db ? snr_db + i : nullptr, wmse ? wmse + i : nullptr));
  return MUFFIN_OK;
}

muffin_handle* muffin_multistart_handle(muffin_multistart* m, int32_t i) {
  if (!m || i < 0 || i >= (int32_t)m->hs.size()) return nullptr;
  return m->hs[i];
}

int muffin_multistart_destroy(muffin_multistart* m) {
  if (!m) return MUFFIN_E_INVAL;
  delete m;
  return MUFFIN_OK;
}

}  // extern "C"
