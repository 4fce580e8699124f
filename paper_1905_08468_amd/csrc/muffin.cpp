// libmuffin runtime: handle, workspace, set-up and the iteration driver.
//
// One iteration (Algorithm 2; Algorithm 5 with sure = 1) is a fixed
// sequence of launches on the caller's stream, with no host
// synchronisation:
//   1. G_s = H^T H X_s for all state sets          (eq. `grad2`; Algs. 3-4)
//   2. S_s = beta_l W_s^T(a1 U_s + a2 U_primal)    (eq. `adjointspat2`)
//   3. X~_s = (X_s - tau (G_s - H^T y + S_s + T_s))_+ and its derivatives
//                                                  (eqs. `stpm`, `stpx`)
//   4. U_s <- sat(U_s + sigma beta_l W_s(z_s))    (eqs. `stpp`, `stpu`)
//   5. V_s <- sat(V_s + sigma alpha_n C z_s), T_s = alpha_n C^T(...)
//                                                  (eqs. `vt`, `v`, `upt`)
//   6. X_s <- X~_s (pointer swap)                   (eq. `updatenode2`)
// State sets: 0 = primal on Y, 1 = primal on Ybar = Y + eps delta,
// 2/3 = d/dmu, d/dgamma of set 0, 4/5 = the same for set 1.  After every
// Delta completed iterations, SUGAR is reduced in FP64 from
// <H^T H X - H^T y, X'> and <H^T delta, Xbar' - X'> (eq. `SUGAR` rewritten
// with adjoints), theta is updated on the device (eq. `adaptgrad`) and the
// derivative states restart from zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <memory>
#include <new>
#include <numeric>
#include <vector>

#include "muffin.h"
#include "internal.hpp"

using namespace muffin;

#define RC(expr)                \
  do {                          \
    int _rc = (expr);           \
    if (_rc != 0) return _rc;   \
  } while (0)

namespace {

// Stages timed with HIP events when timing is on (muffin_set_timing).
enum Stage {
  ST_FFT = 0,          // H^T H X for all sets (5 launches)
  ST_SYN_DEEP,         // synthesis levels J..2
  ST_SYN_L1,           // synthesis level 1 (one launch, all sets)
  ST_PRIMAL,           // primal step (one launch)
  ST_AN_L1_PRIMAL,     // analysis level 1 + dual update, primal sets (one launch)
  ST_AN_DEEP_PRIMAL,   // analysis levels 2..J, primal sets
  ST_AN_L1_DERIV,      // analysis level 1, derivative sets (one launch)
  ST_AN_DEEP_DERIV,    // analysis levels 2..J, derivative sets
  ST_DCT_PRIMAL,       // spectral DCT update, primal sets (one launch)
  ST_DCT_DERIV,        // spectral DCT update, derivative sets (one launch)
  ST_WINDOW,           // SURE/SUGAR reductions, theta update, resets
  ST_FFT_R1,           // the five launches of ST_FFT: first row pass,
  ST_FFT_C1,           //   first column pass,
  ST_FFT_R2,           //   middle row pass,
  ST_FFT_C2,           //   second column pass,
  ST_FFT_R3,           //   last row pass (ST_FFT is their sum)
  ST_COUNT
};

const char* const kStageNames[ST_COUNT] = {
    "fft_chain", "synthesis_deep", "synthesis_l1",
    "primal_step",      "analysis_l1_primal", "analysis_deep_primal", "analysis_l1_deriv",
    "analysis_deep_deriv", "dct_primal", "dct_deriv", "window_update",
    "fft_row1", "fft_col1", "fft_row2", "fft_col2", "fft_row3"};

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> pending_stage;   // stage of each recorded pair
  size_t used = 0;                  // events used since the last collect
  double ms[ST_COUNT] = {};
  long long calls[ST_COUNT] = {};
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int stage, hipStream_t s) {
    if (!on) return;
    hipEvent_t e = get();
    if (e) (void)hipEventRecord(e, s);
    pending_stage.push_back(stage);
  }
  void end(hipStream_t s) {
    if (!on) return;
    hipEvent_t e = get();
    if (e) (void)hipEventRecord(e, s);
  }
  // the FFT chain's pass boundaries (ChainIO::mark): pass p ends the
  // previous pass's interval and starts its own
  struct PassMark {
    Timer* t;
    hipStream_t s;
  };
  static void pass_mark(void* ctx, int p) {
    auto* m = static_cast<PassMark*>(ctx);
    if (p > 0) m->t->end(m->s);
    if (p < 5) m->t->begin(ST_FFT_R1 + p, m->s);
  }
  int collect(hipStream_t s) {
    if (used == 0) return 0;
    if (hipStreamSynchronize(s) != hipSuccess) return -5;
    for (size_t i = 0; i < pending_stage.size() && 2 * i + 1 < used; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, pool[2 * i], pool[2 * i + 1]) == hipSuccess) {
        ms[pending_stage[i]] += t;
        calls[pending_stage[i]] += 1;
      }
    }
    pending_stage.clear();
    used = 0;
    return 0;
  }
  void reset() {
    for (int i = 0; i < ST_COUNT; ++i) {
      ms[i] = 0;
      calls[i] = 0;
    }
  }
  ~Timer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// U planes per band: the P bases of the Daubechies union, or the J scales
// and the coarse plane of the starlet transform
size_t planes_of(const muffin_config* c) {
  return c->dictionary == MUFFIN_DICT_STARLET ? (size_t)c->levels + 1 : (size_t)c->n_bases;
}

int validate(const muffin_config* c) {
  if (!c) return MUFFIN_E_INVAL;
  if (c->dictionary != MUFFIN_DICT_DAUBECHIES && c->dictionary != MUFFIN_DICT_STARLET)
    return MUFFIN_E_INVAL;
  if (c->dictionary == MUFFIN_DICT_STARLET && (c->levels < 1 || c->levels > 5))
    return MUFFIN_E_SHAPE;
  if (c->visibilities != 0 && c->visibilities != 1) return MUFFIN_E_INVAL;
  if (c->visibilities && (!(c->vis_norm2 >= 0) || (c->sure && !(c->vis_count > 0))))
    return MUFFIN_E_INVAL;
  if (!is_pow2(c->n) || c->n < 8 || c->n > 2048) return MUFFIN_E_SHAPE;
  if (c->L < 1 || c->L > 256) return MUFFIN_E_SHAPE;
  if (c->n_bases < 1 || c->n_bases > kMaxBases) return MUFFIN_E_SHAPE;
  if (c->levels < 1 || (c->n >> c->levels) < 1) return MUFFIN_E_SHAPE;
  if (c->mode < MUFFIN_F64 || c->mode > MUFFIN_F32_BF16DCT) return MUFFIN_E_INVAL;
  if (!(c->sigma > 0) || !(c->mu >= 0) || !(c->gamma >= 0)) return MUFFIN_E_INVAL;
  if (c->tau <= 0 && !(c->rho > 0 && c->rho < 1)) return MUFFIN_E_INVAL;
  if (c->tau_rule != MUFFIN_TAU_OPNORM && c->tau_rule != MUFFIN_TAU_PAPER_SUM)
    return MUFFIN_E_INVAL;
  if (!(c->eps_w > 0)) return MUFFIN_E_INVAL;
  if (c->sure) {
    if (c->delta_period < 1) return MUFFIN_E_INVAL;
    if (!(c->eps_fd > 0) || !(c->sigma_w > 0)) return MUFFIN_E_INVAL;
    if (!(c->eta_mu >= 0) || !(c->eta_gamma >= 0)) return MUFFIN_E_INVAL;
  }
  if (c->tau <= 0 && c->pi_iters < 1) return MUFFIN_E_INVAL;
  if (!(c->stop_rel >= 0)) return MUFFIN_E_INVAL;
  if (c->stop_rel > 0 && c->check_every < 1) return MUFFIN_E_INVAL;
  return MUFFIN_OK;
}

}  // namespace muffin

void* muffin::region_alloc(Region* r, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (r == nullptr) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  const size_t need = region_round(bytes);
  if (r->used > r->cap || need > r->cap - r->used) return nullptr;
  void* p = r->base + r->used;
  r->used += need;
  return p;
}

namespace muffin {

// The device buffers of a handle or of a set-up step: hipMalloc'd pieces,
// or pieces of a caller's region (then release() rewinds the region to where
// this object's first piece began; such objects are released in the reverse
// order of their first allocation).
struct Dev {
  std::vector<void*> owned;
  bool failed = false;
  Region* region = nullptr;
  size_t mark = 0;
  bool marked = false;
  Dev() = default;
  explicit Dev(Region* r) : region(r) {}
  template <typename U>
  U* alloc(size_t count) {
    if (failed) return nullptr;
    if (count == 0) count = 1;
    if (region && !marked) {
      mark = region->used;
      marked = true;
    }
    void* p = region_alloc(region, sizeof(U) * count);
    if (!p) {
      failed = true;
      return nullptr;
    }
    if (!region) owned.push_back(p);
    return static_cast<U*>(p);
  }
  // marks the region's current end now, so that release() also rewinds
  // pieces taken from the region by others (plan tables) after this call
  void hold() {
    if (region && !marked) {
      mark = region->used;
      marked = true;
    }
  }
  void release() {
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
    if (region && marked) region->used = mark;
    marked = false;
  }
};

struct ImplBase {
  virtual ~ImplBase() = default;
  virtual int init() = 0;
  virtual int set_problem(const void*, const void*, const double*, const double*,
                          const void*) = 0;
  virtual int run(int iters) = 0;
  virtual int report(muffin_report* r) = 0;
  virtual int get_state(int which, int set, void* out) = 0;
  virtual int set_state(int which, int set, const void* in) = 0;
  virtual int history(double* rows, int max_rows) = 0;
  virtual int weights(double* alpha, double* beta) = 0;
  virtual int op(int kind, const void* in, void* out) = 0;
  virtual int set_initial(const void* x0) = 0;
  virtual int run_chunk(int iters, bool check) = 0;
  virtual int iterate_n(int iters) = 0;  // enqueue only (no checks, no sync)
  virtual void advance(int iters) = 0;   // host counters after graph replays
  virtual int iters_done() const = 0;
  virtual bool ready() const = 0;
  virtual int chunk_poll(int* done, double* rel) = 0;
  virtual size_t state_bytes() = 0;
  virtual int state_save(void* buf, size_t bytes) = 0;
  virtual int state_load(const void* buf, size_t bytes) = 0;
  virtual Timer& timer() = 0;
  virtual hipStream_t stream() = 0;
  virtual int quality(const void* truth, double* snr_db, double* wmse) = 0;
  virtual void preset_beta_H(double v) = 0;
  virtual int autotune(int reps, muffin_tune_result* r) = 0;
};

size_t workspace_bytes_of(const muffin_config* c) {
  const size_t n = c->n, L = c->L, P = planes_of(c);
  const size_t N = n * n, LN = L * N;
  const size_t es = c->mode == MUFFIN_F64 ? 8 : 4;
  const size_t nsets = c->sure ? 6 : 1;
  // per set: X, X~, V, T, G, S + U (P LN) + scratch (4 LN: two spectra, or
  // the wavelet low-pass temporaries)
  const size_t per_set = (6 + P + 4) * LN * es;
  size_t shared = LN * es * (c->sure ? 5 : 2);                  // Y, Ybar, HTy, HTybar, HTd
  shared += L * (n + 1) * 2 * n * 2 * es;                        // transfer functions
  // masks: U (bytes per coefficient for the starlet, bit words per analysis
  // thread for the Daubechies union) and V (bit words per spectral thread)
  const size_t mu_bytes = std::max(P * LN, 4 * dwt_mask_words((int)n, (int)L, c->levels,
                                                                (int)P, (int)es));
  const size_t mv_bytes = std::max(LN, 4 * dct_mask_words((int)N));
  shared += c->sure ? 2 * (mu_bytes + mv_bytes) : 0;
  // weights; partial sums (as allocated by init); theta history; device
  // parameters, flags and small sums
  const size_t nparts = std::max({(size_t)fft_res_blocks((int)n, (int)L, (int)es),
                                  (size_t)dot_blocks(), (size_t)(64 * L * 3), (size_t)4096});
  shared += (N + L) * 8 + nparts * 8 + (size_t)kMaxHistRows * kHistCols * 8 + 64 * 1024;
  if (c->stop_rel > 0) shared += (P + 1) * LN * es;              // U, V snapshots (stop rule)
  return nsets * per_set + shared;
}

// Level-1 tile shapes chosen by muffin_autotune, per size class
// (n, L, P, element size, state sets).
struct TuneTable {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> shapes;
};
TuneTable& tune_table() {
  static TuneTable t;
  return t;
}

template <typename T>
struct Impl final : ImplBase {
  muffin_config cfg;
  hipStream_t st;
  int n, L, P, J, N;
  size_t LN;
  int nsets;
  Dev dev;
  FftPlan<T> fft;
  DwtPlan<T> dwt;
  bool star = false;  // spatial dictionary: starlet (else the Daubechies union)
  bool vis = false;   // data are visibilities: the gradient's operator is the
                      // PSF convolution (chain op 0) instead of H^T H (op 2)
  int gop() const { return vis ? 0 : 2; }
  StarletPlan spl;
  DctPlan<T> dct;
  DevParams* dp = nullptr;
  DevParams hp{};
  Region* region = nullptr;  // non-null: every device buffer comes from it
  T *X[kMaxSets]{}, *Xt[kMaxSets]{}, *U[kMaxSets]{}, *V[kMaxSets]{}, *Tt[kMaxSets]{};
  T *G[kMaxSets]{}, *S[kMaxSets]{}, *scr[kMaxSets]{};
  uint8_t *maskU[2]{}, *maskV[2]{};
  T *Y = nullptr, *Ybar = nullptr, *HTy = nullptr, *HTybar = nullptr, *HTd = nullptr;
  double *alpha = nullptr, *beta = nullptr, *partials = nullptr, *hist = nullptr;
  int* flag = nullptr;
  // stopping rule: U, V of the Y trajectory before a checked iteration, and
  // the six FP64 sums of the relative change
  T *Usnap = nullptr, *Vsnap = nullptr;
  double* relsum = nullptr;
  double* qsum = nullptr;        // quality sums (SNR, WMSE)
  double preset_bH = 0.0;        // > 0: beta_H known, set-up skips the power iteration
  double last_rel = -1.0;
  bool stopped = false;
  // asynchronous chunks (serving): completion event, pinned copy of the sums
  hipEvent_t chunk_ev = nullptr;
  double* relhost = nullptr;
  bool chunk_check = false;
  int max_hist = 0;
  bool have_problem = false;
  int k_done = 0;
  int n_upd = 0;
  double beta_H = 0.0;
  Timer tm;

  Timer& timer() override { return tm; }
  hipStream_t stream() override { return st; }

  Impl(const muffin_config& c, hipStream_t s) : cfg(c), st(s) {
    n = c.n;
    L = c.L;
    P = (int)planes_of(&c);
    J = c.levels;
    star = c.dictionary == MUFFIN_DICT_STARLET;
    vis = c.visibilities != 0;
    spl.n = n;
    spl.L = L;
    spl.J = J;
    N = n * n;
    LN = (size_t)L * N;
    nsets = c.sure ? 6 : 1;
  }
  ~Impl() override {
    if (chunk_ev) (void)hipEventDestroy(chunk_ev);
    if (relhost) (void)hipHostFree(relhost);
    fft_free_plan(fft);
    dct_free_plan(dct);
    dev.release();
  }

  cplx<T>* specA(int s) { return reinterpret_cast<cplx<T>*>(scr[s]); }
  cplx<T>* specB(int s) { return reinterpret_cast<cplx<T>*>(scr[s] + 2 * LN); }
  T* tmp0(int s) { return scr[s]; }
  T* tmp1(int s) { return scr[s] + 2 * LN; }
  // 2 x~ - x of set s: written by the primal step, read by the spatial and
  // spectral analyses of the same iteration (the last quarter of the
  // scratch, which the low-pass temporaries never reach)
  T* zbuf(int s) { return scr[s] + 3 * LN; }

  int init() override {
    dev.region = region;
    for (int s = 0; s < nsets; ++s) {
      X[s] = dev.alloc<T>(LN);
      Xt[s] = dev.alloc<T>(LN);
      U[s] = dev.alloc<T>(LN * P);
      V[s] = dev.alloc<T>(LN);
      Tt[s] = dev.alloc<T>(LN);
      G[s] = dev.alloc<T>(LN);
      S[s] = dev.alloc<T>(LN);
      scr[s] = dev.alloc<T>(4 * LN);
    }
    Y = dev.alloc<T>(LN);
    HTy = dev.alloc<T>(LN);
    if (cfg.sure) {
      Ybar = dev.alloc<T>(LN);
      HTybar = dev.alloc<T>(LN);
      HTd = dev.alloc<T>(LN);
      for (int t = 0; t < 2; ++t) {
        maskU[t] = dev.alloc<uint8_t>(std::max(LN * P, 4 * dwt_mask_words(n, L, J, P, sizeof(T))));
        maskV[t] = dev.alloc<uint8_t>(std::max(LN, 4 * dct_mask_words(N)));
      }
    }
    alpha = dev.alloc<double>(N);
    beta = dev.alloc<double>(L);
    const int nres = fft_res_blocks(n, L, sizeof(T));
    partials = dev.alloc<double>(std::max({nres, dot_blocks(), 64 * L * 3, 4096}));
    max_hist = kMaxHistRows;
    hist = dev.alloc<double>((size_t)max_hist * kHistCols);
    dp = dev.alloc<DevParams>(1);
    flag = dev.alloc<int>(1);
    qsum = dev.alloc<double>(4);
    if (cfg.stop_rel > 0) {
      Usnap = dev.alloc<T>(LN * P);
      Vsnap = dev.alloc<T>(LN);
      relsum = dev.alloc<double>(8);
    }
    if (dev.failed) {
      dev.release();
      return MUFFIN_E_NOMEM;
    }
    RC(fft_make_plan(fft, n, L, st, region));
    dwt.n = n;
    dwt.L = L;
    dwt.P = P;
    dwt.J = J;
    if (!star) RC(dwt_upload_filters(P));
    RC(dct_make_plan(dct, L, N,
                      sizeof(T) == 8 ? DCT_F64
                                     : (cfg.mode == MUFFIN_F32_BF16DCT ? DCT_BF16X3 : DCT_F32),
                      region));
    hp.sigma = cfg.sigma;
    hp.mu = cfg.mu;
    hp.gamma = cfg.gamma;
    MUFFIN_HIP_CHECK(hipMemcpy(dp, &hp, sizeof(hp), hipMemcpyHostToDevice));
    return 0;
  }

  // -- operator helpers ------------------------------------------------
  int chain(const T* const* in, T* const* out, const int* sets, int ns, int op,
            const T* y = nullptr, double* res = nullptr, Timer::PassMark* pm = nullptr) {
    ChainIO<T> io{};
    if (pm) {
      io.mark = &Timer::pass_mark;
      io.mark_ctx = pm;
    }
    for (int i = 0; i < ns; ++i) {
      io.in[i] = in[i];
      io.out[i] = out[i];
      io.specA[i] = specA(sets[i]);
      io.specB[i] = specB(sets[i]);
    }
    io.y = y;
    io.res_partials = res;
    io.nsets = ns;
    return fft_chain(fft, io, op, st);
  }

  int chain1(const T* in, T* out, int op) {
    const int s0 = 0;
    return chain(&in, &out, &s0, 1, op);
  }

  // -- power iteration (FP64) ------------------------------------------
  int power_iteration(const T* psf) {
    FftPlan<double> f64;
    FftPlan<double>* pf = nullptr;
    Dev tmp(region);
    tmp.hold();
    double* psf64 = nullptr;
    if constexpr (sizeof(T) == 8) {
      pf = reinterpret_cast<FftPlan<double>*>(&fft);
    } else {
      // (the plan's tables come first from a region: tmp's pieces follow)
      const int prc = fft_make_plan(f64, n, L, st, region);
      if (prc) {
        fft_free_plan(f64);
        tmp.release();
        return prc;
      }
      pf = &f64;
      psf64 = tmp.alloc<double>((size_t)L * 4 * N);
      cplx<double>* ktmp = tmp.alloc<cplx<double>>((size_t)L * (n + 1) * 2 * n);
      if (tmp.failed) {
        fft_free_plan(f64);
        tmp.release();
        return MUFFIN_E_NOMEM;
      }
      const float* psf32 = reinterpret_cast<const float*>(psf);
      const int crc = convert<float, double>(psf64, psf32, (size_t)L * 4 * N, st);
      RC(crc);
      RC(fft_psf_spectrum(f64, psf64, ktmp, st));
    }
    double* v = tmp.alloc<double>(LN);
    double* w = tmp.alloc<double>(LN);
    cplx<double>* sa = tmp.alloc<cplx<double>>(LN);
    cplx<double>* sb = tmp.alloc<cplx<double>>(LN);
    double* stats = tmp.alloc<double>((size_t)3 * L);
    if (tmp.failed) {
      if (sizeof(T) == 4) fft_free_plan(f64);
      tmp.release();
      return MUFFIN_E_NOMEM;
    }
    const int bpb = 64;
    RC(pi_init(v, LN, 0x5EEDull, st));
    std::vector<double> hs(3 * L);
    double prev = 0.0, lam = 0.0;
    int rc = 0;
    for (int it = 1; it <= cfg.pi_iters; ++it) {
      ChainIO<double> io{};
      io.in[0] = v;
      io.out[0] = w;
      io.specA[0] = sa;
      io.specB[0] = sb;
      io.nsets = 1;
      if ((rc = fft_chain(*pf, io, gop(), st))) break;
      if ((rc = pi_band_dots(v, w, L, N, partials, bpb, st))) break;
      if ((rc = pi_band_finish(partials, L, bpb, stats, st))) break;
      if ((rc = pi_normalise(v, w, stats, L, N, st))) break;
      if (it % 10 == 0 || it == cfg.pi_iters) {
        if (hipMemcpyAsync(hs.data(), stats, sizeof(double) * 3 * L, hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          rc = MUFFIN_E_HIP;
          break;
        }
        lam = 0.0;
        for (int l = 0; l < L; ++l) lam = std::max(lam, hs[3 * l] / hs[3 * l + 2]);
        if (it > 10 && std::fabs(lam - prev) <= cfg.pi_tol * std::fabs(lam)) break;
        prev = lam;
      }
    }
    (void)hipStreamSynchronize(st);
    if (sizeof(T) == 4) fft_free_plan(f64);
    tmp.release();
    if (rc) return rc;
    beta_H = lam;
    return 0;
  }

  int set_problem(const void* dirty, const void* psf, const double* a_host,
                  const double* b_host, const void* delta) override {
    if (!dirty || !psf) return MUFFIN_E_INVAL;
    if (cfg.sure && !delta) return MUFFIN_E_INVAL;
    const T* dy = static_cast<const T*>(dirty);
    const T* ps = static_cast<const T*>(psf);
    const T* de = static_cast<const T*>(delta);
    // non-finite inputs
    MUFFIN_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), st));
    RC(count_nonfinite(dy, LN, flag, st));
    RC(count_nonfinite(ps, (size_t)L * 4 * N, flag, st));
    if (cfg.sure) RC(count_nonfinite(de, LN, flag, st));
    int hflag = 0;
    MUFFIN_HIP_CHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    if (hflag) return MUFFIN_E_NONFINITE;
    MUFFIN_HIP_CHECK(hipMemcpyAsync(Y, dy, sizeof(T) * LN, hipMemcpyDeviceToDevice, st));
    // transfer functions (K-PSF)
    {
      Dev tmp(region);
      cplx<T>* ktmp = tmp.alloc<cplx<T>>((size_t)L * (n + 1) * 2 * n);
      if (tmp.failed) return MUFFIN_E_NOMEM;
      int rc = fft_psf_spectrum(fft, ps, ktmp, st);
      (void)hipStreamSynchronize(st);
      tmp.release();
      RC(rc);
    }
    // weights (Section 2.1)
    std::vector<double> ha(N), hb(L);
    if (!a_host || !b_host) {
      RC(weights_from(Y, L, N, cfg.eps_w, alpha, beta, partials, st));
      if (star) {
        // the starlet is not norm-preserving: beta_l = 1/(||W_s y_l|| + eps)
        // from the transform of the dirty cube (U of set 0 is zeroed below)
        AnalysisIO<T> io{};
        io.nsets = 1;
        io.z_a[0] = Y;
        io.c1_sel[0] = SEL_ONE;
        io.c2_sel[0] = SEL_ZERO;
        io.U[0] = U[0];
        io.tmp0[0] = tmp0(0);
        io.tmp1[0] = tmp1(0);
        io.pure = 1;
        io.pure_scale = 1.0;
        RC(starlet_analysis(spl, io, nullptr, st));
        RC(beta_from<T>(U[0], L, (int)(P * N), cfg.eps_w, beta, partials, st));
      }
      MUFFIN_HIP_CHECK(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * N,
                                      hipMemcpyDeviceToHost, st));
      MUFFIN_HIP_CHECK(hipMemcpyAsync(hb.data(), beta, sizeof(double) * L,
                                      hipMemcpyDeviceToHost, st));
      MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    }
    if (a_host) std::copy(a_host, a_host + N, ha.begin());
    if (b_host) std::copy(b_host, b_host + L, hb.begin());
    for (double v : ha)
      if (!std::isfinite(v) || v < 0) return MUFFIN_E_INVAL;
    for (double v : hb)
      if (!std::isfinite(v) || v < 0) return MUFFIN_E_INVAL;
    MUFFIN_HIP_CHECK(hipMemcpyAsync(alpha, ha.data(), sizeof(double) * N,
                                    hipMemcpyHostToDevice, st));
    MUFFIN_HIP_CHECK(hipMemcpyAsync(beta, hb.data(), sizeof(double) * L,
                                    hipMemcpyHostToDevice, st));
    double ma = 0, sa = 0, mb = 0, sb = 0;
    for (double v : ha) {
      ma = std::max(ma, v * v);
      sa += v * v;
    }
    for (double v : hb) {
      mb = std::max(mb, v * v);
      sb += v * v;
    }
    // Lipschitz constant and tau (Section 2.2)
    beta_H = 0.0;
    if (preset_bH > 0)
      beta_H = preset_bH;
    else if (cfg.tau <= 0 || cfg.pi_iters > 0)
      RC(power_iteration(ps));
    hp = DevParams{};
    hp.mu = cfg.mu;
    hp.gamma = cfg.gamma;
    hp.sigma = cfg.sigma;
    hp.beta_H = beta_H;
    hp.max_beta2 = mb;
    hp.sum_beta2 = sb;
    hp.max_alpha2 = ma;
    hp.sum_alpha2 = sa;
    hp.rho = cfg.rho;
    hp.ws_norm2 = star ? starlet_norm2(n, J) : 1.0;
    hp.eta_mu = cfg.eta_mu;
    hp.eta_gamma = cfg.eta_gamma;
    hp.eps_fd = cfg.eps_fd;
    hp.sigma_w = cfg.sigma_w;
    hp.vis = vis ? 1 : 0;
    hp.res_const = vis ? cfg.vis_norm2 : 0.0;
    hp.n_meas = vis ? cfg.vis_count : double(LN);
    if (cfg.tau > 0) {
      hp.tau_rule = -1;
      hp.tau = cfg.tau;
    } else {
      hp.tau_rule = cfg.tau_rule;
      const double k = cfg.tau_rule == MUFFIN_TAU_OPNORM
                           ? hp.ws_norm2 * cfg.mu * cfg.mu * mb + cfg.gamma * cfg.gamma * ma
                           : hp.ws_norm2 * cfg.mu * cfg.mu * sb + cfg.gamma * cfg.gamma * sa;
      hp.tau = cfg.rho / (0.5 * beta_H + cfg.sigma * k);
    }
    MUFFIN_HIP_CHECK(hipMemcpyAsync(dp, &hp, sizeof(hp), hipMemcpyHostToDevice, st));
    // H^T y, and for ADA-PT the perturbed data Ybar = Y + eps delta (Alg. 5)
    // (visibilities: the inputs are already back-projected, Re H^* v and
    // Re H^* delta, so they stand for H^T y and H^T delta)
    if (vis) RC(copy_dev<T>(HTy, Y, LN, st));
    else RC(chain1(Y, HTy, 1));
    if (cfg.sure) {
      RC(axpy_copy(Ybar, Y, de, cfg.eps_fd, LN, st));
      if (vis) {
        RC(copy_dev<T>(HTybar, Ybar, LN, st));
        RC(copy_dev<T>(HTd, de, LN, st));
      } else {
        RC(chain1(Ybar, HTybar, 1));
        RC(chain1(de, HTd, 1));
      }
    }
    // zero state
    for (int s = 0; s < nsets; ++s) {
      RC(fill_zero(X[s], LN, st));
      RC(fill_zero(U[s], LN * P, st));
      RC(fill_zero(V[s], LN, st));
      RC(fill_zero(Tt[s], LN, st));
    }
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    k_done = 0;
    last_rel = -1.0;
    stopped = false;
    n_upd = 0;
    have_problem = true;
    return 0;
  }

  // -- one iteration ---------------------------------------------------
  int iterate() {
    const bool sure = cfg.sure != 0;
    // 1. H^T H X for every set (one chain: the transfer function is read
    //    once per column for all sets)
    {
      const int sets[kMaxSets] = {0, 1, 2, 3, 4, 5};
      const T* in[kMaxSets];
      T* out[kMaxSets];
      for (int s = 0; s < nsets; ++s) {
        in[s] = X[s];
        out[s] = G[s];
      }
      // timed per pass (the chain's total is their sum)
      Timer::PassMark pm{&tm, st};
      RC(chain(in, out, sets, nsets, gop(), nullptr, nullptr, tm.on ? &pm : nullptr));
    }
    // 2. synthesis
    {
      SynthesisIO<T> io{};
      io.nsets = nsets;
      io.beta = beta;
      // Every set synthesises its own dual variable, S = beta / sqrt(P)
      // W_s^T U (linear, so the mu-derivative's W_s^T (mu U' + U) is
      // mu S' + S of the primal set: the primal step combines them)
      for (int s = 0; s < nsets; ++s) {
        io.Ua[s] = U[s];
        io.S[s] = S[s];
        io.tmp0[s] = tmp0(s);
        io.tmp1[s] = tmp1(s);
      }
      if (star) {
        tm.begin(ST_SYN_L1, st);
        RC(starlet_synthesis(spl, io, st));
        tm.end(st);
      } else {
        if (J >= 2) {
          tm.begin(ST_SYN_DEEP, st);
          RC(dwt_synthesis(dwt, io, dp, st, 2, J));
          tm.end(st);
        }
        tm.begin(ST_SYN_L1, st);
        RC(dwt_synthesis(dwt, io, dp, st, 1, 1));
        tm.end(st);
      }
    }
    // 3. primal step and its derivatives
    {
      PrimalIO<T> io{};
      io.ntraj = sure ? 2 : 1;
      io.nderiv = sure ? 2 : 0;
      const int sets[2][3] = {{0, 2, 3}, {1, 4, 5}};
      for (int t = 0; t < io.ntraj; ++t) {
        for (int d = 0; d <= io.nderiv; ++d) {
          const int s = sets[t][d];
          io.x[t][d] = X[s];
          io.g[t][d] = G[s];
          io.s[t][d] = S[s];
          io.t[t][d] = Tt[s];
          io.xt[t][d] = Xt[s];
          io.z[t][d] = zbuf(s);
        }
        io.hty[t] = t == 0 ? HTy : HTybar;
      }
      tm.begin(ST_PRIMAL, st);
      RC(primal_step(io, LN, dp, st));
      tm.end(st);
    }
    // 4. spatial analysis + dual update
    {
      AnalysisIO<T> io{};
      io.role = ROLE_PRIMAL;
      io.nsets = sure ? 2 : 1;
      io.beta = beta;
      for (int s = 0; s < io.nsets; ++s) {
        io.z_a[s] = zbuf(s);
        io.c1_sel[s] = SEL_MU;
        io.c2_sel[s] = SEL_ZERO;
        io.U[s] = U[s];
        io.mask[s] = sure ? maskU[s] : nullptr;
        io.tmp0[s] = tmp0(s);
        io.tmp1[s] = tmp1(s);
      }
      tm.begin(ST_AN_L1_PRIMAL, st);
      RC(star ? starlet_analysis(spl, io, dp, st) : dwt_analysis(dwt, io, dp, st, 1, 1));
      tm.end(st);
      if (J >= 2 && !star) {
        tm.begin(ST_AN_DEEP_PRIMAL, st);
        RC(dwt_analysis(dwt, io, dp, st, 2, J));
        tm.end(st);
      }
      if (sure) {
        AnalysisIO<T> d{};
        d.role = ROLE_DERIV;
        d.nsets = 4;
        d.beta = beta;
        for (int i = 0; i < 4; ++i) {
          const int s = 2 + i, prim = i < 2 ? 0 : 1;
          const bool is_mu = (i % 2) == 0;
          d.z_a[i] = zbuf(s);
          d.c1_sel[i] = SEL_MU;
          d.z_b[i] = is_mu ? zbuf(prim) : nullptr;
          d.c2_sel[i] = is_mu ? SEL_ONE : SEL_ZERO;
          d.U[i] = U[s];
          d.mask[i] = maskU[prim];
          d.tmp0[i] = tmp0(s);
          d.tmp1[i] = tmp1(s);
        }
        tm.begin(ST_AN_L1_DERIV, st);
        RC(star ? starlet_analysis(spl, d, dp, st) : dwt_analysis(dwt, d, dp, st, 1, 1));
        tm.end(st);
        if (J >= 2 && !star) {
          tm.begin(ST_AN_DEEP_DERIV, st);
          RC(dwt_analysis(dwt, d, dp, st, 2, J));
          tm.end(st);
        }
      }
    }
    // 5. spectral DCT + dual update + adjoint
    {
      DctIO<T> io{};
      io.role = ROLE_PRIMAL;
      io.nsets = sure ? 2 : 1;
      io.alpha = alpha;
      for (int s = 0; s < io.nsets; ++s) {
        io.z_a[s] = zbuf(s);
        io.c1_sel[s] = SEL_GAMMA;
        io.c2_sel[s] = SEL_ZERO;
        io.V[s] = V[s];
        io.Vb[s] = nullptr;
        io.d1_sel[s] = SEL_GAMMA;
        io.d2_sel[s] = SEL_ZERO;
        io.Tout[s] = Tt[s];
        io.mask[s] = sure ? maskV[s] : nullptr;
      }
      tm.begin(ST_DCT_PRIMAL, st);
      RC(dct_update(dct, io, dp, st));
      tm.end(st);
      if (sure) {
        DctIO<T> d{};
        d.role = ROLE_DERIV;
        d.nsets = 4;
        d.alpha = alpha;
        for (int i = 0; i < 4; ++i) {
          const int s = 2 + i, prim = i < 2 ? 0 : 1;
          const bool is_ga = (i % 2) == 1;
          d.z_a[i] = zbuf(s);
          d.c1_sel[i] = SEL_GAMMA;
          d.z_b[i] = is_ga ? zbuf(prim) : nullptr;
          d.c2_sel[i] = is_ga ? SEL_ONE : SEL_ZERO;
          d.V[i] = V[s];
          d.Vb[i] = is_ga ? V[prim] : nullptr;
          d.d1_sel[i] = SEL_GAMMA;
          d.d2_sel[i] = is_ga ? SEL_ONE : SEL_ZERO;
          d.Tout[i] = Tt[s];
          d.mask[i] = maskV[prim];
        }
        tm.begin(ST_DCT_DERIV, st);
        RC(dct_update(dct, d, dp, st));
        tm.end(st);
      }
    }
    // 6. X <- X~
    for (int s = 0; s < nsets; ++s) std::swap(X[s], Xt[s]);
    ++k_done;
    if (sure && k_done % cfg.delta_period == 0) {
      tm.begin(ST_WINDOW, st);
      RC(window_end());
      tm.end(st);
    }
    return 0;
  }

  // ADA-PT update after Delta completed iterations (Alg. 5, eq. `adaptgrad`)
  int window_end() {
    const int q = n_upd++;
    // H^T H X^(k) of the Y trajectory, with ||Y - H X||^2 on the way
    const int nres = fft_res_blocks(n, L, sizeof(T));
    const int nb = dot_blocks();
    {
      const int s0 = 0;
      const T* in = X[0];
      T* out = G[0];
      if (vis) {
        // psf * X, then |v - H X|^2 = |v|^2 + <psf * X - Re H^* v, X> - <Re H^* v, X>
        RC(chain(&in, &out, &s0, 1, 0));
        RC(dot_partials<T>(G[0], HTy, X[0], LN, partials, nb, st));
        RC(reduce_to_slot(partials, nb, dp, SLOT_RES2, st));
        RC(dot_partials<T>(HTy, nullptr, X[0], LN, partials, nb, st));
        RC(reduce_to_slot(partials, nb, dp, SLOT_AUX0, st));
      } else {
        RC(chain(&in, &out, &s0, 1, 2, Y, partials));
        RC(reduce_to_slot(partials, nres, dp, SLOT_RES2, st));
      }
    }
    RC(dot_partials<T>(G[0], HTy, X[2], LN, partials, nb, st));
    RC(reduce_to_slot(partials, nb, dp, SLOT_GX_MU, st));
    RC(dot_partials<T>(G[0], HTy, X[3], LN, partials, nb, st));
    RC(reduce_to_slot(partials, nb, dp, SLOT_GX_GA, st));
    RC(dot_partials<T>(X[4], X[2], HTd, LN, partials, nb, st));
    RC(reduce_to_slot(partials, nb, dp, SLOT_FD_MU, st));
    RC(dot_partials<T>(X[5], X[3], HTd, LN, partials, nb, st));
    RC(reduce_to_slot(partials, nb, dp, SLOT_FD_GA, st));
    RC(dot_partials<T>(X[1], X[0], HTd, LN, partials, nb, st));
    RC(reduce_to_slot(partials, nb, dp, SLOT_FD_X, st));
    (void)q;
    RC(theta_update(dp, hist, max_hist, cfg.delta_period, 1, st));
    if (cfg.deriv_reset) {
      for (int s = 2; s < 6; ++s) {
        RC(fill_zero(X[s], LN, st));
        RC(fill_zero(U[s], LN * P, st));
        RC(fill_zero(V[s], LN, st));
        RC(fill_zero(Tt[s], LN, st));
      }
    }
    return 0;
  }

  // Relative change of the Y trajectory over the iteration just run (the
  // stopping rule): max(|X^k - X^(k-1)| / |X^k|,
  // sqrt(|dU|^2 + |dV|^2) / sqrt(|U^k|^2 + |V^k|^2)), FP64 sums.
  int rel_change(double* out) {
    const int nb = dot_blocks();
    RC(diff_sq<T>(X[0], Xt[0], LN, partials, nb, relsum, st));
    RC(diff_sq<T>(U[0], Usnap, LN * P, partials, nb, relsum + 2, st));
    RC(diff_sq<T>(V[0], Vsnap, LN, partials, nb, relsum + 4, st));
    double h[6];
    MUFFIN_HIP_CHECK(hipMemcpyAsync(h, relsum, sizeof(h), hipMemcpyDeviceToHost, st));
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    auto ratio = [](double num, double den) {
      if (den > 0) return num / den;
      return num > 0 ? HUGE_VAL : 0.0;
    };
    const double rx = ratio(h[0], h[1]);
    const double rd = ratio(h[2] + h[4], h[3] + h[5]);
    *out = std::sqrt(std::max(rx, rd));
    return 0;
  }

  int run(int iters) override {
    if (!have_problem) return MUFFIN_E_STATE;
    if (iters < 0) return MUFFIN_E_INVAL;
    stopped = false;
    for (int i = 0; i < iters; ++i) {
      const bool check = cfg.stop_rel > 0 && (k_done + 1) % cfg.check_every == 0;
      if (check) {
        RC(copy_dev<T>(Usnap, U[0], LN * P, st));
        RC(copy_dev<T>(Vsnap, V[0], LN, st));
      }
      RC(iterate());
      if (tm.on && tm.used > 4096) RC(tm.collect(st));
      if (check) {
        RC(rel_change(&last_rel));
        if (last_rel <= cfg.stop_rel) {
          stopped = true;
          break;
        }
      }
    }
    return 0;
  }

  // Enqueues `iters` iterations without waiting; with check (stop_rel > 0)
  // the last one is followed by the stopping-rule sums, copied to pinned
  // host memory.  chunk_poll reports completion and the relative change.
  int run_chunk(int iters, bool check) override {
    if (!have_problem) return MUFFIN_E_STATE;
    if (iters < 1) return MUFFIN_E_INVAL;
    // (checked iterations are the multiples of check_every, as in run())
    check = check && cfg.stop_rel > 0 && (k_done + iters) % cfg.check_every == 0;
    if (!chunk_ev) {
      MUFFIN_HIP_CHECK(hipEventCreateWithFlags(&chunk_ev, hipEventDisableTiming));
      MUFFIN_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&relhost), 8 * sizeof(double),
                                     hipHostMallocDefault));
    }
    for (int i = 0; i < iters; ++i) {
      const bool last = i == iters - 1;
      if (check && last) {
        RC(copy_dev<T>(Usnap, U[0], LN * P, st));
        RC(copy_dev<T>(Vsnap, V[0], LN, st));
      }
      RC(iterate());
    }
    if (check) {
      const int nb = dot_blocks();
      RC(diff_sq<T>(X[0], Xt[0], LN, partials, nb, relsum, st));
      RC(diff_sq<T>(U[0], Usnap, LN * P, partials, nb, relsum + 2, st));
      RC(diff_sq<T>(V[0], Vsnap, LN, partials, nb, relsum + 4, st));
      MUFFIN_HIP_CHECK(hipMemcpyAsync(relhost, relsum, 6 * sizeof(double),
                                      hipMemcpyDeviceToHost, st));
    }
    MUFFIN_HIP_CHECK(hipEventRecord(chunk_ev, st));
    chunk_check = check;
    return 0;
  }

  int iterate_n(int iters) override {
    if (!have_problem) return MUFFIN_E_STATE;
    for (int i = 0; i < iters; ++i) RC(iterate());
    return 0;
  }
  void advance(int iters) override {
    k_done += iters;
    if (cfg.sure) n_upd += iters / cfg.delta_period;
  }
  int iters_done() const override { return k_done; }
  bool ready() const override { return have_problem && !tm.on; }

  int chunk_poll(int* done, double* rel) override {
    *done = 0;
    if (!chunk_ev) return MUFFIN_E_STATE;
    const hipError_t e = hipEventQuery(chunk_ev);
    if (e == hipErrorNotReady) return 0;
    MUFFIN_HIP_CHECK(e);
    *done = 1;
    if (chunk_check) {
      const double* h = relhost;
      auto ratio = [](double num, double den) {
        if (den > 0) return num / den;
        return num > 0 ? HUGE_VAL : 0.0;
      };
      last_rel = std::sqrt(std::max(ratio(h[0], h[1]), ratio(h[2] + h[4], h[3] + h[5])));
      stopped = last_rel <= cfg.stop_rel;
    }
    *rel = last_rel;
    return 0;
  }

  int set_initial(const void* x0) override {
    if (!have_problem) return MUFFIN_E_STATE;
    if (!x0) return MUFFIN_E_INVAL;
    // both trajectories start from x0; derivative states stay zero
    const int ntraj = cfg.sure ? 2 : 1;
    for (int t = 0; t < ntraj; ++t)
      MUFFIN_HIP_CHECK(hipMemcpyAsync(X[t], x0, sizeof(T) * LN, hipMemcpyDeviceToDevice, st));
    return 0;
  }

  // ---- checkpoint: header, device scalars, per set X, U, V, T, history ----
  struct StateHeader {
    char magic[8];
    int32_t version, n, L, P, J, mode, sure, nsets, elem, k_done, n_upd, max_hist, dict, pad;
    DevParams params;
  };
  size_t state_bytes() override {
    return sizeof(StateHeader) + (size_t)nsets * (3 + P) * LN * sizeof(T) +
           (size_t)max_hist * kHistCols * sizeof(double);
  }
  void state_regions(std::vector<std::pair<void*, size_t>>& r) {
    for (int s = 0; s < nsets; ++s) {
      r.push_back({X[s], LN * sizeof(T)});
      r.push_back({U[s], LN * P * sizeof(T)});
      r.push_back({V[s], LN * sizeof(T)});
      r.push_back({Tt[s], LN * sizeof(T)});
    }
    r.push_back({hist, (size_t)max_hist * kHistCols * sizeof(double)});
  }
  int state_save(void* buf, size_t bytes) override {
    if (!have_problem) return MUFFIN_E_STATE;
    if (!buf || bytes < state_bytes()) return MUFFIN_E_INVAL;
    StateHeader hd{};
    std::memcpy(hd.magic, "MUFFINST", 8);
    hd.version = 2;
    hd.dict = cfg.dictionary;
    hd.n = n;
    hd.L = L;
    hd.P = P;
    hd.J = J;
    hd.mode = cfg.mode;
    hd.sure = cfg.sure;
    hd.nsets = nsets;
    hd.elem = (int)sizeof(T);
    hd.k_done = k_done;
    hd.n_upd = n_upd;
    hd.max_hist = max_hist;
    MUFFIN_HIP_CHECK(hipMemcpyAsync(&hd.params, dp, sizeof(DevParams), hipMemcpyDeviceToHost, st));
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    char* o = static_cast<char*>(buf);
    std::memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    std::vector<std::pair<void*, size_t>> r;
    state_regions(r);
    for (auto& e : r) {
      MUFFIN_HIP_CHECK(hipMemcpy(o, e.first, e.second, hipMemcpyDeviceToHost));
      o += e.second;
    }
    return 0;
  }
  int state_load(const void* buf, size_t bytes) override {
    if (!have_problem) return MUFFIN_E_STATE;
    if (!buf || bytes < sizeof(StateHeader)) return MUFFIN_E_INVAL;
    StateHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, "MUFFINST", 8) != 0 || hd.version != 2) return MUFFIN_E_INVAL;
    if (hd.n != n || hd.L != L || hd.P != P || hd.J != J || hd.mode != cfg.mode ||
        hd.dict != cfg.dictionary ||
        hd.sure != cfg.sure || hd.nsets != nsets || hd.elem != (int)sizeof(T) ||
        hd.max_hist != max_hist)
      return MUFFIN_E_SHAPE;
    if (bytes < state_bytes()) return MUFFIN_E_INVAL;
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    const char* o = static_cast<const char*>(buf) + sizeof(hd);
    std::vector<std::pair<void*, size_t>> r;
    state_regions(r);
    for (auto& e : r) {
      MUFFIN_HIP_CHECK(hipMemcpy(e.first, o, e.second, hipMemcpyHostToDevice));
      o += e.second;
    }
    MUFFIN_HIP_CHECK(hipMemcpy(dp, &hd.params, sizeof(DevParams), hipMemcpyHostToDevice));
    k_done = hd.k_done;
    n_upd = hd.n_upd;
    last_rel = -1.0;
    stopped = false;
    return 0;
  }

  int report(muffin_report* r) override {
    DevParams h{};
    MUFFIN_HIP_CHECK(hipMemcpyAsync(&h, dp, sizeof(h), hipMemcpyDeviceToHost, st));
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    std::memset(r, 0, sizeof(*r));
    r->iters_done = k_done;
    r->theta_updates = h.n_updates;
    r->last_rel_change = last_rel;
    r->stopped = stopped ? 1 : 0;
    r->mu = h.mu;
    r->gamma = h.gamma;
    r->tau = h.tau;
    r->beta_H = h.beta_H;
    if (h.n_updates > 0) {
      const int q = std::min(h.n_updates, max_hist) - 1;
      double row[kHistCols];
      MUFFIN_HIP_CHECK(hipMemcpy(row, hist + (size_t)q * kHistCols, sizeof(row),
                                 hipMemcpyDeviceToHost));
      r->sugar_mu = row[4];
      r->sugar_gamma = row[5];
      r->psure = row[6];
      r->res2 = row[7];
    }
    return 0;
  }

  T* state_ptr(int which, int set, size_t* count) {
    if (set < 0 || set >= nsets) return nullptr;
    *count = which == 1 ? LN * P : LN;
    switch (which) {
      case 0: return X[set];
      case 1: return U[set];
      case 2: return V[set];
      case 3: return Tt[set];
      default: return nullptr;
    }
  }

  int get_state(int which, int set, void* out) override {
    size_t cnt = 0;
    T* p = state_ptr(which, set, &cnt);
    if (!p || !out) return MUFFIN_E_INVAL;
    MUFFIN_HIP_CHECK(hipMemcpyAsync(out, p, sizeof(T) * cnt, hipMemcpyDeviceToDevice, st));
    return 0;
  }

  int set_state(int which, int set, const void* in) override {
    size_t cnt = 0;
    T* p = state_ptr(which, set, &cnt);
    if (!p || !in) return MUFFIN_E_INVAL;
    MUFFIN_HIP_CHECK(hipMemcpyAsync(p, in, sizeof(T) * cnt, hipMemcpyDeviceToDevice, st));
    return 0;
  }

  int history(double* rows, int max_rows) override {
    DevParams h{};
    MUFFIN_HIP_CHECK(hipMemcpyAsync(&h, dp, sizeof(h), hipMemcpyDeviceToHost, st));
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    const int avail = std::min(h.n_updates, max_hist);
    const int cnt = std::min(avail, std::max(0, max_rows));
    if (rows && cnt > 0)
      MUFFIN_HIP_CHECK(hipMemcpy(rows, hist, sizeof(double) * kHistCols * cnt,
                                 hipMemcpyDeviceToHost));
    return avail;
  }

  void preset_beta_H(double v) override { preset_bH = v; }

  // Level-1 launches as the iteration issues them (synthesis of every set;
  // analysis of the primal sets, then of the derivative sets), with the
  // state buffers as operands: the values do not matter for the timing.
  int tune_synthesis() {
    SynthesisIO<T> io{};
    io.nsets = nsets;
    io.beta = beta;
    for (int s = 0; s < nsets; ++s) {
      io.Ua[s] = U[s];
      io.S[s] = S[s];
      io.tmp0[s] = tmp0(s);
      io.tmp1[s] = tmp1(s);
    }
    return dwt_synthesis(dwt, io, dp, st, 1, 1);
  }
  int tune_analysis() {
    const bool sure = cfg.sure != 0;
    AnalysisIO<T> io{};
    io.role = ROLE_PRIMAL;
    io.nsets = sure ? 2 : 1;
    io.beta = beta;
    for (int s = 0; s < io.nsets; ++s) {
      io.z_a[s] = zbuf(s);
      io.c1_sel[s] = SEL_MU;
      io.c2_sel[s] = SEL_ZERO;
      io.U[s] = U[s];
      io.mask[s] = sure ? maskU[s] : nullptr;
      io.tmp0[s] = tmp0(s);
      io.tmp1[s] = tmp1(s);
    }
    RC(dwt_analysis(dwt, io, dp, st, 1, 1));
    if (!sure) return 0;
    AnalysisIO<T> d{};
    d.role = ROLE_DERIV;
    d.nsets = 4;
    d.beta = beta;
    for (int i = 0; i < 4; ++i) {
      const int s = 2 + i, prim = i < 2 ? 0 : 1;
      d.z_a[i] = zbuf(s);
      d.c1_sel[i] = SEL_MU;
      d.z_b[i] = (i % 2) == 0 ? zbuf(prim) : nullptr;
      d.c2_sel[i] = (i % 2) == 0 ? SEL_ONE : SEL_ZERO;
      d.U[i] = U[s];
      d.mask[i] = maskU[prim];
      d.tmp0[i] = tmp0(s);
      d.tmp1[i] = tmp1(s);
    }
    return dwt_analysis(dwt, d, dp, st, 1, 1);
  }

  int autotune(int reps, muffin_tune_result* r) override {
    if (have_problem) return MUFFIN_E_STATE;
    *r = muffin_tune_result{};
    const bool can_syn = sizeof(T) == 4 && !star;
    const bool can_an = can_syn && P == 8;
    auto in_use = [&](int forced, int side) { return forced ? forced : (side >= 64 ? 32 : 16); };
    r->tunable = can_syn ? 1 : 0;
    if (!can_syn) {
      r->syn_tile1 = r->an_tile1 = 16;
      return 0;
    }
    const auto key = std::make_tuple(n, L, P, (int)sizeof(T), nsets);
    {
      std::lock_guard<std::mutex> lk(tune_table().mu);
      auto it = tune_table().shapes.find(key);
      if (it != tune_table().shapes.end()) {
        dwt.syn_tile1 = it->second.first;
        dwt.an_tile1 = it->second.second;
        r->cached = 1;
        r->syn_tile1 = dwt.syn_tile1;
        r->an_tile1 = can_an ? dwt.an_tile1 : 16;
        return 0;
      }
    }
    // defined operands (the buffers are uninitialised before set_problem)
    for (int s = 0; s < nsets; ++s) {
      RC(fill_zero(X[s], LN, st));
      RC(fill_zero(Xt[s], LN, st));
      RC(fill_zero(U[s], LN * P, st));
      RC(fill_zero(zbuf(s), LN, st));
    }
    RC(fill_zero(beta, (size_t)L, st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MUFFIN_HIP_CHECK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return MUFFIN_E_HIP;
    }
    auto time_it = [&](auto launch, double* ms) -> int {
      RC(launch());  // warm-up (also loads the kernel)
      if (hipEventRecord(e0, st) != hipSuccess) return MUFFIN_E_HIP;
      for (int i = 0; i < reps; ++i) RC(launch());
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return MUFFIN_E_HIP;
      float f = 0.f;
      if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return MUFFIN_E_HIP;
      *ms = f / reps;
      return 0;
    };
    int rc = 0;
    const int tiles[2] = {16, 32};
    for (int v = 0; v < 2 && !rc; ++v) {
      dwt.syn_tile1 = tiles[v];
      rc = time_it([&] { return tune_synthesis(); }, &r->syn_ms[v]);
    }
    for (int v = 0; v < 2 && !rc && can_an; ++v) {
      dwt.an_tile1 = tiles[v];
      rc = time_it([&] { return tune_analysis(); }, &r->an_ms[v]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
      dwt.syn_tile1 = dwt.an_tile1 = 0;
      return rc;
    }
    dwt.syn_tile1 = r->syn_ms[1] < r->syn_ms[0] ? 32 : 16;
    dwt.an_tile1 = can_an ? (r->an_ms[1] < r->an_ms[0] ? 32 : 16) : 0;
    r->syn_tile1 = dwt.syn_tile1;
    r->an_tile1 = can_an ? dwt.an_tile1 : in_use(0, 0);
    std::lock_guard<std::mutex> lk(tune_table().mu);
    tune_table().shapes[key] = {dwt.syn_tile1, dwt.an_tile1};
    return 0;
  }

  // Quality against a known sky (Section 4.1): SNR = 10 log10(|x*|^2 /
  // |x* - X|^2) and WMSE = |H (x* - X)|^2 / (N L), FP64 sums.  G and S of
  // the primal set are rebuilt at the start of every iteration, so between
  // iterations they hold x* - X and its image under H.
  int quality(const void* truth, double* snr_db, double* wmse) override {
    if (!have_problem) return MUFFIN_E_STATE;
    if (!truth) return MUFFIN_E_INVAL;
    const T* xs = static_cast<const T*>(truth);
    const int nb = dot_blocks();
    RC(diff_sq<T>(xs, X[0], LN, partials, nb, qsum, st));
    RC(axpy_copy<T>(G[0], xs, X[0], -1.0, LN, st));
    RC(chain1(G[0], S[0], 0));
    if (vis) {
      // |H e|^2 = <e, Re H^* H e> = <e, psf * e> (as the third sum)
      RC(dot_partials<T>(S[0], nullptr, G[0], LN, partials, nb, st));
      RC(reduce_to_buffer(partials, nb, qsum + 3, st));
    } else {
      RC(diff_sq<T>(S[0], S[0], LN, partials, nb, qsum + 2, st));
    }
    double h[4];
    MUFFIN_HIP_CHECK(hipMemcpyAsync(h, qsum, sizeof(h), hipMemcpyDeviceToHost, st));
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    if (snr_db)
      *snr_db = h[0] > 0 ? 10.0 * std::log10(h[1] / h[0]) : std::numeric_limits<double>::infinity();
    if (wmse) *wmse = h[3] / double(LN);
    return 0;
  }

  int weights(double* a, double* b) override {
    if (!have_problem) return MUFFIN_E_STATE;
    MUFFIN_HIP_CHECK(hipStreamSynchronize(st));
    if (a) MUFFIN_HIP_CHECK(hipMemcpy(a, alpha, sizeof(double) * N, hipMemcpyDeviceToHost));
    if (b) MUFFIN_HIP_CHECK(hipMemcpy(b, beta, sizeof(double) * L, hipMemcpyDeviceToHost));
    return 0;
  }

  int op(int kind, const void* in, void* out) override {
    if (!in || !out) return MUFFIN_E_INVAL;
    const T* x = static_cast<const T*>(in);
    T* y = static_cast<T*>(out);
    switch (kind) {
      case 0:
      case 1:
      case 2:
        if (!have_problem) return MUFFIN_E_STATE;
        return chain1(x, y, kind);
      case 3: {
        AnalysisIO<T> io{};
        io.nsets = 1;
        io.z_a[0] = x;
        io.c1_sel[0] = SEL_ONE;
        io.c2_sel[0] = SEL_ZERO;
        io.U[0] = y;
        io.tmp0[0] = tmp0(0);
        io.tmp1[0] = tmp1(0);
        io.pure = 1;
        io.pure_scale = star ? 1.0 : 1.0 / std::sqrt((double)P);
        return star ? starlet_analysis(spl, io, nullptr, st) : dwt_analysis(dwt, io, nullptr, st);
      }
      case 4: {
        SynthesisIO<T> io{};
        io.nsets = 1;
        io.Ua[0] = x;
        io.S[0] = y;
        io.tmp0[0] = tmp0(0);
        io.tmp1[0] = tmp1(0);
        io.pure = 1;
        return star ? starlet_synthesis(spl, io, st) : dwt_synthesis(dwt, io, nullptr, st);
      }
      case 5:
      case 6: {
        DctIO<T> io{};
        io.nsets = 1;
        io.z_a[0] = x;
        io.V[0] = y;
        io.pure = kind == 5 ? 1 : 2;
        return dct_update(dct, io, nullptr, st);
      }
      default:
        return MUFFIN_E_INVAL;
    }
  }
};

}  // namespace

struct muffin_handle {
  muffin_config cfg;
  hipStream_t stream;
  std::unique_ptr<ImplBase> impl;
};

namespace muffin {
int handle_run_chunk(muffin_handle* h, int iters, bool check) {
  return h->impl->run_chunk(iters, check);
}
int handle_chunk_poll(muffin_handle* h, int* done, double* rel) {
  return h->impl->chunk_poll(done, rel);
}
size_t handle_workspace_bytes(const muffin_config* c) { return workspace_bytes_of(c); }
void handle_preset_beta_H(muffin_handle* h, double v) { h->impl->preset_beta_H(v); }
}  // namespace muffin

// Many independent cubes as one graph: one chunk of iterations of every
// handle, captured with a fork/join over the handles' streams (the cubes'
// kernels run concurrently) and replayed per chunk.
struct muffin_batch {
  std::vector<muffin_handle*> hs;
  int chunk = 0;
  hipStream_t root = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool captured = false;

  int capture() {
    // one eager chunk first: every kernel attribute is set outside the
    // capture, and the graph starts from the same pointer parity
    for (auto* h : hs) RC(h->impl->iterate_n(chunk));
    for (auto* h : hs) MUFFIN_HIP_CHECK(hipStreamSynchronize(h->stream));
    MUFFIN_HIP_CHECK(hipStreamBeginCapture(root, hipStreamCaptureModeRelaxed));
    int rc = 0;
    if (hipEventRecord(fork, root) != hipSuccess) rc = MUFFIN_E_HIP;
    for (size_t i = 0; !rc && i < hs.size(); ++i)
      if (hipStreamWaitEvent(hs[i]->stream, fork, 0) != hipSuccess) rc = MUFFIN_E_HIP;
    for (size_t i = 0; !rc && i < hs.size(); ++i) rc = hs[i]->impl->iterate_n(chunk);
    for (size_t i = 0; !rc && i < hs.size(); ++i) {
      if (hipEventRecord(joins[i], hs[i]->stream) != hipSuccess ||
          hipStreamWaitEvent(root, joins[i], 0) != hipSuccess)
        rc = MUFFIN_E_HIP;
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(root, &g);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : MUFFIN_E_HIP;
    }
    graph = g;
    MUFFIN_HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    captured = true;
    return 0;
  }
};

extern "C" {

int muffin_batch_create(muffin_batch** b, muffin_handle* const* handles, int32_t count,
                        int32_t chunk, void* stream) {
  if (!b || !handles || count < 1 || !stream) return MUFFIN_E_INVAL;
  *b = nullptr;
  // the chunk: even (pointer swaps return to the captured state) and a
  // multiple of every adaptive handle's Delta (theta updates at the same
  // iterations as an uninterrupted run)
  long long need = 2;
  for (int i = 0; i < count; ++i) {
    muffin_handle* h = handles[i];
    // (handles may share streams, also with the root: their work then
    // serialises on that stream inside the graph)
    if (!h || !h->stream) return MUFFIN_E_INVAL;
    if (!h->impl->ready()) return MUFFIN_E_STATE;
    if (h->cfg.sure) need = std::lcm(need, (long long)h->cfg.delta_period);
  }
  if (chunk <= 0) chunk = (int32_t)need;
  if (chunk % need != 0) return MUFFIN_E_INVAL;
  for (int i = 0; i < count; ++i)
    if (handles[i]->impl->iters_done() % chunk != 0) return MUFFIN_E_STATE;
  std::unique_ptr<muffin_batch> bb(new (std::nothrow) muffin_batch());
  if (!bb) return MUFFIN_E_NOMEM;
  bb->hs.assign(handles, handles + count);
  bb->chunk = chunk;
  bb->root = static_cast<hipStream_t>(stream);
  if (hipEventCreateWithFlags(&bb->fork, hipEventDisableTiming) != hipSuccess) return MUFFIN_E_HIP;
  bb->joins.resize(count, nullptr);
  for (auto& e : bb->joins)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MUFFIN_E_HIP;
  *b = bb.release();
  return MUFFIN_OK;
}

int muffin_batch_run(muffin_batch* b, int32_t chunks) {
  if (!b || chunks < 0) return MUFFIN_E_INVAL;
  if (chunks == 0) return MUFFIN_OK;
  int done = 0;
  if (!b->captured) {
    RC(b->capture());  // one chunk run eagerly, the next only recorded
    for (auto* h : b->hs) h->impl->advance(-b->chunk);  // (recording advanced them)
    done = 1;
  }
  for (; done < chunks; ++done) {
    MUFFIN_HIP_CHECK(hipGraphLaunch(b->exec, b->root));
    for (auto* h : b->hs) h->impl->advance(b->chunk);
  }
  return MUFFIN_OK;
}

int muffin_batch_destroy(muffin_batch* b) {
  if (!b) return MUFFIN_E_INVAL;
  if (b->root) (void)hipStreamSynchronize(b->root);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto e : b->joins)
    if (e) (void)hipEventDestroy(e);
  delete b;
  return MUFFIN_OK;
}

}  // extern "C"

extern "C" {

int muffin_default_config(muffin_config* c, int32_t n, int32_t L) {
  if (!c) return MUFFIN_E_INVAL;
  std::memset(c, 0, sizeof(*c));
  c->n = n;
  c->L = L;
  c->n_bases = 8;
  int J = 3;
  while (J > 1 && (n >> J) < 1) --J;
  c->levels = J;
  c->mode = MUFFIN_F64;
  c->mu = 1.0;
  c->gamma = 1.0;
  c->sigma = 10.0;
  c->tau = 0.0;
  c->tau_rule = MUFFIN_TAU_OPNORM;
  c->rho = 0.99;
  c->eps_w = 1e-6;
  c->sure = 0;
  c->delta_period = 10;
  c->eta_mu = 1e-3;
  c->eta_gamma = 1e-3;
  c->eps_fd = 0.0;
  c->sigma_w = 0.0;
  c->deriv_reset = 1;
  c->pi_iters = 200;
  c->pi_tol = 1e-10;
  c->stop_rel = 0.0;
  c->check_every = 10;
  return MUFFIN_OK;
}

size_t muffin_workspace_bytes(const muffin_config* c) {
  if (validate(c) != MUFFIN_OK) return 0;
  return workspace_bytes_of(c);
}

int muffin_create(muffin_handle** h, const muffin_config* cfg, void* stream) {
  if (!h) return MUFFIN_E_INVAL;
  *h = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  std::unique_ptr<muffin_handle> hh(new (std::nothrow) muffin_handle());
  if (!hh) return MUFFIN_E_NOMEM;
  hh->cfg = *cfg;
  hh->stream = static_cast<hipStream_t>(stream);
  if (cfg->mode == MUFFIN_F64)
    hh->impl.reset(new (std::nothrow) Impl<double>(*cfg, hh->stream));
  else
    hh->impl.reset(new (std::nothrow) Impl<float>(*cfg, hh->stream));
  if (!hh->impl) return MUFFIN_E_NOMEM;
  rc = hh->impl->init();
  if (rc) return rc;
  *h = hh.release();
  return MUFFIN_OK;
}

int muffin_set_problem(muffin_handle* h, const void* dirty, const void* psf, const double* alpha,
                       const double* beta, const void* delta) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->set_problem(dirty, psf, alpha, beta, delta);
}

int muffin_run(muffin_handle* h, int32_t iters, muffin_report* report) {
  if (!h) return MUFFIN_E_INVAL;
  int rc = h->impl->run(iters);
  if (rc) return rc;
  if (report) return h->impl->report(report);
  return MUFFIN_OK;
}

int muffin_get_sky(muffin_handle* h, void* x_out) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->get_state(0, 0, x_out);
}

int muffin_get_state(muffin_handle* h, int32_t which, int32_t set, void* out) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->get_state(which, set, out);
}

int muffin_set_state(muffin_handle* h, int32_t which, int32_t set, const void* in) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->set_state(which, set, in);
}

int muffin_get_history(muffin_handle* h, double* rows, int32_t max_rows) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->history(rows, max_rows);
}

int muffin_get_weights(muffin_handle* h, double* alpha, double* beta) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->weights(alpha, beta);
}

int muffin_get_report(muffin_handle* h, muffin_report* report) {
  if (!h || !report) return MUFFIN_E_INVAL;
  return h->impl->report(report);
}

int muffin_autotune(muffin_handle* h, int32_t reps, muffin_tune_result* out) {
  if (!h || !out || reps < 1) return MUFFIN_E_INVAL;
  return h->impl->autotune(reps, out);
}

int muffin_quality(muffin_handle* h, const void* truth, double* snr_db, double* wmse) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->quality(truth, snr_db, wmse);
}

int muffin_set_initial(muffin_handle* h, const void* x0) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->set_initial(x0);
}

size_t muffin_state_bytes(muffin_handle* h) {
  if (!h) return 0;
  return h->impl->state_bytes();
}

int muffin_state_save(muffin_handle* h, void* host_buf, size_t bytes) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->state_save(host_buf, bytes);
}

int muffin_state_load(muffin_handle* h, const void* host_buf, size_t bytes) {
  if (!h) return MUFFIN_E_INVAL;
  return h->impl->state_load(host_buf, bytes);
}

int muffin_solve(const muffin_config* cfg, const void* dirty, const void* psf,
                 const double* alpha, const double* beta, const void* delta, const void* x0,
                 int32_t iters, void* sky_out, muffin_report* report, void* stream) {
  if (!sky_out) return MUFFIN_E_INVAL;
  muffin_handle* h = nullptr;
  int rc = muffin_create(&h, cfg, stream);
  if (rc) return rc;
  rc = muffin_set_problem(h, dirty, psf, alpha, beta, delta);
  if (!rc && x0) rc = muffin_set_initial(h, x0);
  if (!rc) rc = muffin_run(h, iters, report);
  if (!rc) rc = muffin_get_sky(h, sky_out);
  if (!rc && hipStreamSynchronize(h->stream) != hipSuccess) rc = MUFFIN_E_HIP;
  muffin_destroy(h);
  return rc;
}

}  // extern "C"

// ---- allocation-free solve ----
// One static device array per GPU holds every buffer and table of the solve
// (the handle's state, the transfer functions, the FFT and DCT tables and
// the set-up temporaries), carved in order by a Region.  Its device address
// on each GPU is looked up once, with that GPU current; host code never
// passes the array's own name to a kernel or a copy.
namespace {
constexpr size_t kNoAllocBytes = size_t(MUFFIN_NOALLOC_BYTES);
constexpr int kNoAllocDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
struct NoAllocSlot {
  std::mutex mu;         // serialises the solves on one GPU
  void* ptr = nullptr;   // device address of `scratch` on that GPU
};
NoAllocSlot g_noalloc[kNoAllocDevices];

// Bytes the solve of *c takes from the array: the resident workspace, the
// FFT and DCT tables, a margin for the 256-byte rounding of every piece, and
// the larger of the two set-up temporaries (the PSF spectra, then the FP64
// power iteration with its own plan in the FP32 forms).
size_t noalloc_need(const muffin_config* c) {
  const size_t n = c->n, L = c->L, N = n * n, LN = L * N;
  const int es = c->mode == MUFFIN_F64 ? 8 : 4;
  const int kind = es == 8 ? DCT_F64 : (c->mode == MUFFIN_F32_BF16DCT ? DCT_BF16X3 : DCT_F32);
  const size_t resident = workspace_bytes_of(c) + fft_plan_bytes((int)n, (int)L, es) +
                          dct_plan_bytes((int)L, kind, es) + 128 * 256;
  const size_t spec = region_round((size_t)2 * es * L * (n + 1) * 2 * n);
  size_t pi = 0;
  if (c->tau <= 0 || c->pi_iters > 0) {
    pi = 2 * region_round(8 * LN) + 2 * region_round(16 * LN) + region_round(24 * L);
    if (es == 4)
      pi += fft_plan_bytes((int)n, (int)L, 8) + region_round(8 * 4 * LN) +
            region_round((size_t)16 * L * (n + 1) * 2 * n);
  }
  return resident + std::max(spec, pi);
}
}  // namespace

extern "C" {

int muffin_solve_noalloc(const muffin_config* cfg, const void* dirty, const void* psf,
                         const double* alpha, const double* beta, const void* delta,
                         const void* x0, int32_t iters, void* sky_out, muffin_report* report,
                         void* stream) {
  if (!sky_out || !dirty || !psf || iters < 0) return MUFFIN_E_INVAL;
  int rc = validate(cfg);
  if (rc) return rc;
  if (noalloc_need(cfg) > kNoAllocBytes) return MUFFIN_E_SCRATCH;
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kNoAllocDevices) return MUFFIN_E_HIP;
  NoAllocSlot& slot = g_noalloc[d];
  std::lock_guard<std::mutex> lock(slot.mu);
  if (!slot.ptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return MUFFIN_E_HIP;
    }
    slot.ptr = ptr;
  }
  Region region;
  region.base = static_cast<char*>(slot.ptr);
  region.cap = kNoAllocBytes;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the same handle and calls as muffin_solve; the Impl's buffers come from
  // the region (its destructor rewinds it), and set_problem zeroes the
  // state, so nothing depends on what an earlier call left in the array
  std::unique_ptr<ImplBase> impl;
  if (cfg->mode == MUFFIN_F64) {
    auto* m = new (std::nothrow) Impl<double>(*cfg, st);
    if (m) m->region = &region;
    impl.reset(m);
  } else {
    auto* m = new (std::nothrow) Impl<float>(*cfg, st);
    if (m) m->region = &region;
    impl.reset(m);
  }
  if (!impl) return MUFFIN_E_NOMEM;
  rc = impl->init();
  if (!rc) rc = impl->set_problem(dirty, psf, alpha, beta, delta);
  if (!rc && x0) rc = impl->set_initial(x0);
  if (!rc) rc = impl->run(iters);
  if (!rc && report) rc = impl->report(report);
  if (!rc) rc = impl->get_state(0, 0, sky_out);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = MUFFIN_E_HIP;
  impl.reset();
  // a region that ran out maps to the size error, not to an allocation error
  if (rc == MUFFIN_E_NOMEM) rc = MUFFIN_E_SCRATCH;
  return rc;
}

int muffin_destroy(muffin_handle* h) {
  if (!h) return MUFFIN_E_INVAL;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return MUFFIN_OK;
}

int muffin_set_timing(muffin_handle* h, int32_t on) {
  if (!h) return MUFFIN_E_INVAL;
  Timer& t = h->impl->timer();
  RC(t.collect(h->impl->stream()));
  t.reset();
  t.on = on != 0;
  return MUFFIN_OK;
}

int muffin_get_timing(muffin_handle* h, double* ms, int64_t* calls, int32_t max_stages) {
  if (!h) return MUFFIN_E_INVAL;
  Timer& t = h->impl->timer();
  RC(t.collect(h->impl->stream()));
  double total[ST_COUNT];
  long long ncalls[ST_COUNT];
  for (int i = 0; i < ST_COUNT; ++i) {
    total[i] = t.ms[i];
    ncalls[i] = t.calls[i];
  }
  // the chain's time is the sum of its passes (timed one by one)
  for (int i = ST_FFT_R1; i <= ST_FFT_R3; ++i) total[ST_FFT] += t.ms[i];
  ncalls[ST_FFT] = std::max(ncalls[ST_FFT], ncalls[ST_FFT_R1]);
  for (int i = 0; i < ST_COUNT && i < max_stages; ++i) {
    if (ms) ms[i] = total[i];
    if (calls) calls[i] = ncalls[i];
  }
  return ST_COUNT;
}

const char* muffin_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : "";
}

const char* muffin_strerror(int code) {
  switch (code) {
    case MUFFIN_OK: return "ok";
    case MUFFIN_E_INVAL: return "invalid argument or configuration";
    case MUFFIN_E_SHAPE: return "unsupported size";
    case MUFFIN_E_NOMEM: return "device allocation failed";
    case MUFFIN_E_SCRATCH: return "problem too large for the static workspace of muffin_solve_noalloc";
    case MUFFIN_E_NONFINITE: return "non-finite value in an input cube";
    case MUFFIN_E_HIP: return "HIP runtime error";
    case MUFFIN_E_STATE: return "call out of order";
    case MUFFIN_E_BUSY: return "serving queue full";
    default: return "unknown error";
  }
}

int muffin_op_H(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(0, in, out) : MUFFIN_E_INVAL;
}
int muffin_op_HT(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(1, in, out) : MUFFIN_E_INVAL;
}
int muffin_op_HTH(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(2, in, out) : MUFFIN_E_INVAL;
}
int muffin_op_Ws(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(3, in, out) : MUFFIN_E_INVAL;
}
int muffin_op_WsT(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(4, in, out) : MUFFIN_E_INVAL;
}
int muffin_op_dct(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(5, in, out) : MUFFIN_E_INVAL;
}
int muffin_op_idct(muffin_handle* h, const void* in, void* out) {
  return h ? h->impl->op(6, in, out) : MUFFIN_E_INVAL;
}

}  // extern "C"
