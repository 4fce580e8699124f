/*
 * libmuffin -- MUFFIN wideband deconvolution with ADA-PT parameter tuning
 * (Ammanouil, Ferrari, Flamary, Ferrari, Mary, arXiv 1905.08468) on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2.1, eqs. `model`, `probopt`, `RegAll`): given the dirty
 * images y_l and PSFs of L bands, estimate the sky cube X >= 0 minimising
 *   sum_l 1/2 ||y_l - H_l x_l||^2 + sum_l mu_l ||W_s x_l||_1
 *                                 + sum_n gamma_n ||W_lambda x^n||_1,
 * with mu_l = mu beta_l, gamma_n = gamma alpha_n (eq. `2regpar`), by the
 * primal-dual iteration of Algorithm 2, optionally with the SURE-driven
 * update of theta = (mu, gamma) every Delta iterations (Algorithm 5).
 *
 * Conventions
 *  - Cubes are band-major, contiguous: element (l, i, j) at l*n*n + i*n + j.
 *    The PSF cube is [L][2n][2n] with the PSF centre at (n, n); H_l is the
 *    linear convolution with it, restricted to the n x n image window.
 *  - Cube pointers are DEVICE pointers on the GPU current when the handle was
 *    created, in the working type of the handle's mode (double for
 *    MUFFIN_F64, float otherwise).  The caller owns them.  Work is enqueued on
 *    the handle's stream; calls return without waiting unless stated.
 *  - alpha/beta weight pointers are HOST double arrays (copied at the call).
 *  - The library owns only its workspace, freed by muffin_destroy.
 *  - Every function returns an int status: 0 = MUFFIN_OK, < 0 an error code
 *    (muffin_strerror); nothing aborts or exits.  On error no output has been
 *    written, except where noted.
 *  - A handle must not be used from two threads at once; distinct handles are
 *    independent.
 */
#ifndef MUFFIN_H
#define MUFFIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct muffin_handle muffin_handle;

enum {
  MUFFIN_OK = 0,
  MUFFIN_E_INVAL = -1,     /* bad configuration value or null pointer */
  MUFFIN_E_SHAPE = -2,     /* unsupported size (n, L, levels, bases) */
  MUFFIN_E_NOMEM = -3,     /* device allocation failed; nothing allocated */
  MUFFIN_E_NONFINITE = -4, /* NaN or Inf in an input cube */
  MUFFIN_E_HIP = -5,       /* HIP runtime error */
  MUFFIN_E_STATE = -6,     /* call out of order (e.g. run before set_problem) */
  MUFFIN_E_BUSY = -7,      /* serving queue full */
  MUFFIN_E_SCRATCH = -8    /* too large for the static workspace of
                              muffin_solve_noalloc */
};

/* Arithmetic forms.  F64: everything in double.  F32: FFT, wavelet,
 * element-wise and DCT work in float; power iteration, SURE/SUGAR sums and the
 * theta update stay in double.  F32_BF16DCT: as F32 with the spectral DCT
 * products on bf16 MFMA with a hi+lo split and float accumulation. */
enum { MUFFIN_F64 = 0, MUFFIN_F32 = 1, MUFFIN_F32_BF16DCT = 2 };

/* Step-size rules (Section 2.2): tau = rho / (beta_H/2 + sigma K) with
 * K = max_l mu_l^2 + max_n gamma_n^2 (OPNORM, the operator norm of the dual
 * operators, ||W_s|| = ||W_lambda|| = 1) or the printed sum
 * K = sum_l mu_l^2 + sum_n gamma_n^2 (PAPER_SUM). */
enum { MUFFIN_TAU_OPNORM = 0, MUFFIN_TAU_PAPER_SUM = 1 };

/* Spatial dictionaries W_s (Section 2.1 names both).  DAUBECHIES: the union
 * of the db1..dbP bases, J levels each, scaled by 1/sqrt(P) (a Parseval
 * frame, ||W_s|| = 1; the paper's experiments).  STARLET: the isotropic
 * undecimated wavelet transform with J scales (B3-spline filter, a trous,
 * periodic): J + 1 planes per band (the scales, then the coarse plane),
 * unscaled; the step rule then uses ||W_s||^2 > 1, computed exactly. */
enum { MUFFIN_DICT_DAUBECHIES = 0, MUFFIN_DICT_STARLET = 1 };

typedef struct {
  int32_t n;            /* image side, power of two, 8 <= n <= 2048 */
  int32_t L;            /* bands, 1 <= L <= 256 */
  int32_t n_bases;      /* P: db1..dbP in W_s, 1..8 (paper: 8) */
  int32_t levels;       /* J: decomposition levels, 1 <= J, n / 2^J >= 1 */
  int32_t mode;         /* MUFFIN_F64 / MUFFIN_F32 / MUFFIN_F32_BF16DCT */
  double mu, gamma;     /* theta at start (eq. `2regpar`) */
  double sigma;         /* dual step (paper: 10) */
  double tau;           /* > 0: fixed primal step; <= 0: from tau_rule */
  int32_t tau_rule;     /* MUFFIN_TAU_OPNORM or MUFFIN_TAU_PAPER_SUM */
  double rho;           /* safety factor of the tau rule, in (0, 1) */
  double eps_w;         /* epsilon of the weight rule (Section 2.1) */
  int32_t sure;         /* 0: plain MUFFIN, fixed theta; 1: ADA-PT (Alg. 5) */
  int32_t delta_period; /* Delta: theta update period (paper: 10) */
  double eta_mu;        /* gradient steps of eq. `adaptgrad` */
  double eta_gamma;
  double eps_fd;        /* epsilon of SURE-FDMC (eq. `PSURE0`), > 0 if sure */
  double sigma_w;       /* noise standard deviation, > 0 if sure */
  int32_t deriv_reset;  /* 1: derivative states restart at each theta update */
  int32_t pi_iters;     /* max power iterations for beta_H (if tau <= 0) */
  double pi_tol;        /* relative change stopping the power iteration */
  double stop_rel;      /* > 0: muffin_run stops once the relative change of
                           the Y trajectory over one iteration,
                           max(|X^k - X^(k-1)| / |X^k|,
                               sqrt(|dU|^2 + |dV|^2) / sqrt(|U^k|^2 + |V^k|^2)),
                           is <= stop_rel (checked every check_every
                           iterations; FP64 sums).  The paper fixes no
                           stopping rule; this is the relative primal-dual
                           residual of the serving form.  0: run exactly
                           the requested iterations. */
  int32_t check_every;  /* iterations between checks of stop_rel, >= 1 */
  int32_t dictionary;   /* MUFFIN_DICT_DAUBECHIES or MUFFIN_DICT_STARLET; with
                           STARLET, levels = J scales (1..5) and n_bases is
                           unused: U and the masks hold J + 1 planes per band */
  int32_t visibilities; /* 0: dirty images (eq. `model`); 1: visibilities
                           (Section 1: only the direct operator changes).
                           muffin_set_problem then takes, from
                           muffin_vis_prepare, the back-projected cube
                           Re H^* v as `dirty`, the point spread function as
                           `psf` and the back-projected probe Re H^* delta as
                           `delta`; the gradient is psf * x - dirty (the
                           windowed convolution by the PSF is Re H^* H) */
  double vis_norm2;     /* visibilities: |v|^2 over all bands (the residual
                           |v - H x|^2 of PSURE is computed from it) */
  double vis_count;     /* visibilities: number of real measurements (two per
                           complex sample), > 0 with sure */
} muffin_config;

typedef struct {
  int32_t iters_done;     /* iterations completed since muffin_set_problem */
  int32_t theta_updates;  /* ADA-PT updates applied */
  double mu, gamma, tau;  /* current values */
  double beta_H;          /* Lipschitz constant used by the tau rule */
  double psure;           /* PSURE-FDMC at the last update (eq. `PSURE0`) */
  double sugar_mu;        /* SUGAR-FDMC at the last update (eq. `SUGAR`) */
  double sugar_gamma;
  double res2;            /* ||Y - H X||^2 at the last update */
  double last_rel_change; /* last checked relative change (stop_rel), or -1 */
  int32_t stopped;        /* 1: the last muffin_run ended on stop_rel */
} muffin_report;

/* Fills *cfg with the paper's defaults for an n x n x L cube: P = 8 bases,
 * J = 3 levels (fewer when n is small), sigma = 10, Delta = 10, OPNORM rule,
 * rho = 0.99, eps_w = 1e-6, plain MUFFIN (sure = 0), mu = gamma = 1, no
 * stopping rule (stop_rel = 0, check_every = 10), the Daubechies union. */
int muffin_default_config(muffin_config* cfg, int32_t n, int32_t L);

/* Device bytes the handle will hold for *cfg (admission control).  Returns 0
 * for an invalid configuration.  muffin_set_problem also takes temporary
 * device memory for its power iteration, freed before it returns: two FP64
 * cubes and two FP64 half spectra (about 6 L n^2 doubles), plus in the FP32
 * forms an FP64 copy of the PSFs and of their transfer functions (about
 * 8 L n^2 doubles more). */
size_t muffin_workspace_bytes(const muffin_config* cfg);

/* Creates a handle: validates *cfg (E_INVAL / E_SHAPE), allocates the
 * workspace (E_NOMEM, nothing left allocated), builds FFT, wavelet and DCT
 * plans.  stream: hipStream_t used for all work (may be 0). */
int muffin_create(muffin_handle** h, const muffin_config* cfg, void* stream);

/* Sets the problem and runs the set-up of Section 2 (once per solve):
 * transfer functions from the PSFs, weights, beta_H (power iteration, FP64),
 * tau, zero state.
 *   dirty: [L][n][n] device, psf: [L][2n][2n] device (working type).
 *   alpha: host double[n*n] or NULL -> 1/(||W_lambda y^n|| + eps_w);
 *   beta:  host double[L]   or NULL -> 1/(||W_s y_l|| + eps_w)
 *          (the weight rule of Section 2.1 with the dirty cube as the
 *           initial estimate).  The orthonormal DCT and the Daubechies
 *           union (a Parseval frame) preserve norms, so those two are plain
 *           norms of y; the starlet does not, and beta then applies it.
 *   delta: [L][n][n] device N(0,1) probe, required when cfg->sure.
 * Checks the cubes for NaN/Inf (E_NONFINITE).  Synchronises the stream. */
int muffin_set_problem(muffin_handle* h, const void* dirty, const void* psf,
                       const double* alpha, const double* beta, const void* delta);

/* Runs `iters` iterations (Algorithm 2, or Algorithm 5 when sure), resuming
 * from the current state.  If report != NULL the stream is synchronised and
 * *report filled; otherwise the call only enqueues work (with stop_rel > 0
 * it synchronises at every check and may stop early). */
int muffin_run(muffin_handle* h, int32_t iters, muffin_report* report);

/* Initial estimate X^(0) = x0 (device cube [L][n][n]) for both trajectories
 * instead of 0 (Algorithm 5's initialisation; dual and derivative states
 * stay zero).  Call after muffin_set_problem. */
int muffin_set_initial(muffin_handle* h, const void* x0);

/* Checkpoint of the iteration state (X, U, V, T of every state set, the
 * device scalars theta, tau, sums, the iteration and update counters and the
 * theta history) in a host buffer of muffin_state_bytes(h) bytes.  Loading
 * requires a handle of the same configuration with the same problem set;
 * mismatches return E_SHAPE, a foreign buffer E_INVAL.  Both synchronise the
 * stream.  A run resumed from a checkpoint continues exactly as the
 * uninterrupted run. */
size_t muffin_state_bytes(muffin_handle* h);
int muffin_state_save(muffin_handle* h, void* host_buf, size_t bytes);
int muffin_state_load(muffin_handle* h, const void* host_buf, size_t bytes);

/* One call: create, set_problem (weights NULL -> rule of Section 2.1),
 * optional x0, run `iters` iterations (or to cfg->stop_rel), copy the sky to
 * sky_out (device [L][n][n]), destroy.  Synchronises `stream`. */
int muffin_solve(const muffin_config* cfg, const void* dirty, const void* psf,
                 const double* alpha, const double* beta, const void* delta, const void* x0,
                 int32_t iters, void* sky_out, muffin_report* report, void* stream);

/* Allocation-free one-call solve, for callers that cannot allocate device
 * memory: code that runs while its caller captures a HIP graph of other
 * work, tight serving loops, harnesses that forbid hipMalloc.  Arguments,
 * results and kernels are those of muffin_solve, but every device buffer and
 * table of the solve (state, transfer functions, FFT and DCT tables, set-up
 * temporaries) is carved from one static device array of
 * MUFFIN_NOALLOC_BYTES bytes per GPU, which the library holds from its
 * loading until the process ends; no hipMalloc, hipFree, hipHostMalloc or
 * other allocating call is made (host memory for a few small structures
 * aside).
 *   Size limit: a configuration whose buffers, tables and set-up temporaries
 *   do not fit returns MUFFIN_E_SCRATCH before any device work (for example,
 *   plain FP32 solves fit up to 128 x 128 x 32 or 256 x 256 x 8 with the
 *   power iteration, ADA-PT in FP32 up to 128 x 128 x 8; passing tau > 0
 *   and pi_iters = 0 skips the power iteration's temporaries).
 *   Sharing: every call on a GPU uses that GPU's one array, which keeps what
 *   the last call left; each solve initialises everything it reads.  Calls
 *   on one GPU are serialised by a per-GPU lock and return only after
 *   `stream` has finished the solve; work the caller enqueues elsewhere that
 *   overlaps a call must not touch its outputs.
 * Synchronises `stream`. */
#define MUFFIN_NOALLOC_BYTES (128u << 20)
int muffin_solve_noalloc(const muffin_config* cfg, const void* dirty, const void* psf,
                         const double* alpha, const double* beta, const void* delta,
                         const void* x0, int32_t iters, void* sky_out, muffin_report* report,
                         void* stream);

/* Copies the current sky estimate X (Y trajectory) to x_out [L][n][n]. */
int muffin_get_sky(muffin_handle* h, void* x_out);

/* State access for checking and checkpointing.
 *   which: 0 = X, 1 = U ([L][P][n][n]), 2 = V, 3 = T.
 *   set:   0 = Y trajectory, 1 = Ybar trajectory, 2/3 = d/dmu, d/dgamma of
 *          the Y trajectory, 4/5 = d/dmu, d/dgamma of the Ybar trajectory. */
int muffin_get_state(muffin_handle* h, int32_t which, int32_t set, void* out);
int muffin_set_state(muffin_handle* h, int32_t which, int32_t set, const void* in);

/* Per-update history rows (k, mu, gamma, tau, sugar_mu, sugar_gamma, psure,
 * res2), at most max_rows; returns the number of rows available. */
int muffin_get_history(muffin_handle* h, double* rows, int32_t max_rows);

/* Copies the weights in use (host arrays alpha[n*n], beta[L]) and the
 * current report without running anything.  Synchronises the stream. */
int muffin_get_weights(muffin_handle* h, double* alpha, double* beta);
int muffin_get_report(muffin_handle* h, muffin_report* report);

/* Optional device timing of the iteration's stages with HIP events recorded
 * on the handle's stream (for measurement; adds event records, no sync).
 * muffin_set_timing clears the totals.  muffin_get_timing synchronises the
 * stream and writes, per stage, the total milliseconds and the number of
 * timed calls; it returns the number of stages.  Stage names come from
 * muffin_stage_name (e.g. "analysis_l1_deriv" is one kernel launch: level-1
 * analysis + dual update of the four derivative sets). */
int muffin_set_timing(muffin_handle* h, int32_t on);
int muffin_get_timing(muffin_handle* h, double* ms, int64_t* calls, int32_t max_stages);
const char* muffin_stage_name(int32_t stage);

int muffin_destroy(muffin_handle* h);
const char* muffin_strerror(int code);

/* ---- serving: continuous batching of independent solves ----
 * A server owns a worker thread and a pool of handles on the device that is
 * current at creation.  Submitted solves wait in a FIFO queue; the worker
 * admits the head request as soon as a slot (max_active) and its workspace
 * (muffin_workspace_bytes, within hbm_budget) are free, reusing an idle
 * handle of the same configuration or creating one (idle handles of other
 * configurations are released when memory is needed).  Admitted solves keep
 * their state resident and iterate in chunks on streams of their own, so
 * their kernels overlap on the device; a solve ends when cfg->stop_rel is
 * met (checked every cfg->check_every iterations) or after max_iters.
 * Results do not depend on what else runs: each solve executes exactly the
 * kernels of a lone muffin_run.
 *
 * Inputs are device pointers (working type of cfg->mode) that the caller
 * keeps valid until the request has been admitted (status RUNNING or later);
 * alpha/beta (host, may be NULL) are copied at submission.  sky_out
 * (device [L][n][n]) is written when the request completes.  Latency is
 * measured from submission to completion on the host's steady clock. */
typedef struct muffin_server muffin_server;

typedef struct {
  size_t hbm_budget;   /* bytes for the pooled handles; 0: 85% of the free memory */
  int32_t max_active;  /* solves iterating at once, 1..64 */
  int32_t max_queue;   /* waiting requests before submit returns E_BUSY */
  int32_t chunk;       /* iterations per scheduling round of a solve without stop rule */
} muffin_server_config;

typedef struct {
  int32_t queued, active, completed, failed, cancelled;
  int32_t pooled_handles;
  size_t bytes_in_use, bytes_budget;
} muffin_server_stats;

enum {
  MUFFIN_REQ_QUEUED = 0,
  MUFFIN_REQ_RUNNING = 1,
  MUFFIN_REQ_DONE = 2,
  MUFFIN_REQ_CANCELLED = 3  /* a failed request reports its (negative) error code */
};

/* Defaults: hbm_budget 0, max_active 8, max_queue 4096, chunk 10. */
int muffin_server_default_config(muffin_server_config* sc);
int muffin_server_create(muffin_server** s, const muffin_server_config* sc);
/* Validates cfg (E_INVAL / E_SHAPE), refuses a solve whose workspace exceeds
 * the budget (E_NOMEM) or a full queue (E_BUSY); *ticket identifies it. */
int muffin_server_submit(muffin_server* s, const muffin_config* cfg, const void* dirty,
                         const void* psf, const double* alpha, const double* beta,
                         const void* delta, int32_t max_iters, void* sky_out, int64_t* ticket);
/* Non-blocking status; report and latency are filled once the request is done. */
int muffin_server_poll(muffin_server* s, int64_t ticket, int32_t* status, muffin_report* report,
                       double* latency_ms);
/* Blocks until the request leaves the queue/running states or timeout_ms
 * (< 0: no limit) passes; then as muffin_server_poll. */
int muffin_server_wait(muffin_server* s, int64_t ticket, double timeout_ms, int32_t* status,
                       muffin_report* report, double* latency_ms);
/* Cancels a queued request, or a running one at its next chunk boundary. */
int muffin_server_cancel(muffin_server* s, int64_t ticket);
int muffin_server_get_stats(muffin_server* s, muffin_server_stats* out);
/* Cancels what is queued or running, joins the worker, frees the pool. */
int muffin_server_destroy(muffin_server* s);

/* ---- batching: many independent cubes as one captured graph ----
 * `count` handles (any sizes, forms and configurations), each with its
 * problem set and a non-null stream, iterate together: one chunk of `chunk`
 * iterations of every handle is captured into one HIP graph with a
 * fork/join over the handles' streams (handles on different streams run
 * concurrently, handles sharing a stream one after the other) and each
 * later chunk is one graph launch on `stream` (the root).  chunk must be even and a
 * multiple of every adaptive handle's Delta (0: the least such value); each
 * handle must stand at a multiple of chunk iterations (e.g. just after
 * muffin_set_problem) and have timing off.  Results are those of the same
 * iterations run with muffin_run on each handle.
 * muffin_batch_run(b, chunks) enqueues chunks x chunk iterations of every
 * handle (the first call runs its first chunk directly and records the
 * graph); synchronise `stream` to wait.  Stopping rules are not evaluated
 * inside a batch. */
typedef struct muffin_batch muffin_batch;
int muffin_batch_create(muffin_batch** b, muffin_handle* const* handles, int32_t count,
                        int32_t chunk, void* stream);
int muffin_batch_run(muffin_batch* b, int32_t chunks);
int muffin_batch_destroy(muffin_batch* b);

/* ---- multi-start ADA-PT: one cube from several initial theta ----
 * Section 4.2 runs ADA-PT on one cube from four initial couples
 * theta^(0) = (mu, gamma) and follows theta, SUGAR, SNR and WMSE per
 * iteration.  A multi-start object holds one handle per start (cfg with
 * mu = mu0[i], gamma = gamma0[i]; cfg->sure may be 0 for a plain sweep of
 * fixed theta), each on a stream of its own, and iterates them as one batch
 * (one graph launch per chunk of every start, as muffin_batch_*).
 *   create:      starts in 1..64; mu0, gamma0 host double[starts], >= 0.
 *                stream: the root stream (NULL: one of its own).
 *   set_problem: as muffin_set_problem, once for all starts; the weights
 *                (alpha/beta NULL: the rule of Section 2.1) and beta_H are
 *                computed by the first start and handed to the others, so
 *                every start sees the same problem bit for bit.  chunk as
 *                in muffin_batch_create (0: the least valid value).
 *   run:         enqueues chunks x chunk iterations of every start on the
 *                root stream, ordered after earlier work on the starts'
 *                streams and before later work on them.
 *   quality:     per start, SNR and WMSE of Section 4.1 against the true
 *                sky (device [L][n][n], working type), FP64 sums;
 *                snr_db, wmse: host double[starts].  Synchronises.
 *   handle:      start i's handle for muffin_get_sky, muffin_get_history,
 *                muffin_get_report (owned by the object; NULL if i is out
 *                of range).
 * Start i's results equal those of a lone muffin_run of its configuration
 * on the same problem. */
typedef struct muffin_multistart muffin_multistart;
int muffin_multistart_create(muffin_multistart** m, const muffin_config* cfg, int32_t starts,
                             const double* mu0, const double* gamma0, void* stream);
int muffin_multistart_set_problem(muffin_multistart* m, const void* dirty, const void* psf,
                                  const double* alpha, const double* beta, const void* delta,
                                  int32_t chunk);
int muffin_multistart_run(muffin_multistart* m, int32_t chunks);
int muffin_multistart_quality(muffin_multistart* m, const void* truth, double* snr_db,
                              double* wmse);
muffin_handle* muffin_multistart_handle(muffin_multistart* m, int32_t i);
int muffin_multistart_destroy(muffin_multistart* m);

/* Reconstruction quality of the current sky estimate X against the true
 * sky x* (Section 4.1): *snr_db = 10 log10(|x*|^2 / |x* - X|^2) and
 * *wmse = |H (x* - X)|^2 / (N L), with |.| the Frobenius norm over the cube
 * and FP64 sums.  truth: device [L][n][n] of the working type.  Either
 * output may be NULL.  Requires muffin_set_problem; synchronises the stream. */
int muffin_quality(muffin_handle* h, const void* truth, double* snr_db, double* wmse);

/* ---- spectral unmixing of a reconstructed cube ----
 * Section 4.3 separates the sources of a reconstructed cube by their
 * spectra: k chosen endmember spectra (three in the paper, taken at bright
 * pixels) and, for every pixel n, the abundances
 *     a^n = argmin_{a >= 0} |x^n - E a|^2
 * (positivity-constrained least squares, x^n the pixel's spectrum, E the
 * L x k matrix whose columns are the spectra).  The solution is exact (all
 * 2^k supports are examined; FP64 arithmetic whatever the cube's type).
 *   plan_create: spectra host double[k][L] (row j = spectrum j), 1 <= k <= 4,
 *                k <= L; E_INVAL if a value is not finite or the spectra are
 *                linearly dependent.  Allocates a few KB of device memory.
 *   run:         cube device [L][n][n] (double if mode is MUFFIN_F64, else
 *                float); abund device [k][n][n] (same type); resid NULL or
 *                device [n][n] (same type) receiving |x^n - E a^n|^2,
 *                computed as |x^n|^2 - b^T a (b = E^T x^n): its absolute
 *                error is of order cond(E^T E) eps |x^n|^2.
 *                Enqueues one kernel on `stream` (NULL: the default stream);
 *                does not synchronise.
 * A plan may be used for any number of cubes with the same L. */
typedef struct muffin_unmix_plan muffin_unmix_plan;
int muffin_unmix_plan_create(muffin_unmix_plan** plan, const double* spectra, int32_t k,
                             int32_t L);
int muffin_unmix_run(const muffin_unmix_plan* plan, const void* cube, int32_t n, int32_t mode,
                     void* abund, void* resid, void* stream);
int muffin_unmix_plan_destroy(muffin_unmix_plan* plan);

/* ---- visibility-domain direct operator ----
 * Band l samples the sky's Fourier transform at K positions (u, v) in
 * cycles across the image (|u|, |v| < n/2), phases referred to the image
 * centre c = n/2: (H x)_k = sum_ij x[i][j] exp(-2 pi i (u_k (i-c) + v_k (j-c)) / n).
 * All sums are exact (no gridding approximation), in FP64, O(K) per output.
 *   uv:    device double [L][K][2];  vis, delta: device double [L][K][2]
 *          (real, imaginary parts).
 *   muffin_vis_prepare: dirty_out = Re H^* vis ([L][n][n]), psf_out = the
 *          real point spread function [L][2n][2n] with offset (0, 0) at
 *          (n, n), i.e. psf[n+a][n+b] = sum_k cos(2 pi (u_k a + v_k b) / n),
 *          delta_out = Re H^* delta (NULL with delta NULL); outputs in the
 *          working type of `mode`; *vis_norm2 = |vis|^2 (NULL: skipped;
 *          otherwise synchronises the stream).  These are the inputs of
 *          muffin_set_problem for a configuration with visibilities = 1.
 *   muffin_vis_degrid: vis_out ([L][K][2] double) = H x, x a device cube
 *          of the working type.  Enqueued on `stream`. */
int muffin_vis_prepare(const double* uv, const double* vis, const double* delta, int32_t L,
                       int32_t K, int32_t n, int32_t mode, void* dirty_out, void* psf_out,
                       void* delta_out, double* vis_norm2, void* stream);
int muffin_vis_degrid(const double* uv, int32_t L, int32_t K, int32_t n, int32_t mode,
                      const void* x, double* vis_out, void* stream);

/* ---- autotuner: wavelet tile shapes per size class ----
 * The FP32 level-1 wavelet kernels of the Daubechies union come in two tile
 * shapes, 16 x 16 and 32 x 32 (coefficients per subband side); both give
 * bit-identical results, their speed depends on the cube's size and the
 * number of state sets.  muffin_autotune times both shapes of the level-1
 * synthesis and analysis launches (as the iteration issues them, `reps`
 * launches each after a warm-up) on the handle's own buffers, keeps the
 * faster shape for the handle, and records it for the size class
 * (n, L, P, mode precision, state sets) in a process-wide table: a later
 * handle of the same class takes the recorded shapes without timing
 * (cached = 1).  Call between muffin_create and muffin_set_problem
 * (E_STATE otherwise: the timing overwrites the state buffers).
 * Synchronises the stream.  Without it the built-in rule applies (32 x 32
 * when the subband side is at least 64). */
typedef struct {
  int32_t tunable;     /* 0: one shape only (FP64, the starlet, or P != 8) */
  int32_t cached;      /* 1: shapes taken from an earlier tuning of the class */
  int32_t syn_tile1;   /* level-1 synthesis tile side in use (16 or 32) */
  int32_t an_tile1;    /* level-1 analysis tile side in use (16 or 32) */
  double syn_ms[2];    /* measured ms per launch with tiles 16 and 32 (0: not timed) */
  double an_ms[2];
} muffin_tune_result;
int muffin_autotune(muffin_handle* h, int32_t reps, muffin_tune_result* out);

/* ---- operator entry points (same kernels as the iteration) ----
 * in/out are device cubes of the handle's working type.
 *   op_H:   out = H_l in_l     (eq. `model`)
 *   op_HT:  out = H_l^T in_l
 *   op_HTH: out = H_l^T H_l in_l (the data-fidelity gradient without y)
 *   op_Ws:  out[L][P][n][n] = W_s in (1/sqrt(P) scaling included; with the
 *           starlet dictionary P = J + 1 planes, unscaled)
 *   op_WsT: out[L][n][n] = W_s^T in
 *   op_dct: out = W_lambda in (DCT-II along bands), op_idct: W_lambda^T in.
 * Require muffin_set_problem (for H) or only muffin_create (W_s, DCT). */
int muffin_op_H(muffin_handle* h, const void* in, void* out);
int muffin_op_HT(muffin_handle* h, const void* in, void* out);
int muffin_op_HTH(muffin_handle* h, const void* in, void* out);
int muffin_op_Ws(muffin_handle* h, const void* in, void* out);
int muffin_op_WsT(muffin_handle* h, const void* in, void* out);
int muffin_op_dct(muffin_handle* h, const void* in, void* out);
int muffin_op_idct(muffin_handle* h, const void* in, void* out);

#ifdef __cplusplus
}
#endif
#endif /* MUFFIN_H */
