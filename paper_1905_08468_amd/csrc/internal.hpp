// Internal declarations shared by the HIP translation units of libmuffin.
// Data layout (band-major, as the paper's N x L matrix X stored column by
// column): a cube is [band][row][col] with pixel n = row * side + col.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace muffin {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }

// Scalars of one solve that kernels read from device memory, so that the
// automatic parameter update can change them without a host round trip.
struct DevParams {
  double mu, gamma;          // theta = (mu, gamma)
  double tau, sigma;         // primal / dual steps
  double beta_H;             // Lipschitz constant of the least-squares gradient
  double max_beta2, sum_beta2, max_alpha2, sum_alpha2;
  double rho;
  double ws_norm2;           // ||W_s||^2 in the step rule (1 for the Daubechies union)
  double eta_mu, eta_gamma;  // ADA-PT gradient steps
  double eps_fd, sigma_w;    // FDMC perturbation size and noise std
  double res_const;          // visibilities: |v|^2 (0 for dirty images)
  double n_meas;             // real measurements (PSURE's noise term)
  int32_t vis;               // 1: visibility data (residual from dot products)
  int32_t pad_;
  int32_t tau_rule;          // 0: operator-norm form, 1: printed sum form
  int32_t n_updates;         // theta updates done
  double sums[8];            // reduction results (see Slot)
};

// Reduction result slots in DevParams::sums.
enum Slot {
  SLOT_RES2 = 0,    // ||Y - H X||^2
  SLOT_GX_MU = 1,   // <H^T H X - H^T Y, X'_mu>
  SLOT_GX_GA = 2,   // <H^T H X - H^T Y, X'_gamma>
  SLOT_FD_MU = 3,   // <H^T delta, Xbar'_mu - X'_mu>
  SLOT_FD_GA = 4,   // <H^T delta, Xbar'_gamma - X'_gamma>
  SLOT_FD_X = 5,    // <H^T delta, Xbar - X>
  SLOT_AUX0 = 6,
  SLOT_AUX1 = 7,
};

constexpr int kMaxSets = 6;
constexpr int kMaxBases = 8;
constexpr int kHistCols = 8;  // k, mu, gamma, tau, sugar_mu, sugar_gamma, psure, res2
constexpr int kMaxHistRows = 4096;  // theta updates kept per handle

// Device memory for buffers and plan tables: hipMalloc (region == nullptr),
// or consecutive 256-byte-aligned pieces of a region the caller owns (the
// allocation-free solve).  region_alloc returns nullptr when the region is
// full (or hipMalloc fails); pieces of a region are never freed one by one:
// the owner rewinds `used`.
struct Region {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};
void* region_alloc(Region* r, size_t bytes);
inline size_t region_round(size_t bytes) { return (bytes + 255) & ~size_t(255); }

// ---------------------------------------------------------------- FFT ----
// FFT plan: side n (image n x n, FFT grid 2n x 2n).
template <typename T>
struct FftPlan {
  int n = 0;
  int L = 0;
  cplx<T>* tw = nullptr;   // tw[k] = exp(-2 pi i k / (2n)), k < 2n
  cplx<T>* twr = nullptr;  // stage twiddle tables, length-n FFT (inside tw's block)
  cplx<T>* twc = nullptr;  // stage twiddle tables, length-2n FFT
  cplx<T>* Kh = nullptr;   // [L][n+1][2n] transfer function / (4 n^2)
  bool borrowed = false;   // tables live in a caller's region (not freed)
};

// One input/output pair of a batched convolution chain.
template <typename T>
struct ChainIO {
  const T* in[kMaxSets];
  T* out[kMaxSets];
  cplx<T>* specA[kMaxSets];   // [L][n][n] spectra (column-major in kx)
  cplx<T>* specB[kMaxSets];
  const T* y;                 // optional: residual ||H in[0] - y||^2
  double* res_partials;       // per-block partial sums, or null
  int nsets;
  // optional: called on the host before each pass (p = 0 row, 1 column,
  // 2 middle row, 3 second column, 4 last row) and after the last (p = 5),
  // for per-pass device timing
  void (*mark)(void* ctx, int p);
  void* mark_ctx;
};

template <typename T>
int fft_make_plan(FftPlan<T>& p, int n, int L, hipStream_t s, Region* r = nullptr);
// device bytes of a plan's tables (as allocated by fft_make_plan)
size_t fft_plan_bytes(int n, int L, int elem_bytes);
template <typename T>
void fft_free_plan(FftPlan<T>& p);
// K-PSF: Kh from the PSF cube [L][2n][2n] (centre (n, n)); tmp holds
// L*(n+1)*2n complex values.
template <typename T>
int fft_psf_spectrum(FftPlan<T>& p, const T* psf, cplx<T>* tmp, hipStream_t s);
// out = H in (op=0), H^T in (op=1), H^T H in (op=2), for every set.
template <typename T>
int fft_chain(const FftPlan<T>& p, const ChainIO<T>& io, int op, hipStream_t s);
// Number of per-block residual partials fft_chain writes for op=2.
int fft_res_blocks(int n, int L, int elem_bytes);

// ---------------------------------------------------------------- DWT ----
template <typename T>
struct DwtPlan {
  int n = 0, L = 0, P = 0, J = 0;
  // level-1 tile side of the FP32 kernels: 0 = built-in rule (32 when the
  // subband side is >= 64), 16 or 32 = forced (the autotuner's choice)
  int syn_tile1 = 0, an_tile1 = 0;
};

// Dual-update roles.
enum DualRole { ROLE_PRIMAL = 0, ROLE_DERIV = 1 };

// Analysis of NSET inputs z_s = c1_s (2 Xt_a - X_a) + c2_s (2 Xt_b - X_b)
// followed by the dual update of U_s with scale sigma * beta_l / sqrt(P).
template <typename T>
struct AnalysisIO {
  // level-1 input z = c1 z_a + c2 z_b, where z_a, z_b are 2 x~ - x of a set
  // (made by the primal step), or the operand itself (set-up and debug ops)
  const T* z_a[kMaxSets];
  const T* z_b[kMaxSets];  // or null
  int c1_sel[kMaxSets];   // which theta factor multiplies the a-term
  int c2_sel[kMaxSets];   // and the b-term (see CoefSel)
  T* U[kMaxSets];         // [L][P][n][n] in/out
  uint8_t* mask[kMaxSets];// [L][P][n][n]: written by primal, read by deriv
  T* tmp0[kMaxSets];      // [L][P][(n/2)^2]
  T* tmp1[kMaxSets];      // [L][P][(n/4)^2]
  int role;
  int nsets;
  const double* beta;     // [L]
  int pure;               // 1: no dual update, write scale*coef into U (debug op)
  double pure_scale;
};

// Synthesis of NSET coefficient sets c_s = a1 U_a + a2 U_b, output
// S_s = beta_l / sqrt(P) * W^T c_s.
template <typename T>
struct SynthesisIO {
  const T* Ua[kMaxSets];     // dual array U of each set
  T* S[kMaxSets];            // out: beta_l / sqrt(P) W_s^T U
  T* tmp0[kMaxSets];
  T* tmp1[kMaxSets];
  int nsets;
  const double* beta;     // [L] or null (then 1)
  int pure;               // 1: plain W^T (debug op)
};

// Coefficient selectors: the factor is read from DevParams at run time.
enum CoefSel { SEL_ZERO = 0, SEL_ONE = 1, SEL_MU = 2, SEL_GAMMA = 3 };

// 32-bit mask words the analysis of an n x n x L cube with J levels writes
// per state set (one per thread and block of every level; the largest of
// the launch shapes it may use).
size_t dwt_mask_words(int n, int L, int J, int P, int elem_bytes);
// Levels lev_lo..lev_hi (1-based; analysis runs them in increasing order,
// synthesis in decreasing order).  0, 0 = all levels.
template <typename T>
int dwt_analysis(const DwtPlan<T>& p, const AnalysisIO<T>& io, const DevParams* dp,
                 hipStream_t s, int lev_lo = 0, int lev_hi = 0);
template <typename T>
int dwt_synthesis(const DwtPlan<T>& p, const SynthesisIO<T>& io, const DevParams* dp,
                  hipStream_t s, int lev_lo = 0, int lev_hi = 0);
int dwt_upload_filters(int P);  // host: derive db1..dbP, copy to device constants

// ------------------------------------------------------------ starlet ----
// W_s as the isotropic undecimated wavelet transform (J scales, J + 1
// planes per band: the wavelet scales, then the coarse plane).  Same IO as
// the Daubechies union; U and the masks are [L][J+1][n][n], no 1/sqrt(P)
// scaling (the analysis step is sigma * beta_l, the synthesis beta_l W^T u);
// tmp0/tmp1 each hold one [L][n][n] intermediate.
struct StarletPlan {
  int n = 0, L = 0, J = 0;
};
template <typename T>
int starlet_analysis(const StarletPlan& p, const AnalysisIO<T>& io, const DevParams* dp,
                     hipStream_t s);
template <typename T>
int starlet_synthesis(const StarletPlan& p, const SynthesisIO<T>& io, hipStream_t s);
double starlet_norm2(int n, int J);  // host: ||W_s||^2 on n x n images

// ---------------------------------------------------------------- DCT ----
enum DctKind { DCT_F64 = 0, DCT_F32 = 1, DCT_BF16X3 = 2 };

template <typename T>
struct DctPlan {
  int L = 0, Lp = 0, N = 0;
  int kind = 0;
  T* C = nullptr;            // [Lp][Lp] padded DCT-II matrix (row k, column l)
  uint16_t* Chi = nullptr;   // bf16 hi/lo fragments of C and C^T (BF16X3 only)
  uint16_t* Clo = nullptr;   // (inside Chi's allocation)
  bool borrowed = false;     // tables live in a caller's region (not freed)
};

template <typename T>
struct DctIO {
  const T* z_a[kMaxSets];    // input z = c1 z_a + c2 z_b (as AnalysisIO)
  const T* z_b[kMaxSets];    // or null
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  T* V[kMaxSets];
  const T* Vb[kMaxSets];     // second term of the adjoint input (new primal V)
  int d1_sel[kMaxSets], d2_sel[kMaxSets];
  T* Tout[kMaxSets];
  uint8_t* mask[kMaxSets];
  int role;
  int nsets;
  const double* alpha;       // [N] or null (then 1)
  int pure;                  // 1: out = C in (debug), 2: out = C^T in (debug)
};

// 32-bit mask words the spectral update writes per state set over N pixels
// (one per thread and block; the largest of its launch shapes).
size_t dct_mask_words(int N);
template <typename T>
int dct_make_plan(DctPlan<T>& p, int L, int N, int kind, Region* r = nullptr);
// device bytes of a plan's tables (as allocated by dct_make_plan)
size_t dct_plan_bytes(int L, int kind, int elem_bytes);
template <typename T>
void dct_free_plan(DctPlan<T>& p);
template <typename T>
int dct_update(const DctPlan<T>& p, const DctIO<T>& io, const DevParams* dp, hipStream_t s);

// ------------------------------------------------------- elementwise ----
template <typename T>
struct PrimalIO {
  // per trajectory: primal set then (optionally) two derivative sets
  const T* x[2][3];
  const T* g[2][3];      // H^T H x
  const T* hty[2];       // H^T y of the trajectory (primal only)
  const T* s[2][3];      // beta_l / sqrt(P) W_s^T u of each set (no mu)
  const T* t[2][3];
  T* xt[2][3];
  T* z[2][3];            // 2 x~ - x of each set, the analyses' input
  int ntraj, nderiv;
};
template <typename T>
int primal_step(const PrimalIO<T>& io, size_t count, const DevParams* dp, hipStream_t s);

// Deterministic FP64 dot products: sum_i (a_i - b_i) * c_i (b optional).
template <typename T>
int dot_partials(const T* a, const T* b, const T* c, size_t count, double* partials,
                 int nblocks, hipStream_t s);
int dot_blocks();
int reduce_to_slot(const double* partials, int count, DevParams* dp, int slot, hipStream_t s);
int reduce_to_buffer(const double* partials, int count, double* out, hipStream_t s);

template <typename T>
int fill_zero(T* p, size_t count, hipStream_t s);
template <typename T>
int axpy_copy(T* out, const T* a, const T* b, double beta, size_t count, hipStream_t s);
template <typename T>
int copy_dev(T* out, const T* in, size_t count, hipStream_t s);
// out[0] = sum (a - b)^2, out[1] = sum a^2 (FP64, deterministic); partials
// holds 2 nblocks doubles.
template <typename T>
int diff_sq(const T* a, const T* b, size_t count, double* partials, int nblocks, double* out,
            hipStream_t s);
template <typename T>
int count_nonfinite(const T* p, size_t count, int* flag, hipStream_t s);
template <typename T, typename U>
int convert(U* out, const T* in, size_t count, hipStream_t s);

// K-W: alpha_n = 1/(||x0^n|| + eps), beta_l = 1/(||x0_l|| + eps).
template <typename T>
int beta_from(const T* w, int L, int per_band, double eps, double* beta, double* partials,
              hipStream_t s);
template <typename T>
int weights_from(const T* x0, int L, int N, double eps, double* alpha, double* beta,
                 double* partials, hipStream_t s);

// K-THETA: SUGAR from the reduction slots, theta update, tau recompute,
// history row (hist[n_updates], iteration (n_updates + 1) * period).
int theta_update(DevParams* dp, double* hist, int max_hist, int period, int apply,
                 hipStream_t s);
int tau_refresh(DevParams* dp, hipStream_t s);

// K-PI helpers (FP64).
int pi_init(double* v, size_t count, unsigned long long seed, hipStream_t s);
int pi_band_dots(const double* v, const double* w, int L, int N, double* partials,
                 int bpb, hipStream_t s);
int pi_band_finish(const double* partials, int L, int bpb, double* vw_ww_vv, hipStream_t s);
int pi_normalise(double* v, const double* w, const double* stats, int L, int N,
                 hipStream_t s);

}  // namespace muffin

// Kernels whose dynamic LDS can exceed 64 KB opt in to the CU's full LDS.
// Workgroup barrier for LDS hand-offs between the waves of a block: waits
// for this wave's LDS (and scalar-load) operations only.  __syncthreads() is
// a workgroup-scope fence that also drains every outstanding global load and
// store, which would expose the latency of loads issued ahead of time (the
// next tile, the next state set) at every barrier.  Global memory written by
// a block is never read back by the same block within a kernel here.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

#define MUFFIN_ALLOW_BIG_LDS(kernel)                                                  \
  do {                                                                                \
    static bool _done = false;                                                        \
    if (!_done) {                                                                     \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),                \
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
      (void)hipGetLastError();                                                        \
      _done = true;                                                                   \
    }                                                                                 \
  } while (0)

#define MUFFIN_HIP_CHECK(expr)                   \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return -5; /* E_HIP */ \
  } while (0)
