// Spectral unmixing of a reconstructed cube (Section 4.3): for every pixel
// n, the abundances a^n = argmin_{a >= 0} |x^n - E a|^2 of k chosen
// endmember spectra (the columns of E, L x k).
//
// One thread per pixel streams its spectrum down the band-major cube (loads
// coalesced across the pixels of a wave), accumulating b = E^T x^n and
// |x^n|^2 in FP64 with the endmember values read as block-uniform scalars.
// The k-dimensional problem is then solved exactly: the solution is the
// least-squares solution on its support S (a_S = (E_S^T E_S)^-1 b_S, with
// inverses precomputed on the host, G = E^T E, FP64) that satisfies the
// optimality conditions: a_S >= 0 and a non-negative gradient g = G a - b
// off the support.  The kernel scans all 2^k supports and keeps, among
// those with a_S >= 0, the one whose off-support gradient is least negative
// (ties: the smaller objective 1/2 a^T G a - b^T a = -1/2 b^T a).  Choosing
// by the objective alone is not robust: when G is ill-conditioned, dropping
// a tiny abundance changes the objective by less than its rounding, while
// the gradient it leaves behind stays well above rounding.  The cube is read
// once: the kernel is bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "muffin.h"
#include "internal.hpp"

namespace muffin {
namespace {

constexpr int kUnmixMaxK = 4;
constexpr int kUnmixNT = 256;
constexpr int kSubsets = 1 << kUnmixMaxK;

// inv[m][i][j]: inverse of G restricted to support m (zero outside it)
struct UnmixTable {
  double inv[kSubsets][kUnmixMaxK][kUnmixMaxK];
  double G[kUnmixMaxK][kUnmixMaxK];
};

template <typename T, int K>
__global__ void __launch_bounds__(kUnmixNT) unmix_kernel(const T* __restrict__ X, int L, int N,
                                                         const double* __restrict__ E,
                                                         const UnmixTable* __restrict__ tab,
                                                         T* __restrict__ A, T* __restrict__ R) {
  const int p = blockIdx.x * kUnmixNT + threadIdx.x;
  const int pc = p < N ? p : N - 1;  // the tail reads a valid pixel, writes nothing
  double b[K], xx = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) b[j] = 0.0;
  const T* x = X + pc;
  int l = 0;
  for (; l + 8 <= L; l += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[(size_t)(l + u) * N];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double d = double(v[u]);
      xx = fma(d, d, xx);
#pragma unroll
      for (int j = 0; j < K; ++j) b[j] = fma(E[j * L + l + u], d, b[j]);
    }
  }
  for (; l < L; ++l) {
    const double d = double(x[(size_t)l * N]);
    xx = fma(d, d, xx);
#pragma unroll
    for (int j = 0; j < K; ++j) b[j] = fma(E[j * L + l], d, b[j]);
  }
  // the empty support: a = 0, gradient -b, objective 0
  double best[K], fbest = 0.0, vbest = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    best[j] = 0.0;
    vbest = fmax(vbest, b[j]);
  }
#pragma unroll
  for (int m = 1; m < (1 << K); ++m) {
    double a[K], f = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) s = fma(tab->inv[m][i][j], b[j], s);
      a[i] = s;
      if (m >> i & 1) ok = ok && s >= 0.0;
      f = fma(-0.5 * s, b[i], f);
    }
    double v = 0.0;  // largest negative part of the gradient off the support
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (m >> i & 1) continue;
      double g = -b[i];
#pragma unroll
      for (int j = 0; j < K; ++j) g = fma(tab->G[i][j], a[j], g);
      v = fmax(v, -g);
    }
    if (ok && (v < vbest || (v == vbest && f < fbest))) {
      vbest = v;
      fbest = f;
#pragma unroll
      for (int i = 0; i < K; ++i) best[i] = (m >> i & 1) ? a[i] : 0.0;
    }
  }
  if (p < N) {
#pragma unroll
    for (int j = 0; j < K; ++j) A[(size_t)j * N + p] = T(best[j]);
    // |x - E a|^2 = |x|^2 - b^T a at the least-squares solution on S
    if (R) R[p] = T(fmax(xx + 2.0 * fbest, 0.0));
  }
}

// inverse of a symmetric positive-definite m x m matrix by Cholesky;
// false when it is not positive definite
bool spd_inverse(int m, const double* a, double* inv) {
  std::vector<double> c(m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double d = a[j * m + j];
    for (int k = 0; k < j; ++k) d -= c[j * m + k] * c[j * m + k];
    if (!(d > 0.0)) return false;
    c[j * m + j] = std::sqrt(d);
    for (int i = j + 1; i < m; ++i) {
      double s = a[i * m + j];
      for (int k = 0; k < j; ++k) s -= c[i * m + k] * c[j * m + k];
      c[i * m + j] = s / c[j * m + j];
    }
  }
  // columns of the inverse: solve C C^T y = e_col
  for (int col = 0; col < m; ++col) {
    std::vector<double> y(m, 0.0);
    for (int i = 0; i < m; ++i) {
      double s = i == col ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= c[i * m + k] * y[k];
      y[i] = s / c[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < m; ++k) s -= c[k * m + i] * y[k];
      y[i] = s / c[i * m + i];
    }
    for (int i = 0; i < m; ++i) inv[i * m + col] = y[i];
  }
  return true;
}

}  // namespace
}  // namespace muffin

using namespace muffin;

struct muffin_unmix_plan {
  int k = 0, L = 0;
  double* E = nullptr;       // device [k][L]
  UnmixTable* tab = nullptr;  // device
};

extern "C" {

int muffin_unmix_plan_create(muffin_unmix_plan** out, const double* spectra, int32_t k,
                             int32_t L) {
  if (!out || !spectra || k < 1 || k > kUnmixMaxK || L < k) return MUFFIN_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < k * L; ++i)
    if (!std::isfinite(spectra[i])) return MUFFIN_E_INVAL;
  // Gram matrix and the inverses of all its principal submatrices
  std::vector<double> G(k * k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double s = 0.0;
      for (int l = 0; l < L; ++l) s += spectra[i * L + l] * spectra[j * L + l];
      G[i * k + j] = s;
    }
  UnmixTable h;
  std::memset(&h, 0, sizeof(h));
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) h.G[i][j] = G[i * k + j];
  for (int m = 1; m < (1 << k); ++m) {
    int idx[kUnmixMaxK], q = 0;
    for (int i = 0; i < k; ++i)
      if (m >> i & 1) idx[q++] = i;
    double sub[kUnmixMaxK * kUnmixMaxK], inv[kUnmixMaxK * kUnmixMaxK];
    for (int r = 0; r < q; ++r)
      for (int c = 0; c < q; ++c) sub[r * q + c] = G[idx[r] * k + idx[c]];
    if (!spd_inverse(q, sub, inv)) return MUFFIN_E_INVAL;  // dependent spectra
    for (int r = 0; r < q; ++r)
      for (int c = 0; c < q; ++c) h.inv[m][idx[r]][idx[c]] = inv[r * q + c];
  }
  std::unique_ptr<muffin_unmix_plan> pl(new (std::nothrow) muffin_unmix_plan());
  if (!pl) return MUFFIN_E_NOMEM;
  pl->k = k;
  pl->L = L;
  if (hipMalloc(&pl->E, sizeof(double) * k * L) != hipSuccess) return MUFFIN_E_NOMEM;
  if (hipMalloc(&pl->tab, sizeof(UnmixTable)) != hipSuccess) {
    (void)hipFree(pl->E);
    return MUFFIN_E_NOMEM;
  }
  if (hipMemcpy(pl->E, spectra, sizeof(double) * k * L, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->tab, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(pl->E);
    (void)hipFree(pl->tab);
    return MUFFIN_E_HIP;
  }
  *out = pl.release();
  return MUFFIN_OK;
}

int muffin_unmix_run(const muffin_unmix_plan* pl, const void* cube, int32_t n, int32_t mode,
                     void* abund, void* resid, void* stream) {
  if (!pl || !cube || !abund || n < 1) return MUFFIN_E_INVAL;
  if (mode != MUFFIN_F64 && mode != MUFFIN_F32 && mode != MUFFIN_F32_BF16DCT) return MUFFIN_E_INVAL;
  const long long N = (long long)n * n;
  if (N > (1LL << 30)) return MUFFIN_E_SHAPE;
  const int nb = (int)((N + kUnmixNT - 1) / kUnmixNT);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f64 = mode == MUFFIN_F64;
#define MUFFIN_UNMIX_LAUNCH(T, K)                                                         \
  unmix_kernel<T, K><<<nb, kUnmixNT, 0, s>>>(static_cast<const T*>(cube), pl->L, (int)N,  \
                                            pl->E, pl->tab, static_cast<T*>(abund),      \
                                            static_cast<T*>(resid))
  switch (pl->k * 2 + (f64 ? 1 : 0)) {
    case 2: MUFFIN_UNMIX_LAUNCH(float, 1); break;
    case 3: MUFFIN_UNMIX_LAUNCH(double, 1); break;
    case 4: MUFFIN_UNMIX_LAUNCH(float, 2); break;
    case 5: MUFFIN_UNMIX_LAUNCH(double, 2); break;
    case 6: MUFFIN_UNMIX_LAUNCH(float, 3); break;
    case 7: MUFFIN_UNMIX_LAUNCH(double, 3); break;
    case 8: MUFFIN_UNMIX_LAUNCH(float, 4); break;
    default: MUFFIN_UNMIX_LAUNCH(double, 4); break;
  }
#undef MUFFIN_UNMIX_LAUNCH
  MUFFIN_HIP_CHECK(hipGetLastError());
  return MUFFIN_OK;
}

int muffin_unmix_plan_destroy(muffin_unmix_plan* pl) {
  if (!pl) return MUFFIN_E_INVAL;
  (void)hipFree(pl->E);
  (void)hipFree(pl->tab);
  delete pl;
  return MUFFIN_OK;
}

}  // extern "C"
