// Spatial sparse-analysis operator W_s (eq. `RegAll`, Section 2.1) and its
// adjoint: the union of the first P Daubechies orthonormal bases
// (Section 4.2, implementation details), each a J-level 2-D separable
// periodised DWT in the Mallat layout, stacked and scaled by 1/sqrt(P) so
// that W_s^T W_s = I.
//
// Analysis is fused with the dual update of eqs. `stpp`/`stpu`
// (Algorithm 2) and its derivative (Algorithms 3-4):
//   p = u + sigma beta_l W_s(z),  u <- sat(p)            (primal, mask 1[|p|<=1])
//   p' = u' + sigma beta_l W_s(z'), u' <- 1[|p|<=1] p'   (derivative)
// where z is a run-time combination of (2 x~ - x) terms.  Synthesis computes
// s = beta_l W_s^T (a1 U_a + a2 U_b) (eq. `adjointspat2` and its derivatives).
//
// Tiles: a block owns a TO x TO tile of every subband of one level and one
// band; its input tile (2 TO + 14)^2 with the periodic halo of the longest
// filter (db8, 16 taps) is staged in LDS once.  At level 1 all P bases read
// the same input, so a block loops over the bases and the input (computed on
// the fly from x~ and x) is read once.  Levels >= 2 work per basis on the
// low-pass band of the previous level.
#include "internal.hpp"

#include <complex>
#include <cmath>
#include <vector>

namespace muffin {

__constant__ double c_hd[kMaxBases][16];
__constant__ double c_gd[kMaxBases][16];
__constant__ float c_hf[kMaxBases][16];
__constant__ float c_gf[kMaxBases][16];

template <typename T>
__device__ __forceinline__ T filt_h(int p, int m);
template <>
__device__ __forceinline__ double filt_h<double>(int p, int m) { return c_hd[p][m]; }
template <>
__device__ __forceinline__ float filt_h<float>(int p, int m) { return c_hf[p][m]; }
template <typename T>
__device__ __forceinline__ T filt_g(int p, int m);
template <>
__device__ __forceinline__ double filt_g<double>(int p, int m) { return c_gd[p][m]; }
template <>
__device__ __forceinline__ float filt_g<float>(int p, int m) { return c_gf[p][m]; }

// ---------------------------------------------------------------------------
// Host: Daubechies extremal-phase low-pass filters by spectral factorisation.
// |m0(w)|^2 = cos^{2p}(w/2) Pp(sin^2(w/2)), Pp(y) = sum_{k<p} C(p-1+k, k) y^k.
// Each root y_j of Pp gives the reciprocal pair of roots of
// z^2 - (2 - 4 y_j) z + 1; the extremal-phase filter takes the root outside
// the unit circle.  Roots of Pp by Durand-Kerner in long double, then the
// polynomial (1 + z)^p prod (z - r_j) normalised to sum sqrt(2).
// ---------------------------------------------------------------------------
using cld = std::complex<long double>;

static std::vector<cld> poly_roots(const std::vector<long double>& a) {
  // a: coefficients, ascending powers, a.back() != 0
  const int d = (int)a.size() - 1;
  std::vector<cld> r(d);
  if (d == 0) return r;
  const cld seed(0.4L, 0.9L);
  cld cur(1.0L, 0.0L);
  for (int i = 0; i < d; ++i) {
    r[i] = cur;
    cur *= seed;
  }
  auto eval = [&](cld z) {
    cld v(a[d], 0.0L);
    for (int k = d - 1; k >= 0; --k) v = v * z + a[k];
    return v / a[d];
  };
  for (int it = 0; it < 2000; ++it) {
    long double change = 0.0L;
    for (int i = 0; i < d; ++i) {
      cld den(1.0L, 0.0L);
      for (int j = 0; j < d; ++j)
        if (j != i) den *= (r[i] - r[j]);
      const cld step = eval(r[i]) / den;
      r[i] -= step;
      change = std::max(change, std::abs(step));
    }
    if (change < 1e-30L) break;
  }
  // Newton polish on the original polynomial
  for (int i = 0; i < d; ++i) {
    for (int it = 0; it < 5; ++it) {
      cld v(a[d], 0.0L), dv(0.0L, 0.0L);
      for (int k = d - 1; k >= 0; --k) {
        dv = dv * r[i] + v;
        v = v * r[i] + a[k];
      }
      if (std::abs(dv) == 0.0L) break;
      r[i] -= v / dv;
    }
  }
  return r;
}

static std::vector<long double> daub_lowpass(int p) {
  std::vector<long double> P(p);
  for (int k = 0; k < p; ++k) {
    long double c = 1.0L;  // C(p-1+k, k)
    for (int i = 1; i <= k; ++i) c = c * (p - 1 + i) / i;
    P[k] = c;
  }
  std::vector<cld> poly{cld(1.0L, 0.0L)};
  auto mul = [&](const std::vector<cld>& b) {
    std::vector<cld> out(poly.size() + b.size() - 1, cld(0.0L, 0.0L));
    for (size_t i = 0; i < poly.size(); ++i)
      for (size_t j = 0; j < b.size(); ++j) out[i + j] += poly[i] * b[j];
    poly.swap(out);
  };
  for (int i = 0; i < p; ++i) mul({cld(1.0L, 0.0L), cld(1.0L, 0.0L)});
  if (p > 1) {
    for (const cld& y : poly_roots(P)) {
      const cld b = 2.0L - 4.0L * y;
      const cld disc = std::sqrt(b * b - 4.0L);
      cld r1 = (b + disc) / 2.0L, r2 = (b - disc) / 2.0L;
      const cld r = std::abs(r1) > std::abs(r2) ? r1 : r2;
      mul({-r, cld(1.0L, 0.0L)});
    }
  }
  cld s(0.0L, 0.0L);
  for (auto& c : poly) s += c;
  std::vector<long double> h(poly.size());
  for (size_t i = 0; i < poly.size(); ++i) h[i] = (poly[i] * std::sqrt(2.0L) / s).real();
  return h;
}

int dwt_upload_filters(int P) {
  double hd[kMaxBases][16] = {}, gd[kMaxBases][16] = {};
  float hf[kMaxBases][16] = {}, gf[kMaxBases][16] = {};
  for (int p = 1; p <= P; ++p) {
    const std::vector<long double> h = daub_lowpass(p);
    const int len = 2 * p;
    for (int m = 0; m < len; ++m) {
      const long double g = ((m & 1) ? -1.0L : 1.0L) * h[len - 1 - m];
      hd[p - 1][m] = (double)h[m];
      gd[p - 1][m] = (double)g;
      hf[p - 1][m] = (float)h[m];
      gf[p - 1][m] = (float)g;
    }
  }
  MUFFIN_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_hd), hd, sizeof(hd)));
  MUFFIN_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_gd), gd, sizeof(gd)));
  MUFFIN_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_hf), hf, sizeof(hf)));
  MUFFIN_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_gf), gf, sizeof(gf)));
  return 0;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double coef_of(int sel, const DevParams* dp) {
  switch (sel) {
    case SEL_ONE: return 1.0;
    case SEL_MU: return dp->mu;
    case SEL_GAMMA: return dp->gamma;
    default: return 0.0;
  }
}

__device__ __forceinline__ int xcd_remap_d(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
static inline int xcd_grid_h(int nb) { return ((nb + 7) >> 3) << 3; }

constexpr int kHalo = 14;  // 2 * 8 - 2: longest filter
constexpr int kSHal = 7;   // synthesis halo (8 - 1)

template <typename T>
struct AnArgs {
  const T* xt_a[kMaxSets];
  const T* x_a[kMaxSets];
  const T* xt_b[kMaxSets];
  const T* x_b[kMaxSets];
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  T* U[kMaxSets];
  uint8_t* mask[kMaxSets];
  const T* llin[kMaxSets];   // level >= 2: [L][P][Ms*Ms]
  T* llout[kMaxSets];        // [L][P][(Ms/2)^2] (not at the last level)
  const double* beta;
  const DevParams* dp;
  int n, L, P, level, last;
  int Ms;                    // block side at this level
  int tiles;                 // tiles per side of a subband
  int nblocks;               // logical blocks in x
  int role, pure;
  double pure_scale;
};

// Row filter of basis p over the staged input: rowbuf[r][k] = low, [TO+k] = high.
template <typename T, int TO, int NT, int PB>
__device__ __forceinline__ void an_rows(const T* in, T* rowbuf, int IN) {
  constexpr int KPT = 4;
  constexpr int TAPS = 2 * PB;
  constexpr int NR = 2 * TO + TAPS - 2;  // rows needed
  constexpr int KG = TO / KPT;
  T h[TAPS], g[TAPS];
#pragma unroll
  for (int m = 0; m < TAPS; ++m) {
    h[m] = filt_h<T>(PB - 1, m);
    g[m] = filt_g<T>(PB - 1, m);
  }
  for (int t = threadIdx.x; t < NR * KG; t += NT) {
    const int r = t / KG, k0 = (t - r * KG) * KPT;
    const T* src = in + r * IN + 2 * k0;
    T w[2 * KPT + TAPS - 2];
#pragma unroll
    for (int i = 0; i < 2 * KPT + TAPS - 2; ++i) w[i] = src[i];
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      T lo = T(0), hi = T(0);
#pragma unroll
      for (int m = 0; m < TAPS; ++m) {
        lo += h[m] * w[2 * k + m];
        hi += g[m] * w[2 * k + m];
      }
      rowbuf[r * (2 * TO) + k0 + k] = lo;
      rowbuf[r * (2 * TO) + TO + k0 + k] = hi;
    }
  }
}

// Column filter + output of basis pidx.
template <typename T, int TO, int NT, int PB>
__device__ __forceinline__ void an_cols(const AnArgs<T>& a, const T* rowbuf, int set, int band,
                                        int pidx, int kr0, int kc0, double scale) {
  constexpr int TAPS = 2 * PB;
  T h[TAPS], g[TAPS];
#pragma unroll
  for (int m = 0; m < TAPS; ++m) {
    h[m] = filt_h<T>(PB - 1, m);
    g[m] = filt_g<T>(PB - 1, m);
  }
  const int n = a.n, half = a.Ms >> 1;
  const size_t plane = (size_t)n * n;
  T* U = a.U[set] + ((size_t)band * a.P + pidx) * plane;
  uint8_t* M = a.mask[set] ? a.mask[set] + ((size_t)band * a.P + pidx) * plane : nullptr;
  T* llo = a.last ? nullptr : a.llout[set] + ((size_t)band * a.P + pidx) * (size_t)half * half;
  for (int t = threadIdx.x; t < (TO / 2) * (2 * TO); t += NT) {
    const int q = t % (2 * TO), kp = t / (2 * TO);
    const int kr = 2 * kp;
    T w[TAPS + 2];
#pragma unroll
    for (int i = 0; i < TAPS + 2; ++i) w[i] = rowbuf[(2 * kr + i) * (2 * TO) + q];
    const bool dcol = q >= TO;
    const int kc = kc0 + (dcol ? q - TO : q);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      T lo = T(0), hi = T(0);
#pragma unroll
      for (int m = 0; m < TAPS; ++m) {
        lo += h[m] * w[2 * e + m];
        hi += g[m] * w[2 * e + m];
      }
      const int krow = kr0 + kr + e;
      if (krow >= half || kc >= half) continue;
      // low-pass rows: (row-low, col-low) = LL, (row-high, col-low) = top right
      // high-pass rows: bottom left / bottom right
      const int colq = dcol ? half + kc : kc;
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const T c = part == 0 ? lo : hi;
        const int row = part == 0 ? krow : half + krow;
        if (part == 0 && !dcol && !a.last) {
          llo[(size_t)krow * half + kc] = c;  // LL goes to the next level
          continue;
        }
        const size_t idx = (size_t)row * n + colq;
        if (a.pure) {
          U[idx] = T(a.pure_scale) * c;
          continue;
        }
        const T pv = U[idx] + T(scale) * c;
        if (a.role == ROLE_PRIMAL) {
          U[idx] = pv < T(-1) ? T(-1) : (pv > T(1) ? T(1) : pv);
          if (M) M[idx] = (pv >= T(-1) && pv <= T(1)) ? 1 : 0;
        } else {
          U[idx] = M[idx] ? pv : T(0);
        }
      }
    }
  }
}

template <typename T, int TO, int NT>
__global__ void __launch_bounds__(NT) dwt_an(AnArgs<T> a) {
  constexpr int IN = 2 * TO + kHalo;
  __shared__ T s_in[IN * IN];
  __shared__ T s_row[IN * 2 * TO];
  const int lb = xcd_remap_d(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  const int tiles2 = a.tiles * a.tiles;
  const int band = lb / tiles2;
  const int tile = lb - band * tiles2;
  const int kr0 = (tile / a.tiles) * TO, kc0 = (tile % a.tiles) * TO;
  const int set = a.level == 1 ? blockIdx.y : blockIdx.y / a.P;
  const int pone = a.level == 1 ? -1 : blockIdx.y % a.P;
  const int Ms = a.Ms, msk = Ms - 1;
  const int n = a.n;
  // ---- stage the input tile (periodic wrap) ----
  if (a.level == 1) {
    const double c1 = coef_of(a.c1_sel[set], a.dp), c2 = coef_of(a.c2_sel[set], a.dp);
    const T* xa = a.x_a[set] + (size_t)band * n * n;
    const T* ta = a.xt_a[set] + (size_t)band * n * n;
    const T* xb = a.x_b[set] ? a.x_b[set] + (size_t)band * n * n : nullptr;
    const T* tb = a.xt_b[set] ? a.xt_b[set] + (size_t)band * n * n : nullptr;
    for (int t = threadIdx.x; t < IN * IN; t += NT) {
      const int r = t / IN, c = t - r * IN;
      const size_t idx = (size_t)((2 * kr0 + r) & msk) * n + ((2 * kc0 + c) & msk);
      T z = T(c1) * (T(2) * ta[idx] - xa[idx]);
      if (xb) z += T(c2) * (T(2) * tb[idx] - xb[idx]);
      s_in[t] = z;
    }
  } else {
    const T* src = a.llin[set] + ((size_t)band * a.P + pone) * (size_t)Ms * Ms;
    for (int t = threadIdx.x; t < IN * IN; t += NT) {
      const int r = t / IN, c = t - r * IN;
      s_in[t] = src[(size_t)((2 * kr0 + r) & msk) * Ms + ((2 * kc0 + c) & msk)];
    }
  }
  __syncthreads();
  const double beta = a.beta ? a.beta[band] : 1.0;
  const double scale = a.dp ? a.dp->sigma * beta / sqrt((double)a.P) : 0.0;
  const int p0 = a.level == 1 ? 0 : pone;
  const int p1 = a.level == 1 ? a.P : pone + 1;
  for (int pidx = p0; pidx < p1; ++pidx) {
    switch (pidx + 1) {
#define MUFFIN_AN_CASE(PB)                                                   \
  case PB:                                                                   \
    an_rows<T, TO, NT, PB>(s_in, s_row, IN);                                 \
    __syncthreads();                                                         \
    an_cols<T, TO, NT, PB>(a, s_row, set, band, pidx, kr0, kc0, scale);      \
    break;
      MUFFIN_AN_CASE(1)
      MUFFIN_AN_CASE(2)
      MUFFIN_AN_CASE(3)
      MUFFIN_AN_CASE(4)
      MUFFIN_AN_CASE(5)
      MUFFIN_AN_CASE(6)
      MUFFIN_AN_CASE(7)
      MUFFIN_AN_CASE(8)
#undef MUFFIN_AN_CASE
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------
template <typename T>
struct SyArgs {
  const T* Ua[kMaxSets];
  const T* Ub[kMaxSets];
  int a1_sel[kMaxSets], a2_sel[kMaxSets];
  const T* llin[kMaxSets];   // level < J: [L][P][half^2]
  T* llout[kMaxSets];        // level >= 2: [L][P][Ms^2]
  T* S[kMaxSets];            // level 1: [L][n][n]
  const double* beta;
  const DevParams* dp;
  int n, L, P, level, J;
  int Ms, tiles, nblocks, pure;
};

// Column synthesis of basis PB: from the four quadrants (low/high rows of the
// c and d column halves) into rbuf[2TC][2 (TC + HAL)].
template <typename T, int TC, int NT, int PB>
__device__ __forceinline__ void sy_cols(const T* q, T* rbuf) {
  constexpr int TAPS = 2 * PB;
  constexpr int W = TC + kSHal;
  T he[PB], ho[PB], ge[PB], go[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) {
    he[e] = filt_h<T>(PB - 1, 2 * e);
    ho[e] = filt_h<T>(PB - 1, 2 * e + 1);
    ge[e] = filt_g<T>(PB - 1, 2 * e);
    go[e] = filt_g<T>(PB - 1, 2 * e + 1);
  }
  (void)TAPS;
  // q layout: [quad][W][W], quad 0 = low rows / c cols, 1 = high rows / c cols,
  // 2 = low rows / d cols, 3 = high rows / d cols
  for (int t = threadIdx.x; t < TC * 2 * W; t += NT) {
    const int col = t % (2 * W), a = t / (2 * W);
    const int half = col >= W;
    const int cc = half ? col - W : col;
    const T* ql = q + (half ? 2 : 0) * W * W + cc;
    const T* qh = q + (half ? 3 : 1) * W * W + cc;
    T ev = T(0), od = T(0);
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      const int row = a - e + kSHal;
      const T l = ql[row * W], hgh = qh[row * W];
      ev += he[e] * l + ge[e] * hgh;
      od += ho[e] * l + go[e] * hgh;
    }
    rbuf[(2 * a) * (2 * W) + col] = ev;
    rbuf[(2 * a + 1) * (2 * W) + col] = od;
  }
}

// Row synthesis of basis PB, accumulated into acc[] for this thread's
// outputs (ri, 2b) and (ri, 2b + 1).
template <typename T, int TC, int NT, int PB, int NPT>
__device__ __forceinline__ void sy_rows(const T* rbuf, T (&acc)[NPT][2]) {
  constexpr int W = TC + kSHal;
  T he[PB], ho[PB], ge[PB], go[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) {
    he[e] = filt_h<T>(PB - 1, 2 * e);
    ho[e] = filt_h<T>(PB - 1, 2 * e + 1);
    ge[e] = filt_g<T>(PB - 1, 2 * e);
    go[e] = filt_g<T>(PB - 1, 2 * e + 1);
  }
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int t = threadIdx.x + i * NT;
    const int b = t % TC, ri = t / TC;
    const T* rc = rbuf + ri * (2 * W);
    const T* rd = rc + W;
    T ev = T(0), od = T(0);
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      const int c = b - e + kSHal;
      ev += he[e] * rc[c] + ge[e] * rd[c];
      od += ho[e] * rc[c] + go[e] * rd[c];
    }
    acc[i][0] += ev;
    acc[i][1] += od;
  }
}

template <typename T, int TC, int NT>
__global__ void __launch_bounds__(NT) dwt_sy(SyArgs<T> a) {
  constexpr int W = TC + kSHal;
  constexpr int NPT = (2 * TC * TC) / NT;  // outputs (pairs) per thread
  static_assert(NPT * NT == 2 * TC * TC, "tile/threads");
  __shared__ T s_q[4 * W * W];
  __shared__ T s_r[2 * TC * 2 * W];
  const int lb = xcd_remap_d(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  const int tiles2 = a.tiles * a.tiles;
  const int band = lb / tiles2;
  const int tile = lb - band * tiles2;
  const int kr0 = (tile / a.tiles) * TC, kc0 = (tile % a.tiles) * TC;
  const int set = a.level == 1 ? blockIdx.y : blockIdx.y / a.P;
  const int pone = a.level == 1 ? -1 : blockIdx.y % a.P;
  const int n = a.n, Ms = a.Ms, half = Ms >> 1, hm = half - 1;
  const size_t plane = (size_t)n * n;
  const double a1 = a.pure ? 1.0 : coef_of(a.a1_sel[set], a.dp);
  const double a2 = a.pure ? 0.0 : coef_of(a.a2_sel[set], a.dp);
  T acc[NPT][2];
#pragma unroll
  for (int i = 0; i < NPT; ++i) acc[i][0] = acc[i][1] = T(0);
  const int p0 = a.level == 1 ? 0 : pone;
  const int p1 = a.level == 1 ? a.P : pone + 1;
  for (int pidx = p0; pidx < p1; ++pidx) {
    const T* Ua = a.Ua[set] + ((size_t)band * a.P + pidx) * plane;
    const T* Ub = a.Ub[set] ? a.Ub[set] + ((size_t)band * a.P + pidx) * plane : nullptr;
    const T* ll = a.level < a.J ? a.llin[set] + ((size_t)band * a.P + pidx) * (size_t)half * half
                                : nullptr;
    for (int t = threadIdx.x; t < 4 * W * W; t += NT) {
      const int quad = t / (W * W), rem = t - quad * W * W;
      const int r = rem / W, c = rem - r * W;
      const int kr = (kr0 - kSHal + r) & hm, kc = (kc0 - kSHal + c) & hm;
      const int roff = (quad & 1) ? half : 0, coff = (quad & 2) ? half : 0;
      T v;
      if (quad == 0 && ll) {
        v = ll[(size_t)kr * half + kc];
      } else {
        const size_t idx = (size_t)(roff + kr) * n + (coff + kc);
        v = T(a1) * Ua[idx];
        if (Ub) v += T(a2) * Ub[idx];
      }
      s_q[t] = v;
    }
    __syncthreads();
    switch (pidx + 1) {
#define MUFFIN_SY_CASE(PB)                        \
  case PB:                                        \
    sy_cols<T, TC, NT, PB>(s_q, s_r);             \
    __syncthreads();                              \
    sy_rows<T, TC, NT, PB, NPT>(s_r, acc);        \
    break;
      MUFFIN_SY_CASE(1)
      MUFFIN_SY_CASE(2)
      MUFFIN_SY_CASE(3)
      MUFFIN_SY_CASE(4)
      MUFFIN_SY_CASE(5)
      MUFFIN_SY_CASE(6)
      MUFFIN_SY_CASE(7)
      MUFFIN_SY_CASE(8)
#undef MUFFIN_SY_CASE
    }
    __syncthreads();
  }
  // ---- store ----
  const int o0 = 2 * kr0, q0 = 2 * kc0;
  if (a.level == 1) {
    const double beta = a.beta ? a.beta[band] : 1.0;
    const T sc = T(beta / sqrt((double)a.P));
    T* S = a.S[set] + (size_t)band * plane;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = threadIdx.x + i * NT;
      const int b = t % TC, ri = t / TC;
      const int row = o0 + ri, col = q0 + 2 * b;
      if (row < Ms && col < Ms) {
        S[(size_t)row * n + col] = sc * acc[i][0];
        S[(size_t)row * n + col + 1] = sc * acc[i][1];
      }
    }
  } else {
    T* out = a.llout[set] + ((size_t)band * a.P + pone) * (size_t)Ms * Ms;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int t = threadIdx.x + i * NT;
      const int b = t % TC, ri = t / TC;
      const int row = o0 + ri, col = q0 + 2 * b;
      if (row < Ms && col < Ms) {
        out[(size_t)row * Ms + col] = acc[i][0];
        out[(size_t)row * Ms + col + 1] = acc[i][1];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int kTO = 16;
constexpr int kNT = 256;

template <typename T>
int dwt_analysis(const DwtPlan<T>& p, const AnalysisIO<T>& io, const DevParams* dp,
                 hipStream_t s, int lev_lo, int lev_hi) {
  if (lev_lo <= 0) lev_lo = 1;
  if (lev_hi <= 0 || lev_hi > p.J) lev_hi = p.J;
  for (int lev = lev_lo; lev <= lev_hi; ++lev) {
    AnArgs<T> a{};
    for (int i = 0; i < io.nsets; ++i) {
      a.xt_a[i] = io.xt_a[i];
      a.x_a[i] = io.x_a[i];
      a.xt_b[i] = io.xt_b[i];
      a.x_b[i] = io.x_b[i];
      a.c1_sel[i] = io.c1_sel[i];
      a.c2_sel[i] = io.c2_sel[i];
      a.U[i] = io.U[i];
      a.mask[i] = io.mask[i];
      // LL_j lives in tmp0 for odd j, tmp1 for even j
      a.llin[i] = lev >= 2 ? ((lev - 1) % 2 == 1 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.llout[i] = lev % 2 == 1 ? io.tmp0[i] : io.tmp1[i];
    }
    a.beta = io.beta;
    a.dp = dp;
    a.n = p.n;
    a.L = p.L;
    a.P = p.P;
    a.level = lev;
    a.last = lev == p.J;
    a.Ms = p.n >> (lev - 1);
    const int half = a.Ms >> 1;
    a.tiles = (half + kTO - 1) / kTO;
    a.nblocks = a.tiles * a.tiles * p.L;
    a.role = io.role;
    a.pure = io.pure;
    a.pure_scale = io.pure_scale;
    dim3 grid(xcd_grid_h(a.nblocks), lev == 1 ? io.nsets : io.nsets * p.P);
    dwt_an<T, kTO, kNT><<<grid, kNT, 0, s>>>(a);
    MUFFIN_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

template <typename T>
int dwt_synthesis(const DwtPlan<T>& p, const SynthesisIO<T>& io, const DevParams* dp,
                  hipStream_t s, int lev_lo, int lev_hi) {
  if (lev_lo <= 0) lev_lo = 1;
  if (lev_hi <= 0 || lev_hi > p.J) lev_hi = p.J;
  for (int lev = lev_hi; lev >= lev_lo; --lev) {
    SyArgs<T> a{};
    for (int i = 0; i < io.nsets; ++i) {
      a.Ua[i] = io.Ua[i];
      a.Ub[i] = io.Ub[i];
      a.a1_sel[i] = io.a1_sel[i];
      a.a2_sel[i] = io.a2_sel[i];
      // output of level j (j >= 2, side n >> (j-1)): tmp0 for even j, tmp1 for odd j
      a.llin[i] = lev < p.J ? ((lev + 1) % 2 == 0 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.llout[i] = lev >= 2 ? (lev % 2 == 0 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.S[i] = io.S[i];
    }
    a.beta = io.beta;
    a.dp = dp;
    a.n = p.n;
    a.L = p.L;
    a.P = p.P;
    a.level = lev;
    a.J = p.J;
    a.Ms = p.n >> (lev - 1);
    a.pure = io.pure;
    const int half = a.Ms >> 1;
    a.tiles = (half + kTO - 1) / kTO;
    a.nblocks = a.tiles * a.tiles * p.L;
    dim3 grid(xcd_grid_h(a.nblocks), lev == 1 ? io.nsets : io.nsets * p.P);
    dwt_sy<T, kTO, kNT><<<grid, kNT, 0, s>>>(a);
    MUFFIN_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

template int dwt_analysis<double>(const DwtPlan<double>&, const AnalysisIO<double>&,
                                  const DevParams*, hipStream_t, int, int);
template int dwt_analysis<float>(const DwtPlan<float>&, const AnalysisIO<float>&,
                                 const DevParams*, hipStream_t, int, int);
template int dwt_synthesis<double>(const DwtPlan<double>&, const SynthesisIO<double>&,
                                   const DevParams*, hipStream_t, int, int);
template int dwt_synthesis<float>(const DwtPlan<float>&, const SynthesisIO<float>&,
                                  const DevParams*, hipStream_t, int, int);

}  // namespace muffin
