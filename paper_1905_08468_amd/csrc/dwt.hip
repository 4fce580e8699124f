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

#ifndef MUFFIN_DWT_MIN_WAVES
#define MUFFIN_DWT_MIN_WAVES 1
#endif
// minimum waves per SIMD the wavelet kernels are compiled for (register cap)
constexpr int kDwtMinWaves = MUFFIN_DWT_MIN_WAVES;
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

// Outputs of one thread in the column filter of a basis: rows kr0 + 2 kp + e
// (e = 0, 1) of column q of the row-filtered tile, low (part 0) and high
// (part 1) pass.  q < TO are the row-low columns, q >= TO the row-high ones.
// Index of output (e, part) in the basis plane, or -1 for the low-low band
// that goes to the next level (or out of range).
template <int TO>
__device__ __forceinline__ long an_out_index(int e, int part, int kr0, int kc0, int half, int n,
                                             bool last) {
  const int q = threadIdx.x % (2 * TO), kp = threadIdx.x / (2 * TO);
  const bool dcol = q >= TO;
  const int kc = kc0 + (dcol ? q - TO : q);
  const int krow = kr0 + 2 * kp + e;
  if (krow >= half || kc >= half) return -1;
  if (part == 0 && !dcol && !last) return -1;
  const int row = part == 0 ? krow : half + krow;
  const int colq = dcol ? half + kc : kc;
  return (long)row * n + colq;
}

// Column filter of basis PB and the dual update (or low-pass output) of this
// thread's four outputs; u/m hold the prefetched dual values and masks.
template <typename T, int TO, int NT, int PB>
__device__ __forceinline__ void an_cols(const AnArgs<T>& a, const T* rowbuf, int set, int band,
                                        int kr0, int kc0, double scale, const T (&u)[4],
                                        const uint8_t (&m)[4]) {
  constexpr int TAPS = 2 * PB;
  T h[TAPS], g[TAPS];
#pragma unroll
  for (int k = 0; k < TAPS; ++k) {
    h[k] = filt_h<T>(PB - 1, k);
    g[k] = filt_g<T>(PB - 1, k);
  }
  const int pidx = PB - 1;
  const int n = a.n, half = a.Ms >> 1;
  const size_t plane = (size_t)n * n;
  T* U = a.U[set] + ((size_t)band * a.P + pidx) * plane;
  uint8_t* M = a.mask[set] ? a.mask[set] + ((size_t)band * a.P + pidx) * plane : nullptr;
  T* llo = a.last ? nullptr : a.llout[set] + ((size_t)band * a.P + pidx) * (size_t)half * half;
  const int q = threadIdx.x % (2 * TO), kp = threadIdx.x / (2 * TO);
  const bool dcol = q >= TO;
  const int kc = kc0 + (dcol ? q - TO : q);
  const int kr = 2 * kp;
  T w[TAPS + 2];
#pragma unroll
  for (int i = 0; i < TAPS + 2; ++i) w[i] = rowbuf[(2 * kr + i) * (2 * TO) + q];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    T lo = T(0), hi = T(0);
#pragma unroll
    for (int k = 0; k < TAPS; ++k) {
      lo += h[k] * w[2 * e + k];
      hi += g[k] * w[2 * e + k];
    }
    const int krow = kr0 + kr + e;
    if (krow >= half || kc >= half) continue;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      const T c = part == 0 ? lo : hi;
      if (part == 0 && !dcol && !a.last) {
        llo[(size_t)krow * half + kc] = c;  // LL goes to the next level
        continue;
      }
      const int row = part == 0 ? krow : half + krow;
      const size_t idx = (size_t)row * n + (dcol ? half + kc : kc);
      if (a.pure) {
        U[idx] = T(a.pure_scale) * c;
        continue;
      }
      const T pv = u[2 * e + part] + T(scale) * c;
      if (a.role == ROLE_PRIMAL) {
        U[idx] = pv < T(-1) ? T(-1) : (pv > T(1) ? T(1) : pv);
        if (M) M[idx] = (pv >= T(-1) && pv <= T(1)) ? 1 : 0;
      } else {
        U[idx] = (M && m[2 * e + part]) ? pv : T(0);
      }
    }
  }
}

// DEEP = false: level 1 (one staged image tile for all bases); true: the
// coarser levels (one low-low tile per basis).  Separate instantiations keep
// the level-1 kernel's register budget free of the per-basis staging.
// PN: number of bases when known at compile time (8, the paper's union of
// db1..db8), or 0 to take it from the arguments; with it known, every basis
// step and every prefetch is unconditional.
template <typename T, int TO, int NT, bool DEEP, int PN>
__global__ void __launch_bounds__(NT, kDwtMinWaves) dwt_an(AnArgs<T> a) {
  static_assert((TO / 2) * (2 * TO) == NT, "one thread per column-filter output quad");
  constexpr int IN = 2 * TO + kHalo;
  __shared__ T s_in[IN * IN];
  __shared__ T s_row[IN * 2 * TO];
  const int lb = xcd_remap_d(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  const int tiles2 = a.tiles * a.tiles;
  const int band = lb / tiles2;
  const int tile = lb - band * tiles2;
  const int kr0 = (tile / a.tiles) * TO, kc0 = (tile % a.tiles) * TO;
  const int set = blockIdx.y;
  const int Ms = a.Ms, msk = Ms - 1, half = Ms >> 1;
  const int n = a.n;
  // Every block runs through all bases: at level 1 they filter the same
  // staged image tile, at the coarser levels each basis filters its own
  // low-low band (the next one is fetched while the current one is filtered).
  const int p0 = 0, p1 = PN ? PN : a.P;
  const size_t plane = (size_t)n * n;
  // ---- dual values and masks this thread updates, one basis ahead ----
  // Loads are unconditional (clamped to a valid element; values of positions
  // the thread does not update are ignored) and land in a slot chosen at
  // compile time, so no register copy makes the wave wait for them before
  // they are used.
  int oidx[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const long idx = an_out_index<TO>(i >> 1, i & 1, kr0, kc0, half, n, a.last);
    oidx[i] = idx < 0 ? 0 : (int)idx;
  }
  const bool has_m = a.role == ROLE_DERIV && a.mask[set] != nullptr;
  T u[2][4];
  uint8_t m[2][4];
  auto fetch_um = [&](int pidx, T (&uo)[4], uint8_t (&mo)[4]) {
    const size_t pl = ((size_t)band * a.P + (pidx < a.P ? pidx : a.P - 1)) * plane;
    const T* U = a.U[set] + pl;
#pragma unroll
    for (int i = 0; i < 4; ++i) uo[i] = U[oidx[i]];
    if (has_m) {  // uniform; mo is only read when has_m
      const uint8_t* M = a.mask[set] + pl;
#pragma unroll
      for (int i = 0; i < 4; ++i) mo[i] = M[oidx[i]];
    }
  };
  fetch_um(0, u[0], m[0]);
  // ---- coarser levels: this thread's tile offsets in a basis' LL plane ----
  // (wrapped into the plane, so every offset is valid, also for t >= IN^2)
  constexpr int NI = (IN * IN + NT - 1) / NT;
  int ioff[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int t = threadIdx.x + i * NT;
    const int r = t / IN, c = t - r * IN;
    ioff[i] = ((2 * kr0 + r) & msk) * Ms + ((2 * kc0 + c) & msk);
  }
  T nxt[NI];
  auto fetch_ll = [&](int pidx) {
    const T* src = a.llin[set] + ((size_t)band * a.P + pidx) * (size_t)Ms * Ms;
#pragma unroll
    for (int i = 0; i < NI; ++i) nxt[i] = src[ioff[i]];
  };
  // ---- stage the input tile (periodic wrap) ----
  if constexpr (!DEEP) {
    // level 1: z = c1 (2 x~ - x) [+ c2 (2 x~b - xb)], all loads issued first
    const double c1 = coef_of(a.c1_sel[set], a.dp), c2 = coef_of(a.c2_sel[set], a.dp);
    const T* xa = a.x_a[set] + (size_t)band * plane;
    const T* ta = a.xt_a[set] + (size_t)band * plane;
    const bool has_b = a.x_b[set] != nullptr;
    const T* xb = has_b ? a.x_b[set] + (size_t)band * plane : xa;
    const T* tb = has_b ? a.xt_b[set] + (size_t)band * plane : ta;
    T v0[NI], v1[NI], v2[NI], v3[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      v0[i] = ta[ioff[i]];
      v1[i] = xa[ioff[i]];
      if (has_b) {
        v2[i] = tb[ioff[i]];
        v3[i] = xb[ioff[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int t = threadIdx.x + i * NT;
      T z = T(c1) * (T(2) * v0[i] - v1[i]);
      if (has_b) z += T(c2) * (T(2) * v2[i] - v3[i]);
      if (t < IN * IN) s_in[t] = z;
    }
  } else {
    fetch_ll(0);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int t = threadIdx.x + i * NT;
      if (t < IN * IN) s_in[t] = nxt[i];
    }
  }
  lds_barrier();
  const double beta = a.beta ? a.beta[band] : 1.0;
  const double scale = a.dp ? a.dp->sigma * beta / sqrt((double)a.P) : 0.0;
#define MUFFIN_AN_STEP(PB)                                                      \
  if (PB - 1 >= p0 && PB - 1 < p1) {                                            \
    const bool more = DEEP && PB < p1;                                          \
    if (more) fetch_ll(PB);                                                     \
    if (PB < p1) fetch_um(PB, u[PB & 1], m[PB & 1]);                            \
    an_rows<T, TO, NT, PB>(s_in, s_row, IN);                                    \
    lds_barrier();                                                            \
    an_cols<T, TO, NT, PB>(a, s_row, set, band, kr0, kc0, scale, u[(PB - 1) & 1], \
                           m[(PB - 1) & 1]);                                    \
    if (more) {                                                                 \
      _Pragma("unroll") for (int i = 0; i < NI; ++i) {                          \
        const int t = threadIdx.x + i * NT;                                     \
        if (t < IN * IN) s_in[t] = nxt[i];                                      \
      }                                                                         \
    }                                                                           \
    lds_barrier();                                                            \
  }
  MUFFIN_AN_STEP(1)
  MUFFIN_AN_STEP(2)
  MUFFIN_AN_STEP(3)
  MUFFIN_AN_STEP(4)
  MUFFIN_AN_STEP(5)
  MUFFIN_AN_STEP(6)
  MUFFIN_AN_STEP(7)
  MUFFIN_AN_STEP(8)
#undef MUFFIN_AN_STEP
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
// c and d column halves) into rbuf[2TC][2 (TC + HAL)].  Each thread slides
// over APT consecutive coefficient rows, so every LDS value it loads feeds
// several outputs.
template <typename T, int TC, int NT, int PB>
__device__ __forceinline__ void sy_cols(const T* q, T* rbuf) {
  constexpr int W = TC + kSHal;
  constexpr int APT = 4;
  constexpr int NA = TC / APT;
  constexpr int NW = APT + PB - 1;
  T he[PB], ho[PB], ge[PB], go[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) {
    he[e] = filt_h<T>(PB - 1, 2 * e);
    ho[e] = filt_h<T>(PB - 1, 2 * e + 1);
    ge[e] = filt_g<T>(PB - 1, 2 * e);
    go[e] = filt_g<T>(PB - 1, 2 * e + 1);
  }
  // q layout: [quad][W][W], quad 0 = low rows / c cols, 1 = high rows / c cols,
  // 2 = low rows / d cols, 3 = high rows / d cols
  for (int t = threadIdx.x; t < NA * 2 * W; t += NT) {
    const int col = t % (2 * W), a0 = (t / (2 * W)) * APT;
    const int hf = col >= W;
    const int cc = hf ? col - W : col;
    const T* ql = q + (hf ? 2 : 0) * W * W + cc;
    const T* qh = q + (hf ? 3 : 1) * W * W + cc;
    // coefficient rows a - e + HAL for a in [a0, a0 + APT), e < PB
    const int row0 = a0 - PB + 1 + kSHal;
    T wl[NW], wh[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      wl[i] = ql[(row0 + i) * W];
      wh[i] = qh[(row0 + i) * W];
    }
#pragma unroll
    for (int a = 0; a < APT; ++a) {
      // explicit FMA chains: two fused operations per tap and output
      T ev = T(0), od = T(0);
#pragma unroll
      for (int e = 0; e < PB; ++e) {
        const T l = wl[a - e + PB - 1], hh = wh[a - e + PB - 1];
        ev = fma(he[e], l, ev);
        ev = fma(ge[e], hh, ev);
        od = fma(ho[e], l, od);
        od = fma(go[e], hh, od);
      }
      rbuf[(2 * (a0 + a)) * (2 * W) + col] = ev;
      rbuf[(2 * (a0 + a) + 1) * (2 * W) + col] = od;
    }
  }
}

// Row synthesis of basis PB, accumulated into acc[b][0..1] = outputs
// (ri, 2 (b0 + b)) and (ri, 2 (b0 + b) + 1) of this thread.
template <typename T, int TC, int NT, int PB>
__device__ __forceinline__ void sy_rows(const T* rbuf, T (&acc)[2][2]) {
  constexpr int W = TC + kSHal;
  constexpr int BPT = 2;
  constexpr int NW = BPT + PB - 1;
  static_assert(2 * TC * (TC / BPT) == NT, "one thread per output quad");
  T he[PB], ho[PB], ge[PB], go[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) {
    he[e] = filt_h<T>(PB - 1, 2 * e);
    ho[e] = filt_h<T>(PB - 1, 2 * e + 1);
    ge[e] = filt_g<T>(PB - 1, 2 * e);
    go[e] = filt_g<T>(PB - 1, 2 * e + 1);
  }
  const int t = threadIdx.x;
  const int ri = t / (TC / BPT), b0 = (t % (TC / BPT)) * BPT;
  const T* rc = rbuf + ri * (2 * W);
  const T* rd = rc + W;
  const int c0 = b0 - PB + 1 + kSHal;
  T wc[NW], wd[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    wc[i] = rc[c0 + i];
    wd[i] = rd[c0 + i];
  }
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    // accumulated straight into acc (FMA chains across the bases)
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      const T c = wc[b - e + PB - 1], d = wd[b - e + PB - 1];
      acc[b][0] = fma(he[e], c, acc[b][0]);
      acc[b][0] = fma(ge[e], d, acc[b][0]);
      acc[b][1] = fma(ho[e], c, acc[b][1]);
      acc[b][1] = fma(go[e], d, acc[b][1]);
    }
  }
}

// Stores a thread's output quad (acc[b][e] -> dst[2 b + e]) scaled by sc;
// only the first pair when the row ends after it.
template <typename T>
__device__ __forceinline__ void store4(T* dst, const T (&acc)[2][2], T sc, bool full) {
  if (full) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4*>(dst) =
          make_float4(sc * acc[0][0], sc * acc[0][1], sc * acc[1][0], sc * acc[1][1]);
    } else {
      reinterpret_cast<double2*>(dst)[0] = make_double2(sc * acc[0][0], sc * acc[0][1]);
      reinterpret_cast<double2*>(dst)[1] = make_double2(sc * acc[1][0], sc * acc[1][1]);
    }
  } else {
    dst[0] = sc * acc[0][0];
    dst[1] = sc * acc[0][1];
  }
}

// DEEP = false: level 1 (the bases' syntheses summed into S); true: the
// coarser levels (one output per basis).
// PN: number of bases when known at compile time, or 0 (see dwt_an).
// UB: the set combines two dual arrays (a1 U_a + a2 U_b, the d/dmu sets).
template <typename T, int TC, int NT, bool DEEP, int PN, bool UB>
__device__ __forceinline__ void sy_block(const SyArgs<T>& a, int lb, T* s_q, T* s_r) {
  constexpr int W = TC + kSHal;
  constexpr int NQ = (4 * W * W + NT - 1) / NT;  // tile values per thread
  const int tiles2 = a.tiles * a.tiles;
  const int band = lb / tiles2;
  const int tile = lb - band * tiles2;
  const int kr0 = (tile / a.tiles) * TC, kc0 = (tile % a.tiles) * TC;
  const int set = blockIdx.y;
  const int n = a.n, Ms = a.Ms, half = Ms >> 1, hm = half - 1;
  const size_t plane = (size_t)n * n;
  const double a1 = a.pure ? 1.0 : coef_of(a.a1_sel[set], a.dp);
  const double a2 = a.pure ? 0.0 : coef_of(a.a2_sel[set], a.dp);
  // Every block runs through all bases (the next basis' tile is fetched while
  // the current one is filtered): at level 1 their syntheses are summed, at
  // the coarser levels each basis has an output of its own.
  const int p0 = 0, p1 = PN ? PN : a.P;
  const bool has_ll = a.level < a.J;
  // this thread's outputs: 4 consecutive values of one row
  const int o0 = 2 * kr0, q0 = 2 * kc0;
  const int ri = threadIdx.x / (TC / 2), b0 = (threadIdx.x % (TC / 2)) * 2;
  const int row = o0 + ri, col = q0 + 2 * b0;
  // coarser levels: store the synthesis of basis pidx and clear acc
  auto store_level = [&](int pidx, T (&acc)[2][2]) {
    if (row < Ms && col < Ms) {
      T* dst = a.llout[set] + ((size_t)band * a.P + pidx) * (size_t)Ms * Ms +
               (size_t)row * Ms + col;
      store4(dst, acc, T(1), col + 3 < Ms);
    }
    acc[0][0] = acc[0][1] = acc[1][0] = acc[1][1] = T(0);
  };
  // Offsets of this thread's tile values inside one basis plane (periodic
  // wrap), computed once: the low-low quadrant reads the coarser level's
  // output (offset in a half x half plane, flagged by a negative value) when
  // there is one, the other quadrants read U.
  // Byte offsets of this thread's tile values inside their source plane
  // (periodic wrap; also valid for the idle tail t >= 4 W^2).  Values of the
  // low-low quadrant (t < W^2) come from the coarser level's output when
  // there is one, the others from U.
  constexpr int Q0 = W * W;
  uint32_t off[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int t = threadIdx.x + i * NT;
    const int quad = t / (W * W), rem = t - quad * W * W;
    const int r = rem / W, c = rem - r * W;
    const int kr = (kr0 - kSHal + r) & hm, kc = (kc0 - kSHal + c) & hm;
    if (quad == 0 && has_ll) {
      off[i] = (uint32_t)((kr * half + kc) * (int)sizeof(T));
    } else {
      const int roff = (quad & 1) ? half : 0, coff = (quad & 2) ? half : 0;
      off[i] = (uint32_t)(((roff + kr) * n + (coff + kc)) * (int)sizeof(T));
    }
  }
  const T ta1 = T(a1), ta2 = T(a2);
  constexpr bool has_ub = UB;
  auto ld = [](const T* base, uint32_t boff) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
  };
  // Raw tile values of one basis: ra from U (or the coarser level's output
  // for the low-low quadrant), rb from the second dual array when the set
  // combines two.  The source of slot i is known from i except for the one
  // slot that straddles the low-low quadrant's end, so the loads take a
  // uniform base and a 32-bit offset; they are unconditional (no branch
  // between a load and its use), so all of them stay in flight while the
  // previous basis is filtered, and the combination is applied when the tile
  // is written to LDS.
  T ra[NQ], rb[NQ];
  auto fetch = [&](int pidx) {
    const T* Ua = a.Ua[set] + ((size_t)band * a.P + pidx) * plane;
    const T* Ub = has_ub ? a.Ub[set] + ((size_t)band * a.P + pidx) * plane : Ua;
    const T* ll = has_ll ? a.llin[set] + ((size_t)band * a.P + pidx) * (size_t)half * half : Ua;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const bool q0 = has_ll && (int)threadIdx.x + i * NT < Q0;
      if constexpr (UB) {
        // two arrays: per-lane source and address (measured faster here
        // than two uniform-base loads per slot); the low-low values of
        // the coarsest level are U values and are combined too
        ra[i] = ld(q0 ? ll : Ua, off[i]);
        rb[i] = ld(Ub, q0 ? 0u : off[i]);
      } else if ((i + 1) * NT <= Q0) {
        ra[i] = ld(ll, off[i]);  // (ll = Ua at the coarsest level)
      } else if (i * NT >= Q0) {
        ra[i] = ld(Ua, off[i]);
      } else {
        ra[i] = ld(q0 ? ll : Ua, off[i]);
      }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int t = threadIdx.x + i * NT;
      if (t < 4 * W * W) {
        const bool q0 = has_ll && t < Q0;
        T v = ra[i];
        if (!q0) {
          v = ta1 * v;
          if (has_ub) v = fma(ta2, rb[i], v);
        }
        s_q[t] = v;
      }
    }
  };
  T acc[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
  fetch(p0);
  commit();
  lds_barrier();
#define MUFFIN_SY_STEP(PB)                                                        \
  if (PB - 1 >= p0 && PB - 1 < p1) {                                              \
    const bool more = PB < p1;                                                    \
    if (more) fetch(PB);                                                          \
    sy_cols<T, TC, NT, PB>(s_q, s_r);                                             \
    lds_barrier();                                                              \
    sy_rows<T, TC, NT, PB>(s_r, acc);                                             \
    if constexpr (DEEP) store_level(PB - 1, acc);                                 \
    if (more) commit();                                                           \
    lds_barrier();                                                              \
  }
  MUFFIN_SY_STEP(1)
  MUFFIN_SY_STEP(2)
  MUFFIN_SY_STEP(3)
  MUFFIN_SY_STEP(4)
  MUFFIN_SY_STEP(5)
  MUFFIN_SY_STEP(6)
  MUFFIN_SY_STEP(7)
  MUFFIN_SY_STEP(8)
#undef MUFFIN_SY_STEP
  // ---- level 1: the sum over bases, scaled by beta_l / sqrt(P) ----
  if (!DEEP && row < Ms && col < Ms) {
    const double beta = a.beta ? a.beta[band] : 1.0;
    T* dst = a.S[set] + (size_t)band * plane + (size_t)row * n + col;
    store4(dst, acc, T(beta / sqrt((double)a.P)), col + 3 < Ms);
  }
}

// One launch per kind of set: UB (the sets combining two dual arrays) or not,
// so each kernel holds one compact instantiation.
template <typename T, int TC, int NT, bool DEEP, int PN, bool UB>
__global__ void __launch_bounds__(NT, kDwtMinWaves) dwt_sy(SyArgs<T> a) {
  constexpr int W = TC + kSHal;
  __shared__ T s_q[4 * W * W];
  __shared__ T s_r[2 * TC * 2 * W];
  const int lb = xcd_remap_d(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  sy_block<T, TC, NT, DEEP, PN, UB>(a, lb, s_q, s_r);
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
    dim3 grid(xcd_grid_h(a.nblocks), io.nsets);
    if (p.P == 8) {
      if (lev == 1)
        dwt_an<T, kTO, kNT, false, 8><<<grid, kNT, 0, s>>>(a);
      else
        dwt_an<T, kTO, kNT, true, 8><<<grid, kNT, 0, s>>>(a);
    } else {
      if (lev == 1)
        dwt_an<T, kTO, kNT, false, 0><<<grid, kNT, 0, s>>>(a);
      else
        dwt_an<T, kTO, kNT, true, 0><<<grid, kNT, 0, s>>>(a);
    }
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
    // two launches: the sets without a second dual array, then those with one
    for (int ub = 0; ub < 2; ++ub) {
      SyArgs<T> a{};
      int ns = 0;
      for (int i = 0; i < io.nsets; ++i) {
        if ((io.Ub[i] != nullptr) != (ub == 1)) continue;
        a.Ua[ns] = io.Ua[i];
        a.Ub[ns] = io.Ub[i];
        a.a1_sel[ns] = io.a1_sel[i];
        a.a2_sel[ns] = io.a2_sel[i];
        // output of level j (j >= 2, side n >> (j-1)): tmp0 for even j, tmp1 for odd j
        a.llin[ns] = lev < p.J ? ((lev + 1) % 2 == 0 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
        a.llout[ns] = lev >= 2 ? (lev % 2 == 0 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
        a.S[ns] = io.S[i];
        ++ns;
      }
      if (ns == 0) continue;
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
      dim3 grid(xcd_grid_h(a.nblocks), ns);
      // (the basis count stays a run-time value here: compiled for P = 8 the
      // fully unrolled kernel needs 137 VGPRs and runs at half the occupancy)
      if (lev == 1) {
        if (ub) dwt_sy<T, kTO, kNT, false, 0, true><<<grid, kNT, 0, s>>>(a);
        else dwt_sy<T, kTO, kNT, false, 0, false><<<grid, kNT, 0, s>>>(a);
      } else {
        if (ub) dwt_sy<T, kTO, kNT, true, 0, true><<<grid, kNT, 0, s>>>(a);
        else dwt_sy<T, kTO, kNT, true, 0, false><<<grid, kNT, 0, s>>>(a);
      }
      MUFFIN_HIP_CHECK(hipGetLastError());
    }
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
