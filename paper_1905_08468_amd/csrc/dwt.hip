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
#include <type_traits>
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

// Raw buffer access: a resource over one plane (block-uniform base, size in
// elements; reads past the end return 0, writes past it are dropped) and
// loads/stores at 32-bit byte offsets, so the tile traffic spends no
// per-lane 64-bit address arithmetic.  The base and size are taken from the
// first lane, so the resource is known to be uniform wherever the compiler
// places its computation (a resource it took for divergent would cost a
// loop over lanes at every access).
template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const E* base, size_t count) {
  const uint64_t pv = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)pv);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(pv >> 32));
  const int bytes = __builtin_amdgcn_readfirstlane((int)(count * sizeof(E)));
  return __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, bytes, 0x00020000);
}
// boff: per-lane byte offset; soff: block-uniform byte offset (e.g. of one
// basis' plane inside a resource over all bases of a band)
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t boff, uint32_t soff = 0) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, boff, soff, 0));
  else
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, boff, soff, 0));
}
typedef unsigned int muffin_u32x2 __attribute__((__vector_size__(8)));
typedef float muffin_f32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t boff, T v,
                                       uint32_t soff = 0) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, boff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(muffin_u32x2, v), r, boff, soff, 0);
}

template <typename T>
struct AnArgs {
  const T* z_a[kMaxSets];    // level-1 input z = c1 z_a + c2 z_b
  const T* z_b[kMaxSets];
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  T* U[kMaxSets];
  uint8_t* mask[kMaxSets];   // this level's mask words (uint32 per block thread) or null
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

// Row pitch of the row-filtered tile: odd, so the row filter's stores (four
// rows of eight lanes, four values apart, per 32 lanes) hit distinct banks.
template <int TO>
constexpr int an_pitch() { return 2 * TO + 1; }

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
      rowbuf[r * an_pitch<TO>() + k0 + k] = lo;
      rowbuf[r * an_pitch<TO>() + TO + k0 + k] = hi;
    }
  }
}

// Outputs of one thread in the column filter of a basis: rows kr0 + 2 kp + e
// (e = 0, 1) of column q of the row-filtered tile, low (part 0) and high
// (part 1) pass; q < TO are the row-low columns, q >= TO the row-high ones.
// Output i = 2 e + part updates U at element uoff[i] of the basis plane
// (to_u), except the low-low band, which goes to the next level at element
// loff[e] of its plane (to_ll).  Offsets of unused outputs are 0 (valid
// reads).  The same for every basis: computed once per block.
struct AnLanes {
  uint32_t uoff[4], loff[2];
  bool to_u[4], to_ll[2];
  template <int TO>
  __device__ __forceinline__ void init(int kr0, int kc0, int half, int n, bool last) {
    const int q = threadIdx.x % (2 * TO), kp = threadIdx.x / (2 * TO);
    const bool dcol = q >= TO;
    const int kc = kc0 + (dcol ? q - TO : q);
    const int colq = dcol ? half + kc : kc;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int krow = kr0 + 2 * kp + e;
      const bool ok = krow < half && kc < half;
      const bool ll = !dcol && !last;
      to_ll[e] = ok && ll;
      loff[e] = to_ll[e] ? (uint32_t)(krow * half + kc) : 0u;
      to_u[2 * e] = ok && !ll;
      uoff[2 * e] = to_u[2 * e] ? (uint32_t)(krow * n + colq) : 0u;
      to_u[2 * e + 1] = ok;
      uoff[2 * e + 1] = ok ? (uint32_t)((half + krow) * n + colq) : 0u;
    }
  }
};

// Column filter of basis PB and the dual update (or low-pass output) of this
// thread's four outputs; u holds the prefetched dual values.  The masks
// 1[|p| <= 1] of a thread's outputs are bits 4 (PB - 1) + i of one 32-bit
// word per thread and block (mw): set by the primal role, read by the
// derivative role, whose launch has the same blocks and threads.
// rU, rL: the band's planes of U and of the next level; sU, sL: byte
// offsets of this basis' plane in them.
template <typename T, int TO, int NT, int PB>
__device__ __forceinline__ void an_cols(const AnArgs<T>& a, const T* rowbuf, const AnLanes& ln,
                                        __amdgpu_buffer_rsrc_t rU, __amdgpu_buffer_rsrc_t rL,
                                        uint32_t sU, uint32_t sL, bool mask_out, bool mask_in,
                                        T scale, const T (&u)[4], uint32_t& mw) {
  constexpr int TAPS = 2 * PB;
  T h[TAPS], g[TAPS];
#pragma unroll
  for (int k = 0; k < TAPS; ++k) {
    h[k] = filt_h<T>(PB - 1, k);
    g[k] = filt_g<T>(PB - 1, k);
  }
  const int q = threadIdx.x % (2 * TO), kp = threadIdx.x / (2 * TO);
  const T* col = rowbuf + (4 * kp) * an_pitch<TO>() + q;
  T w[TAPS + 2];
#pragma unroll
  for (int i = 0; i < TAPS + 2; ++i) w[i] = col[i * an_pitch<TO>()];
  auto update = [&](int i, T c) {
    const uint32_t bo = ln.uoff[i] * (uint32_t)sizeof(T);
    if (a.pure) {
      buf_st<T>(rU, bo, T(a.pure_scale) * c, sU);
      return;
    }
    const T pv = u[i] + scale * c;
    if (a.role == ROLE_PRIMAL) {
      buf_st<T>(rU, bo, pv < T(-1) ? T(-1) : (pv > T(1) ? T(1) : pv), sU);
      if (mask_out && pv >= T(-1) && pv <= T(1)) mw |= 1u << (4 * (PB - 1) + i);
    } else {
      buf_st<T>(rU, bo, (mask_in && ((mw >> (4 * (PB - 1) + i)) & 1u)) ? pv : T(0), sU);
    }
  };
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    T lo = T(0), hi = T(0);
#pragma unroll
    for (int k = 0; k < TAPS; ++k) {
      lo += h[k] * w[2 * e + k];
      hi += g[k] * w[2 * e + k];
    }
    if (ln.to_ll[e]) buf_st<T>(rL, ln.loff[e] * (uint32_t)sizeof(T), lo, sL);  // LL: next level
    if (ln.to_u[2 * e]) update(2 * e, lo);
    if (ln.to_u[2 * e + 1]) update(2 * e + 1, hi);
  }
}

// DEEP = false: level 1 (one staged image tile for all bases); true: the
// coarser levels (one low-low tile per basis).  Separate instantiations keep
// the level-1 kernel's register budget free of the per-basis staging.
// PN: number of bases when known at compile time (8, the paper's union of
// db1..db8), or 0 to take it from the arguments; with it known, every basis
// step and every prefetch is unconditional.
// V4 (FP32, input plane side a multiple of four): the input tile is fetched
// as aligned 16-byte vectors (a row of IN values as ceil(IN / 4) of them; the
// values past IN are dropped) and staged as 8-byte pairs, keeping the pitch
// IN of the row filter's reads.
template <typename T, int TO, int NT, bool DEEP, int PN, bool V4>
__global__ void __launch_bounds__(NT, kDwtMinWaves) dwt_an(AnArgs<T> a) {
  static_assert((TO / 2) * (2 * TO) == NT, "one thread per column-filter output quad");
  static_assert(!V4 || sizeof(T) == 4, "vector staging of FP32 tiles");
  constexpr int IN = 2 * TO + kHalo;
  static_assert(IN % 2 == 0, "8-byte aligned pairs in the staged rows");
  __shared__ __align__(16) T s_in[IN * IN];
  __shared__ T s_row[IN * an_pitch<TO>()];
  const int lb = xcd_remap_d(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  const int tiles2 = a.tiles * a.tiles;
  // (block-uniform; kept in scalar registers so plane addressing stays scalar)
  const int band = __builtin_amdgcn_readfirstlane(lb / tiles2);
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
  AnLanes ln;
  ln.init<TO>(kr0, kc0, half, n, a.last);
  const bool has_m = a.role == ROLE_DERIV && a.mask[set] != nullptr;
  const bool mask_out = a.role == ROLE_PRIMAL && a.mask[set] != nullptr && !a.pure;
  // the band's planes of U, masks and next-level outputs (all bases); a
  // basis is selected by a uniform offset (planes a launch does not have:
  // any valid base, never accessed)
  const size_t bpl = (size_t)band * a.P;
  const size_t hh = (size_t)half * half;
  const auto rU = plane_rsrc(a.U[set] + bpl * plane, (size_t)a.P * plane);
  const auto rL = plane_rsrc(a.last ? a.U[set] : a.llout[set] + bpl * hh,
                             a.last ? plane : (size_t)a.P * hh);
  T u[2][4];
  // mask word of this thread (see an_cols); the derivative role reads it once
  uint32_t* mwp = a.mask[set] ? reinterpret_cast<uint32_t*>(a.mask[set]) + (size_t)lb * NT +
                                    threadIdx.x
                              : nullptr;
  uint32_t mw = has_m ? *mwp : 0u;
  auto fetch_um = [&](int pidx, T (&uo)[4]) {
    const uint32_t sp = (uint32_t)((pidx < a.P ? pidx : a.P - 1) * plane);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      uo[i] = buf_ld<T>(rU, ln.uoff[i] * (uint32_t)sizeof(T), sp * (uint32_t)sizeof(T));
  };
  fetch_um(0, u[0]);
  // ---- this thread's tile offsets (bytes) in a plane of side Ms ----
  // (wrapped into the plane, so every offset is valid, also for t >= IN^2;
  // in the vector form the idle tail reads nothing)
  using E = typename std::conditional<V4, muffin_f32x4, T>::type;  // fetched element
  constexpr int VW = V4 ? 4 : 1;               // values per element
  constexpr int RE = (IN + VW - 1) / VW;       // elements per tile row
  constexpr int NI = (IN * RE + NT - 1) / NT;  // elements per thread
  constexpr uint32_t kNone = 0x7ffffff0u;      // past every plane: reads 0, no traffic
  uint32_t ioff[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int t = threadIdx.x + i * NT;
    const int r = t / RE, c = (t - r * RE) * VW;
    ioff[i] = V4 && t >= IN * RE
                  ? kNone
                  : (uint32_t)((((2 * kr0 + r) & msk) * Ms + ((2 * kc0 + c) & msk)) *
                               (int)sizeof(T));
  }
  auto ld = [&](__amdgpu_buffer_rsrc_t r, uint32_t o, uint32_t so) -> E {
    if constexpr (V4)
      return __builtin_bit_cast(muffin_f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, o, so, 0));
    else
      return buf_ld<T>(r, o, so);
  };
  // element i of this thread into the staged tile
  auto stage = [&](int i, const E& v) {
    const int t = threadIdx.x + i * NT;
    if constexpr (V4) {
      const int r = t / RE, c = (t - r * RE) * VW;
      if (t < IN * RE) {
        T* d = s_in + r * IN + c;
        *reinterpret_cast<float2*>(d) = make_float2(v.x, v.y);
        if (c + 2 < IN) *reinterpret_cast<float2*>(d + 2) = make_float2(v.z, v.w);
      }
    } else {
      if (t < IN * IN) s_in[t] = v;
    }
  };
  E nxt[NI];
  const size_t mpl = (size_t)Ms * Ms;
  const auto rI = plane_rsrc(DEEP ? a.llin[set] + bpl * mpl : a.U[set], DEEP ? a.P * mpl : plane);
  auto fetch_ll = [&](int pidx) {
    const uint32_t sp = (uint32_t)(pidx * mpl * sizeof(T));
#pragma unroll
    for (int i = 0; i < NI; ++i) nxt[i] = ld(rI, ioff[i], sp);
  };
  // ---- stage the input tile (periodic wrap) ----
  if constexpr (!DEEP) {
    // level 1: z = c1 z_a [+ c2 z_b] (z = 2 x~ - x of a set), all loads
    // issued first
    const double c1 = coef_of(a.c1_sel[set], a.dp), c2 = coef_of(a.c2_sel[set], a.dp);
    const auto rza = plane_rsrc(a.z_a[set] + (size_t)band * plane, plane);
    const bool has_b = a.z_b[set] != nullptr;
    const auto rzb = plane_rsrc((has_b ? a.z_b[set] : a.z_a[set]) + (size_t)band * plane, plane);
    E va[NI], vb[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      va[i] = ld(rza, ioff[i], 0u);
      if (has_b) vb[i] = ld(rzb, ioff[i], 0u);
    }
    const T tc1 = T(c1), tc2 = T(c2);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      E z = tc1 * va[i];
      if (has_b) z += tc2 * vb[i];
      stage(i, z);
    }
  } else {
    fetch_ll(0);
#pragma unroll
    for (int i = 0; i < NI; ++i) stage(i, nxt[i]);
  }
  lds_barrier();
  const double beta = a.beta ? a.beta[band] : 1.0;
  const T scale = T(a.dp ? a.dp->sigma * beta / sqrt((double)a.P) : 0.0);
  auto cols = [&](auto pb, const T (&uu)[4]) {
    constexpr int PB = decltype(pb)::value;
    const uint32_t sp = (uint32_t)((PB - 1) * plane);
    an_cols<T, TO, NT, PB>(a, s_row, ln, rU, rL, sp * (uint32_t)sizeof(T),
                           (uint32_t)((PB - 1) * hh * sizeof(T)), mask_out, has_m, scale, uu, mw);
  };
#define MUFFIN_AN_STEP(PB)                                                      \
  if (PB - 1 >= p0 && PB - 1 < p1) {                                            \
    const bool more = DEEP && PB < p1;                                          \
    if (more) fetch_ll(PB);                                                     \
    if (PB < p1) fetch_um(PB, u[PB & 1]);                                       \
    an_rows<T, TO, NT, PB>(s_in, s_row, IN);                                    \
    lds_barrier();                                                            \
    cols(std::integral_constant<int, PB>{}, u[(PB - 1) & 1]);                   \
    if (more) {                                                                 \
      _Pragma("unroll") for (int i = 0; i < NI; ++i) stage(i, nxt[i]);          \
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
  if (mask_out) *mwp = mw;
}

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------
template <typename T>
struct SyArgs {
  const T* Ua[kMaxSets];
  const T* llin[kMaxSets];   // level < J: [L][P][half^2]
  T* llout[kMaxSets];        // level >= 2: [L][P][Ms^2]
  T* S[kMaxSets];            // level 1: [L][n][n]
  const double* beta;        // [L] or null (then 1)
  int n, L, P, level, J;
  int Ms, tiles, nblocks;
};

// Per-thread LDS positions of the separable synthesis, the same for every
// basis (computed once per block): the column pass slides over APT
// coefficient rows of one column of a quadrant pair, the row pass produces
// 2 BPT consecutive outputs of one row.  V4: the staged tile's rows start
// one column earlier (at a multiple of four) and have WC = W + 1 columns, so
// that they are fetched as aligned 16-byte vectors; column CO of a staged
// row is the first one the filters read.
template <int TC, int NT, int APT_, int BPT_, bool V4 = false>
struct SyLanes {
  static constexpr int W = TC + kSHal;
  static constexpr int WC = V4 ? W + 1 : W;
  static constexpr int CO = V4 ? 1 : 0;
  static constexpr int QS = W * WC;  // values of one staged quadrant
  // row pitch of rbuf: odd, so the row pass's reads (8 rows x 8 lanes per
  // wave, 4 values apart within a row) spread over all banks
  static constexpr int RP = 2 * W + 1;
  static constexpr int APT = APT_;
  static constexpr int BPT = BPT_;
  static constexpr int NA = TC / APT;
  static_assert(NA * 2 * W <= NT, "one column-pass item per thread");
  static_assert(2 * TC * (TC / BPT) == NT, "one row-pass output group per thread");
  bool col_on;
  int ql, qh;   // column pass: first coefficient (row a0) of the low/high quadrant
  int rout;     // column pass: first output (row 2 a0, column col) in rbuf
  int rc;       // row pass: first value (column b0) of the c half of row ri
  __device__ __forceinline__ SyLanes() {
    const int t = threadIdx.x;
    col_on = t < NA * 2 * W;
    const int col = t % (2 * W), a0 = (t / (2 * W)) * APT;
    const int hf = col >= W;
    const int cc = hf ? col - W : col;
    ql = (hf ? 2 : 0) * QS + a0 * WC + cc + CO;
    qh = ql + QS;
    rout = (2 * a0) * RP + col;
    const int ri = t / (TC / BPT), b0 = (t % (TC / BPT)) * BPT;
    rc = ri * RP + b0;
  }
};

// Column synthesis of basis PB: from the four quadrants (low/high rows of the
// c and d column halves) into rbuf[2TC][2 (TC + HAL) + 1].  Each thread slides
// over APT consecutive coefficient rows, so every LDS value it loads feeds
// several outputs.  Window entry i holds coefficient row a0 + HAL + 1 - PB + i
// (output a - a0 uses entries a - a0 - e + PB - 1, e < PB), so every LDS
// offset from the thread's base is a compile-time constant.
template <typename T, int PB, typename Lanes>
__device__ __forceinline__ void sy_cols(const T* q, T* rbuf, const Lanes& ln) {
  constexpr int W = Lanes::W;
  constexpr int APT = Lanes::APT;
  constexpr int NW = APT + PB - 1;
  constexpr int R0 = kSHal + 1 - PB;  // first window row relative to a0
  T he[PB], ho[PB], ge[PB], go[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) {
    he[e] = filt_h<T>(PB - 1, 2 * e);
    ho[e] = filt_h<T>(PB - 1, 2 * e + 1);
    ge[e] = filt_g<T>(PB - 1, 2 * e);
    go[e] = filt_g<T>(PB - 1, 2 * e + 1);
  }
  // q layout: [quad][W][WC], quad 0 = low rows / c cols, 1 = high rows / c cols,
  // 2 = low rows / d cols, 3 = high rows / d cols
  if (ln.col_on) {
    const T* ql = q + ln.ql;
    const T* qh = q + ln.qh;
    T wl[NW], wh[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      wl[i] = ql[(R0 + i) * Lanes::WC];
      wh[i] = qh[(R0 + i) * Lanes::WC];
    }
    T* out = rbuf + ln.rout;
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
      out[(2 * a) * Lanes::RP] = ev;
      out[(2 * a + 1) * Lanes::RP] = od;
    }
  }
}

// Row synthesis of basis PB, accumulated into acc[b][0..1] = outputs
// (ri, 2 (b0 + b)) and (ri, 2 (b0 + b) + 1) of this thread.
template <typename T, int PB, typename Lanes>
__device__ __forceinline__ void sy_rows(const T* rbuf, T (&acc)[Lanes::BPT][2], const Lanes& ln) {
  constexpr int W = Lanes::W;
  constexpr int BPT = Lanes::BPT;
  constexpr int NW = BPT + PB - 1;
  constexpr int C0 = kSHal + 1 - PB;  // first window column relative to b0
  T he[PB], ho[PB], ge[PB], go[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) {
    he[e] = filt_h<T>(PB - 1, 2 * e);
    ho[e] = filt_h<T>(PB - 1, 2 * e + 1);
    ge[e] = filt_g<T>(PB - 1, 2 * e);
    go[e] = filt_g<T>(PB - 1, 2 * e + 1);
  }
  const T* rc = rbuf + ln.rc;
  const T* rd = rc + W;
  T wc[NW], wd[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    wc[i] = rc[C0 + i];
    wd[i] = rd[C0 + i];
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

// Stores a thread's 2 BPT outputs (acc[b][e] -> dst[2 b + e]) scaled by sc,
// those before the row's end (room = values left in the row; groups of four,
// or the first pair only when the row is shorter than four).
template <typename T, int BPT>
__device__ __forceinline__ void store_row(T* dst, const T (&acc)[BPT][2], T sc, int room) {
#pragma unroll
  for (int g = 0; g < BPT / 2; ++g) {
    const T(&a0)[2] = acc[2 * g];
    const T(&a1)[2] = acc[2 * g + 1];
    T* d = dst + 4 * g;
    if (room >= 4 * g + 4) {
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(d) = make_float4(sc * a0[0], sc * a0[1], sc * a1[0], sc * a1[1]);
      } else {
        reinterpret_cast<double2*>(d)[0] = make_double2(sc * a0[0], sc * a0[1]);
        reinterpret_cast<double2*>(d)[1] = make_double2(sc * a1[0], sc * a1[1]);
      }
    } else if (room > 4 * g) {
      d[0] = sc * a0[0];
      d[1] = sc * a0[1];
    }
  }
}

// DEEP = false: level 1 (the bases' syntheses summed into S); true: the
// coarser levels (one output per basis).
// PN: number of bases when known at compile time, or 0 (see dwt_an).
// V4 (FP32, half-plane side a multiple of four): the tile is staged as
// 16-byte vectors (see SyLanes).
template <typename T, int TC, int NT, int APT, int BPT, bool DEEP, int PN, bool V4>
__device__ __forceinline__ void sy_block(const SyArgs<T>& a, int lb, T* s_q, T* s_r) {
  static_assert(!V4 || sizeof(T) == 4, "vector staging of FP32 tiles");
  using Lanes = SyLanes<TC, NT, APT, BPT, V4>;
  using E = typename std::conditional<V4, muffin_f32x4, T>::type;  // staged element
  constexpr int VW = V4 ? 4 : 1;                  // values per element
  constexpr int W = TC + kSHal;
  constexpr int RE = Lanes::WC / VW;              // elements per staged row
  constexpr int QE = W * RE;                      // elements per quadrant
  constexpr int NQ = (4 * QE + NT - 1) / NT;      // elements per thread
  const int tiles2 = a.tiles * a.tiles;
  // (block-uniform; kept in scalar registers so plane addressing stays scalar)
  const int band = __builtin_amdgcn_readfirstlane(lb / tiles2);
  const int tile = lb - band * tiles2;
  const int kr0 = (tile / a.tiles) * TC, kc0 = (tile % a.tiles) * TC;
  const int set = blockIdx.y;
  const int n = a.n, Ms = a.Ms, half = Ms >> 1, hm = half - 1;
  const size_t plane = (size_t)n * n;
  // Every block runs through all bases (the next basis' tile is fetched while
  // the current one is filtered): at level 1 their syntheses are summed, at
  // the coarser levels each basis has an output of its own.
  const int p0 = 0, p1 = PN ? PN : a.P;
  const bool has_ll = a.level < a.J;
  // this thread's outputs: 2 BPT consecutive values of one row
  const int o0 = 2 * kr0, q0 = 2 * kc0;
  const int ri = threadIdx.x / (TC / BPT), b0 = (threadIdx.x % (TC / BPT)) * BPT;
  const int row = o0 + ri, col = q0 + 2 * b0;
  // coarser levels: store the synthesis of basis pidx and clear acc
  auto store_level = [&](int pidx, T (&acc)[BPT][2]) {
    if (row < Ms && col < Ms) {
      T* dst = a.llout[set] + ((size_t)band * a.P + pidx) * (size_t)Ms * Ms +
               (size_t)row * Ms + col;
      store_row<T, BPT>(dst, acc, T(1), Ms - col);
    }
#pragma unroll
    for (int b = 0; b < BPT; ++b) acc[b][0] = acc[b][1] = T(0);
  };
  // Offsets of this thread's tile values inside one basis plane (periodic
  // wrap), computed once: the low-low quadrant reads the coarser level's
  // output (offset in a half x half plane, flagged by a negative value) when
  // there is one, the other quadrants read U.
  // Byte offsets of this thread's tile values inside their source plane
  // (periodic wrap; the idle tail t >= 4 QE reads nothing in the vector
  // form, a valid value otherwise).  Values of the low-low quadrant (t < QE)
  // come from the coarser level's output when there is one, the others from
  // U.  A vector never straddles the wrap (both are multiples of four).
  constexpr int Q0 = QE;
  constexpr uint32_t kNone = 0x7ffffff0u;  // past every plane: reads 0, no traffic
  uint32_t off[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int t = threadIdx.x + i * NT;
    const int quad = t / QE, rem = t - quad * QE;
    const int r = rem / RE, c = (rem - r * RE) * VW;
    const int kr = (kr0 - kSHal + r) & hm, kc = (kc0 - kSHal - Lanes::CO + c) & hm;
    if (V4 && t >= 4 * QE) {
      off[i] = kNone;
    } else if (quad == 0 && has_ll) {
      off[i] = (uint32_t)((kr * half + kc) * (int)sizeof(T));
    } else {
      const int roff = (quad & 1) ? half : 0, coff = (quad & 2) ? half : 0;
      off[i] = (uint32_t)(((roff + kr) * n + (coff + kc)) * (int)sizeof(T));
    }
  }
  // Raw tile values of one basis, from U (or the coarser level's output for
  // the low-low quadrant).  The source of slot i is known from i except for
  // the one slot that straddles the low-low quadrant's end (loaded from both
  // planes, then selected).  The loads are unconditional (no branch between
  // a load and its use), so all of them stay in flight while the previous
  // basis is filtered.
  E ra[NQ];
  auto ld = [&](__amdgpu_buffer_rsrc_t r, uint32_t o) -> E {
    if constexpr (V4)
      return __builtin_bit_cast(muffin_f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0));
    else
      return buf_ld<T>(r, o);
  };
  auto fetch = [&](int pidx) {
    const auto ru = plane_rsrc(a.Ua[set] + ((size_t)band * a.P + pidx) * plane, plane);
    const auto rl = has_ll ? plane_rsrc(a.llin[set] + ((size_t)band * a.P + pidx) *
                                            (size_t)half * half, (size_t)half * half)
                           : ru;  // (the coarsest level reads U everywhere)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      if ((i + 1) * NT <= Q0) {
        ra[i] = ld(rl, off[i]);
      } else if (i * NT >= Q0) {
        ra[i] = ld(ru, off[i]);
      } else {
        const bool q0 = has_ll && (int)threadIdx.x + i * NT < Q0;
        const E vl = ld(rl, q0 ? off[i] : (V4 ? kNone : 0u));
        const E vu = ld(ru, V4 && q0 ? kNone : off[i]);
        ra[i] = q0 ? vl : vu;
      }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int t = threadIdx.x + i * NT;
      if (t < 4 * QE) reinterpret_cast<E*>(s_q)[t] = ra[i];
    }
  };
  const Lanes lanes;
  T acc[BPT][2];
#pragma unroll
  for (int b = 0; b < BPT; ++b) acc[b][0] = acc[b][1] = T(0);
  fetch(p0);
  commit();
  lds_barrier();
#define MUFFIN_SY_STEP(PB)                                                        \
  if (PB - 1 >= p0 && PB - 1 < p1) {                                              \
    const bool more = PB < p1;                                                    \
    if (more) fetch(PB);                                                          \
    sy_cols<T, PB>(s_q, s_r, lanes);                                              \
    lds_barrier();                                                              \
    sy_rows<T, PB>(s_r, acc, lanes);                                              \
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
    store_row<T, BPT>(dst, acc, T(beta / sqrt((double)a.P)), Ms - col);
  }
}

// TC x TC coefficient tiles of every quadrant per block (2 TC x 2 TC outputs).
template <typename T, int TC, int NT, int APT, int BPT, bool DEEP, int PN, bool V4>
__global__ void __launch_bounds__(NT, kDwtMinWaves) dwt_sy(SyArgs<T> a) {
  constexpr int W = TC + kSHal;
  __shared__ __align__(16) T s_q[4 * SyLanes<TC, NT, APT, BPT, V4>::QS];
  __shared__ T s_r[2 * TC * (2 * W + 1)];
  const int lb = xcd_remap_d(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  sy_block<T, TC, NT, APT, BPT, DEEP, PN, V4>(a, lb, s_q, s_r);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int kTO = 16;
constexpr int kNT = 256;
constexpr int kSyTC1 = 32;   // level-1 synthesis tile (coefficients per side)
constexpr int kSyNT1 = 512;
constexpr int kAnTO1 = 32;   // level-1 analysis tile (outputs per subband side)
constexpr int kAnNT1 = 1024;

template <typename T>
int dwt_analysis(const DwtPlan<T>& p, const AnalysisIO<T>& io, const DevParams* dp,
                 hipStream_t s, int lev_lo, int lev_hi) {
  if (lev_lo <= 0) lev_lo = 1;
  if (lev_hi <= 0 || lev_hi > p.J) lev_hi = p.J;
  // launch shape of a level: FP32 with the paper's 8 bases, subbands of side
  // >= 64: 32 x 32 output tiles per subband (input halo re-reads
  // (64 + 14)^2 / 64^2 = 1.49x instead of (32 + 14)^2 / 32^2 = 2.07x)
  constexpr bool big = sizeof(T) == 4;
  auto shape = [&](int lev, bool& wide, int& tiles, int& nblocks, int& nt) {
    const int half = (p.n >> (lev - 1)) >> 1;
    wide = big && p.P == 8 && (lev == 1 && p.an_tile1 ? p.an_tile1 == kAnTO1 : half >= 64);
    const int to = wide ? kAnTO1 : kTO;
    tiles = (half + to - 1) / to;
    nblocks = tiles * tiles * p.L;
    nt = wide ? kAnNT1 : kNT;
  };
  // mask words of the levels one after another (the primal and derivative
  // roles of a level have the same launch shape)
  size_t woff = 0;
  for (int lev = 1; lev < lev_lo; ++lev) {
    bool w;
    int t, nb, nt;
    shape(lev, w, t, nb, nt);
    woff += (size_t)nb * nt;
  }
  for (int lev = lev_lo; lev <= lev_hi; ++lev) {
    bool wide;
    int tiles, nblocks, nt;
    shape(lev, wide, tiles, nblocks, nt);
    AnArgs<T> a{};
    for (int i = 0; i < io.nsets; ++i) {
      a.z_a[i] = io.z_a[i];
      a.z_b[i] = io.z_b[i];
      a.c1_sel[i] = io.c1_sel[i];
      a.c2_sel[i] = io.c2_sel[i];
      a.U[i] = io.U[i];
      a.mask[i] = io.mask[i] ? reinterpret_cast<uint8_t*>(reinterpret_cast<uint32_t*>(io.mask[i]) +
                                                          woff)
                             : nullptr;
      // LL_j lives in tmp0 for odd j, tmp1 for even j
      a.llin[i] = lev >= 2 ? ((lev - 1) % 2 == 1 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.llout[i] = lev % 2 == 1 ? io.tmp0[i] : io.tmp1[i];
    }
    woff += (size_t)nblocks * nt;
    a.beta = io.beta;
    a.dp = dp;
    a.n = p.n;
    a.L = p.L;
    a.P = p.P;
    a.level = lev;
    a.last = lev == p.J;
    a.Ms = p.n >> (lev - 1);
    a.tiles = tiles;
    a.nblocks = nblocks;
    a.role = io.role;
    a.pure = io.pure;
    a.pure_scale = io.pure_scale;
    dim3 grid(xcd_grid_h(a.nblocks), io.nsets);
    // FP32 input tiles are fetched as aligned 16-byte vectors when the
    // input plane's side is a multiple of four (no vector straddles the wrap)
    const bool v4 = big && a.Ms % 4 == 0;
    if (wide) {
      if constexpr (big) {
        if (lev == 1)
          dwt_an<T, kAnTO1, kAnNT1, false, 8, true><<<grid, kAnNT1, 0, s>>>(a);
        else
          dwt_an<T, kAnTO1, kAnNT1, true, 8, true><<<grid, kAnNT1, 0, s>>>(a);
      }
    } else if (p.P == 8) {
      if (lev == 1) {
        if (v4) dwt_an<T, kTO, kNT, false, 8, big><<<grid, kNT, 0, s>>>(a);
        else dwt_an<T, kTO, kNT, false, 8, false><<<grid, kNT, 0, s>>>(a);
      } else {
        if (v4) dwt_an<T, kTO, kNT, true, 8, big><<<grid, kNT, 0, s>>>(a);
        else dwt_an<T, kTO, kNT, true, 8, false><<<grid, kNT, 0, s>>>(a);
      }
    } else {
      if (lev == 1) {
        if (v4) dwt_an<T, kTO, kNT, false, 0, big><<<grid, kNT, 0, s>>>(a);
        else dwt_an<T, kTO, kNT, false, 0, false><<<grid, kNT, 0, s>>>(a);
      } else {
        if (v4) dwt_an<T, kTO, kNT, true, 0, big><<<grid, kNT, 0, s>>>(a);
        else dwt_an<T, kTO, kNT, true, 0, false><<<grid, kNT, 0, s>>>(a);
      }
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
    SyArgs<T> a{};
    for (int i = 0; i < io.nsets; ++i) {
      a.Ua[i] = io.Ua[i];
      // output of level j (j >= 2, side n >> (j-1)): tmp0 for even j, tmp1 for odd j
      a.llin[i] = lev < p.J ? ((lev + 1) % 2 == 0 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.llout[i] = lev >= 2 ? (lev % 2 == 0 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.S[i] = io.S[i];
    }
    a.beta = io.beta;
    a.n = p.n;
    a.L = p.L;
    a.P = p.P;
    a.level = lev;
    a.J = p.J;
    a.Ms = p.n >> (lev - 1);
    const int half = a.Ms >> 1;
    // level 1 in FP32: 32 x 32 coefficient tiles, whose halo re-reads
    // (39^2 / 32^2 = 1.49x) are far below those of 16 x 16 tiles
    // (23^2 / 16^2 = 2.07x); FP64 (twice the LDS per tile) and the coarser
    // levels keep 16 x 16 (measured: no gain there)
    constexpr bool big = sizeof(T) == 4;
    const bool wide = big && lev == 1 && (p.syn_tile1 ? p.syn_tile1 == kSyTC1 : half >= 64);
    const int tc = wide ? kSyTC1 : kTO;
    a.tiles = (half + tc - 1) / tc;
    a.nblocks = a.tiles * a.tiles * p.L;
    dim3 grid(xcd_grid_h(a.nblocks), io.nsets);
    // (the basis count stays a run-time value here: compiled for P = 8 the
    // fully unrolled kernel needs 137 VGPRs and runs at half the occupancy)
    // FP32 tiles are staged as aligned 16-byte vectors when the half-plane
    // side is a multiple of four (no vector then straddles the wrap)
    const bool v4 = big && half % 4 == 0;
    if (wide) {
      if constexpr (big) dwt_sy<T, kSyTC1, kSyNT1, 8, 4, false, 0, true><<<grid, kSyNT1, 0, s>>>(a);
    } else if (lev == 1) {
      if (v4) dwt_sy<T, kTO, kNT, 4, 2, false, 0, big><<<grid, kNT, 0, s>>>(a);
      else dwt_sy<T, kTO, kNT, 4, 2, false, 0, false><<<grid, kNT, 0, s>>>(a);
    } else {
      if (v4) dwt_sy<T, kTO, kNT, 4, 2, true, 0, big><<<grid, kNT, 0, s>>>(a);
      else dwt_sy<T, kTO, kNT, 4, 2, true, 0, false><<<grid, kNT, 0, s>>>(a);
    }
    MUFFIN_HIP_CHECK(hipGetLastError());
  }
  return 0;
}
size_t dwt_mask_words(int n, int L, int J, int P, int elem_bytes) {
  size_t words = 0;
  for (int lev = 1; lev <= J; ++lev) {
    const int half = (n >> (lev - 1)) >> 1;
    const size_t t16 = (size_t)((half + kTO - 1) / kTO), t32 = (size_t)((half + kAnTO1 - 1) / kAnTO1);
    size_t w = t16 * t16 * kNT;
    if (elem_bytes == 4 && P == 8) w = std::max(w, t32 * t32 * (size_t)kAnNT1);
    words += w * (size_t)L;
  }
  return words;
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
