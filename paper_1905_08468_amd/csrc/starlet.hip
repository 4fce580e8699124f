// W_s as the isotropic undecimated wavelet transform (IUWT, "starlet"), the
// other spatial dictionary named in Section 2.1.  With h the cubic B-spline
// filter [1 4 6 4 1] / 16 and H_j the separable periodic smoothing by h
// dilated by 2^(j-1) ("a trous": taps 2^(j-1) apart):
//   analysis   c_0 = z, c_j = H_j c_(j-1), w_j = c_(j-1) - c_j (j = 1..J),
//              W_s z = (w_1, ..., w_J, c_J)              planes [L][J+1][n][n]
//   adjoint    r_J = u_c, r_(j-1) = u_j + H_j (r_j - u_j), W_s^T u = r_0
// (H_j is symmetric, so the adjoint of each scale is the same smoothing).
//
// One launch per scale, every state set in it (blockIdx.y).  A block owns a
// TS x TS tile: it stages the tile and a halo of 2 * 2^(j-1) samples on
// each side in LDS (periodic wrap), filters rows then columns, and applies
// the scale's step at its outputs.  The analysis fuses the dual update of
// the MUFFIN iteration (the same roles as the Daubechies analysis: primal
// step with clip and mask, derivative step under the primal's mask, or a
// plain transform); the synthesis of scale 1 writes beta_l W_s^T u.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace muffin {
namespace {

constexpr int kStTS = 32;   // outputs per tile side
constexpr int kStNT = 256;

template <typename T>
__device__ __forceinline__ T b3(int m) {  // h[m], m = 0..4
  return m == 2 ? T(0.375) : (m == 1 || m == 3 ? T(0.25) : T(0.0625));
}

__device__ __forceinline__ double st_coef(int sel, const DevParams* dp) {
  switch (sel) {
    case SEL_ONE: return 1.0;
    case SEL_MU: return dp->mu;
    case SEL_GAMMA: return dp->gamma;
    default: return 0.0;
  }
}

template <typename T>
struct StArgs {
  // analysis, scale 1: z = c1 z_a + c2 z_b (z = 2 x~ - x of a set)
  const T* z_a[kMaxSets];
  const T* z_b[kMaxSets];
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  // the scale's input plane: analysis c_(j-1) (scales >= 2), synthesis r_j,
  // at in[set] + (band * in_planes + in_plane) * N
  const T* in[kMaxSets];
  int in_planes, in_plane;
  T* out[kMaxSets];          // analysis c_j (j < J) / synthesis r_(j-1) or S
  T* U[kMaxSets];            // [L][J+1][n][n]
  uint8_t* mask[kMaxSets];   // [L][J+1][n][n]
  const double* beta;        // [L] or null (then 1)
  const DevParams* dp;       // null for the plain transform
  int n, L, J, level, planes;
  int role, pure;
  double pure_scale;
  int tiles, nblocks;
};

// Staged tile of a scale with halo R: W = TS + 2 R rows of WC values, the
// output tile's column c at c + CR.  FP32 rows start at a multiple of four
// (halo rounded up to RA >= 4) and are fetched as 16-byte vectors; FP64 rows
// are the W values themselves.
template <typename T>
struct StGeom {
  static constexpr bool V4 = sizeof(T) == 4;
  int R, W, RA, WC, CR;
  __device__ __host__ explicit StGeom(int level) {
    R = 2 << (level - 1);
    W = kStTS + 2 * R;
    RA = V4 ? (R < 4 ? 4 : R) : R;
    WC = kStTS + 2 * RA;
    CR = RA;
  }
};

// fetch the staged tile of one plane (periodic wrap; n % 4 == 0) through f,
// which maps a value of the plane at element g (or a vector at g) to the
// value to stage
template <typename T, typename F>
__device__ __forceinline__ void st_stage(T* s_in, const StGeom<T>& sg, int i0, int j0, int n,
                                         F f) {
  const int msk = n - 1;
  if constexpr (StGeom<T>::V4) {
    const int RE = sg.WC / 4;
    for (int t = threadIdx.x; t < sg.W * RE; t += kStNT) {
      const int r = t / RE, c = (t - r * RE) * 4;
      const size_t g = (size_t)((i0 - sg.R + r) & msk) * n + ((j0 - sg.RA + c) & msk);
      *reinterpret_cast<float4*>(s_in + r * sg.WC + c) = f(g, float4{});
    }
  } else {
    for (int t = threadIdx.x; t < sg.W * sg.WC; t += kStNT) {
      const int r = t / sg.WC, c = t - r * sg.WC;
      s_in[t] = f((size_t)((i0 - sg.R + r) & msk) * n + ((j0 - sg.R + c) & msk), T{});
    }
  }
}

// separable smoothing of the staged tile: rows of s_in into s_row, then the
// column at (r, c) of the output tile
template <typename T>
__device__ __forceinline__ void st_rows(const T* s_in, T* s_row, const StGeom<T>& sg, int d) {
  for (int t = threadIdx.x; t < sg.W * kStTS; t += kStNT) {
    const int r = t / kStTS, c = t - r * kStTS;
    const T* p = s_in + r * sg.WC + c + sg.CR;
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < 5; ++m) acc = fma(b3<T>(m), p[(m - 2) * d], acc);
    s_row[t] = acc;
  }
}

template <typename T>
__device__ __forceinline__ T st_col(const T* s_row, int r, int c, int R, int d) {
  const T* p = s_row + (r + R) * kStTS + c;
  T acc = T(0);
#pragma unroll
  for (int m = 0; m < 5; ++m) acc = fma(b3<T>(m), p[(m - 2) * d * kStTS], acc);
  return acc;
}

// Blocks are handed to the 8 XCDs round-robin; logical block b of XCD x is
// (x * per + b), so neighbouring tiles (which share halo rows) share an L2.
__device__ __forceinline__ int st_remap(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
static inline int st_grid(int nb) { return ((nb + 7) >> 3) << 3; }

// outputs per thread of a tile
constexpr int kStOPT = kStTS * kStTS / kStNT;
static_assert(kStOPT * kStNT == kStTS * kStTS, "whole outputs per thread");

// analysis scale `level` with the fused dual update of planes level-1 (and J)
template <typename T>
__global__ void __launch_bounds__(kStNT) st_an(StArgs<T> a) {
  extern __shared__ __align__(16) unsigned char st_smem[];
  T* s_in = reinterpret_cast<T*>(st_smem);
  const int d = 1 << (a.level - 1), R = 2 * d;
  const StGeom<T> sg(a.level);
  T* s_row = s_in + sg.W * sg.WC;
  const int lb = st_remap(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  const int tiles2 = a.tiles * a.tiles;
  const int band = lb / tiles2, tile = lb - band * tiles2;
  const int i0 = (tile / a.tiles) * kStTS, j0 = (tile % a.tiles) * kStTS;
  const int set = blockIdx.y, n = a.n;
  const size_t N = (size_t)n * n;
  const size_t boff = (size_t)band * N;
  // dual values (and masks) of this thread's outputs, fetched before the
  // tile so their latency overlaps the staging and the filtering (indices
  // of outputs outside the image are clamped to a valid element)
  const bool last = a.level == a.J;
  const bool mask_out = a.role == ROLE_PRIMAL && a.mask[set] != nullptr && !a.pure;
  const bool mask_in = a.role == ROLE_DERIV && a.mask[set] != nullptr;
  T* U = a.U[set];
  uint8_t* M = a.mask[set];
  const size_t pw = ((size_t)band * a.planes + (a.level - 1)) * N;  // plane of w_j
  const size_t pc = ((size_t)band * a.planes + a.J) * N;            // plane of c_J
  size_t opix[kStOPT];
  T uw[kStOPT], uc[kStOPT];
  uint8_t mw[kStOPT], mc[kStOPT];
#pragma unroll
  for (int k = 0; k < kStOPT; ++k) {
    const int t = threadIdx.x + k * kStNT;
    const int r = t / kStTS, c = t - r * kStTS;
    const int gi = min(i0 + r, n - 1), gj = min(j0 + c, n - 1);
    opix[k] = (size_t)gi * n + gj;
    if (!a.pure) {
      uw[k] = U[pw + opix[k]];
      if (last) uc[k] = U[pc + opix[k]];
      if (mask_in) {
        mw[k] = M[pw + opix[k]];
        if (last) mc[k] = M[pc + opix[k]];
      }
    }
  }
  if (a.level == 1) {
    const double c1 = st_coef(a.c1_sel[set], a.dp), c2 = st_coef(a.c2_sel[set], a.dp);
    const T* za = a.z_a[set] + boff;
    const bool has_b = a.z_b[set] != nullptr;
    const T* zb = has_b ? a.z_b[set] + boff : za;
    const T tc1 = T(c1), tc2 = T(c2);
    st_stage(s_in, sg, i0, j0, n, [&](size_t g, auto v) {
      using V = decltype(v);
      V z = *reinterpret_cast<const V*>(za + g);
      z = z * tc1;
      if (has_b) {
        const V b = *reinterpret_cast<const V*>(zb + g);
        z = z + b * tc2;
      }
      return z;
    });
  } else {
    const T* src = a.in[set] + ((size_t)band * a.in_planes + a.in_plane) * N;
    st_stage(s_in, sg, i0, j0, n,
             [&](size_t g, auto v) { return *reinterpret_cast<const decltype(v)*>(src + g); });
  }
  lds_barrier();
  st_rows(s_in, s_row, sg, d);
  lds_barrier();
  const double beta = a.beta ? a.beta[band] : 1.0;
  const T scale = T(a.dp ? a.dp->sigma * beta : 0.0);
  auto update = [&](size_t idx, T val, T uold, uint8_t mold) {
    if (a.pure) {
      U[idx] = T(a.pure_scale) * val;
      return;
    }
    const T pv = uold + scale * val;
    if (a.role == ROLE_PRIMAL) {
      U[idx] = pv < T(-1) ? T(-1) : (pv > T(1) ? T(1) : pv);
      if (mask_out) M[idx] = (pv >= T(-1) && pv <= T(1)) ? 1 : 0;
    } else {
      U[idx] = (mask_in && mold) ? pv : T(0);
    }
  };
#pragma unroll
  for (int k = 0; k < kStOPT; ++k) {
    const int t = threadIdx.x + k * kStNT;
    const int r = t / kStTS, c = t - r * kStTS;
    if (i0 + r >= n || j0 + c >= n) continue;
    const T cj = st_col(s_row, r, c, R, d);
    const T z0 = s_in[(r + R) * sg.WC + c + sg.CR];
    const size_t pix = opix[k];
    update(pw + pix, z0 - cj, uw[k], mw[k]);  // w_j
    if (last)
      update(pc + pix, cj, uc[k], mc[k]);     // the coarse plane c_J
    else
      a.out[set][boff + pix] = cj;            // c_j for the next scale
  }
}

// synthesis scale `level`: r_(level-1) = u_level + H (r_level - u_level)
template <typename T>
__global__ void __launch_bounds__(kStNT) st_sy(StArgs<T> a) {
  extern __shared__ __align__(16) unsigned char st_smem[];
  T* s_in = reinterpret_cast<T*>(st_smem);
  const int d = 1 << (a.level - 1), R = 2 * d;
  const StGeom<T> sg(a.level);
  T* s_row = s_in + sg.W * sg.WC;
  const int lb = st_remap(blockIdx.x, a.nblocks);
  if (lb >= a.nblocks) return;
  const int tiles2 = a.tiles * a.tiles;
  const int band = lb / tiles2, tile = lb - band * tiles2;
  const int i0 = (tile / a.tiles) * kStTS, j0 = (tile % a.tiles) * kStTS;
  const int set = blockIdx.y, n = a.n;
  const size_t N = (size_t)n * n;
  const T* rin = a.in[set] + ((size_t)band * a.in_planes + a.in_plane) * N;
  const T* u = a.U[set] + ((size_t)band * a.planes + (a.level - 1)) * N;
  // u at this thread's outputs, fetched first (clamped indices)
  T uo[kStOPT];
#pragma unroll
  for (int k = 0; k < kStOPT; ++k) {
    const int t = threadIdx.x + k * kStNT;
    const int r = t / kStTS, c = t - r * kStTS;
    uo[k] = u[(size_t)min(i0 + r, n - 1) * n + min(j0 + c, n - 1)];
  }
  st_stage(s_in, sg, i0, j0, n, [&](size_t g, auto v) {
    using V = decltype(v);
    return *reinterpret_cast<const V*>(rin + g) - *reinterpret_cast<const V*>(u + g);
  });
  lds_barrier();
  st_rows(s_in, s_row, sg, d);
  lds_barrier();
  const T sc = T(a.level == 1 && a.beta ? a.beta[band] : 1.0);
  T* out = a.out[set] + (size_t)band * N;
#pragma unroll
  for (int k = 0; k < kStOPT; ++k) {
    const int t = threadIdx.x + k * kStNT;
    const int r = t / kStTS, c = t - r * kStTS;
    const int gi = i0 + r, gj = j0 + c;
    if (gi >= n || gj >= n) continue;
    out[(size_t)gi * n + gj] = sc * (uo[k] + st_col(s_row, r, c, R, d));
  }
}

template <typename T>
size_t st_lds_bytes(int level) {
  const StGeom<T> sg(level);
  return sizeof(T) * ((size_t)sg.W * sg.WC + (size_t)sg.W * kStTS);
}

template <typename T>
int st_prepare(StArgs<T>& a, const StarletPlan& p, int level) {
  a.n = p.n;
  a.L = p.L;
  a.J = p.J;
  a.level = level;
  a.planes = p.J + 1;
  a.tiles = (p.n + kStTS - 1) / kStTS;
  a.nblocks = a.tiles * a.tiles * p.L;
  return 0;
}

}  // namespace

double starlet_norm2(int n, int J) {
  // W_s^T W_s is diagonal in the 2-D DFT; its eigenvalue at (kx, ky) is
  // sum_j |C_(j-1) - C_j|^2 + |C_J|^2 with C_j the product of the scales'
  // (real, separable) filter responses.
  std::vector<std::vector<double>> g(J, std::vector<double>(n));
  const double tw = 2.0 * M_PI / n;
  for (int j = 0; j < J; ++j) {
    const int d = 1 << j;
    for (int k = 0; k < n; ++k) {
      const double w = tw * k * d;
      g[j][k] = (6.0 + 8.0 * std::cos(w) + 2.0 * std::cos(2.0 * w)) / 16.0;
    }
  }
  double best = 0.0;
  for (int kx = 0; kx < n; ++kx)
    for (int ky = 0; ky < n; ++ky) {
      double c = 1.0, s = 0.0;
      for (int j = 0; j < J; ++j) {
        const double cn = c * g[j][kx] * g[j][ky];
        s += (c - cn) * (c - cn);
        c = cn;
      }
      s += c * c;
      best = std::max(best, s);
    }
  return best;
}

template <typename T>
int starlet_analysis(const StarletPlan& p, const AnalysisIO<T>& io, const DevParams* dp,
                     hipStream_t s) {
  for (int lev = 1; lev <= p.J; ++lev) {
    StArgs<T> a{};
    st_prepare(a, p, lev);
    for (int i = 0; i < io.nsets; ++i) {
      a.z_a[i] = io.z_a[i];
      a.z_b[i] = io.z_b[i];
      a.c1_sel[i] = io.c1_sel[i];
      a.c2_sel[i] = io.c2_sel[i];
      a.U[i] = io.U[i];
      a.mask[i] = io.mask[i];
      // c_j lives in tmp0 for odd j, tmp1 for even j
      a.in[i] = lev >= 2 ? ((lev - 1) % 2 == 1 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
      a.out[i] = lev < p.J ? (lev % 2 == 1 ? io.tmp0[i] : io.tmp1[i]) : nullptr;
    }
    a.in_planes = 1;
    a.in_plane = 0;
    a.beta = io.beta;
    a.dp = dp;
    a.role = io.role;
    a.pure = io.pure;
    a.pure_scale = io.pure_scale;
    const size_t shm = st_lds_bytes<T>(lev);
    MUFFIN_ALLOW_BIG_LDS((st_an<T>));
    st_an<T><<<dim3(st_grid(a.nblocks), io.nsets), kStNT, shm, s>>>(a);
    MUFFIN_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

template <typename T>
int starlet_synthesis(const StarletPlan& p, const SynthesisIO<T>& io, hipStream_t s) {
  for (int lev = p.J; lev >= 1; --lev) {
    StArgs<T> a{};
    st_prepare(a, p, lev);
    for (int i = 0; i < io.nsets; ++i) {
      a.U[i] = const_cast<T*>(io.Ua[i]);
      // r_j (j < J) lives in tmp0 for odd j, tmp1 for even j; r_J is the
      // coarse plane of U
      a.in[i] = lev == p.J ? io.Ua[i] : (lev % 2 == 1 ? io.tmp0[i] : io.tmp1[i]);
      a.out[i] = lev == 1 ? io.S[i] : ((lev - 1) % 2 == 1 ? io.tmp0[i] : io.tmp1[i]);
    }
    a.in_planes = lev == p.J ? p.J + 1 : 1;
    a.in_plane = lev == p.J ? p.J : 0;
    a.beta = io.beta;
    const size_t shm = st_lds_bytes<T>(lev);
    MUFFIN_ALLOW_BIG_LDS((st_sy<T>));
    st_sy<T><<<dim3(st_grid(a.nblocks), io.nsets), kStNT, shm, s>>>(a);
    MUFFIN_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

template int starlet_analysis<double>(const StarletPlan&, const AnalysisIO<double>&,
                                      const DevParams*, hipStream_t);
template int starlet_analysis<float>(const StarletPlan&, const AnalysisIO<float>&,
                                     const DevParams*, hipStream_t);
template int starlet_synthesis<double>(const StarletPlan&, const SynthesisIO<double>&,
                                       hipStream_t);
template int starlet_synthesis<float>(const StarletPlan&, const SynthesisIO<float>&,
                                      hipStream_t);

}  // namespace muffin
