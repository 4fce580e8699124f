// Spectral analysis operator W_lambda (orthonormal DCT-II along the bands of
// every pixel spectrum; Section 4.2) and its adjoint, fused with the spectral
// dual update of Algorithm 2 (eqs. `vt`, `v`, `upt`) and its derivatives
// (Algorithms 3-4):
//   v~ = v + sigma alpha_n C z,      v <- sat(v~)             (primal)
//   v~' = v' + sigma alpha_n C z',   v' <- 1[|v~|<=1] v~'      (derivative)
//   t  = alpha_n C^T (d1 v + d2 v_b)
// where z is a run-time combination of (2 x~ - x) terms and C the L x L
// DCT-II matrix.  With the band-major layout the DCT of all pixel spectra is
// the product C (L x L) times Z (L x pixels): no transpose is needed.
//
// A block owns 64 (FP32) or 32 (FP64) pixels and all bands; each wave owns 16 pixel
// columns and runs the two products on MFMA 16x16x4 tiles (FP64 or FP32),
// the v update in registers between them.  The pixel tile lives in LDS and is
// overwritten in place by the adjoint input.
#include "internal.hpp"

#include <cmath>
#include <vector>

namespace muffin {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
  typedef dbl4 type;
};
template <>
struct Acc4<float> {
  typedef flt4 type;
};

__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma16(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double dct_coef(int sel, const DevParams* dp) {
  switch (sel) {
    case SEL_ONE: return 1.0;
    case SEL_MU: return dp->mu;
    case SEL_GAMMA: return dp->gamma;
    default: return 0.0;
  }
}

template <typename T>
struct DctArgs {
  const T* xt_a[kMaxSets];
  const T* x_a[kMaxSets];
  const T* xt_b[kMaxSets];
  const T* x_b[kMaxSets];
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  T* V[kMaxSets];
  const T* Vb[kMaxSets];
  int d1_sel[kMaxSets], d2_sel[kMaxSets];
  T* Tout[kMaxSets];
  uint8_t* mask[kMaxSets];
  const T* C;          // [Lp][Lp]
  const double* alpha; // [N] or null
  const DevParams* dp;
  int L, Lp, N;
  int role, pure;
};

// Waves per block (16 pixel columns each): the LDS tile Lp x pixels stays at
// 64 KB for L = 256 in both precisions.
template <typename T>
constexpr int dct_waves() { return sizeof(T) == 8 ? 2 : 4; }
constexpr int kDctMaxKt = 16;  // Lp <= 256

// MFMA 16x16x4 operand layout (64 lanes): A[i][k] with i = lane % 16,
// k = lane / 16; B[k][j] with k = lane / 16, j = lane % 16.  Result r of a
// lane is D[4 (lane / 16) + r][lane % 16] for the FP32 instruction and
// D[lane / 16 + 4 r][lane % 16] for the FP64 one (measured on gfx950).
template <typename T>
__device__ __forceinline__ int out_row(int lk, int r) {
  return sizeof(T) == 8 ? lk + 4 * r : 4 * lk + r;
}
template <typename T>
__global__ void __launch_bounds__(64 * dct_waves<T>()) dct_kernel(DctArgs<T> a) {
  typedef typename Acc4<T>::type acc_t;
  constexpr int kDctWaves = dct_waves<T>();
  constexpr int kDctPix = 16 * kDctWaves;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Z = reinterpret_cast<T*>(smem_raw);  // [Lp][kDctPix]
  const int set = blockIdx.y;
  const int pix0 = blockIdx.x * kDctPix;
  const int L = a.L, Lp = a.Lp, N = a.N;
  const int nkt = Lp >> 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const DevParams* dp = a.dp;

  // ---- stage z = c1 (2 xt_a - x_a) + c2 (2 xt_b - x_b), zero padded ----
  {
    const double c1 = a.pure ? 1.0 : dct_coef(a.c1_sel[set], dp);
    const double c2 = a.pure ? 0.0 : dct_coef(a.c2_sel[set], dp);
    const T* ta = a.xt_a[set];
    const T* xa = a.x_a[set];
    const T* tb = a.xt_b[set];
    const T* xb = a.x_b[set];
    for (int t = threadIdx.x; t < Lp * kDctPix; t += 64 * kDctWaves) {
      const int l = t / kDctPix, j = t - l * kDctPix;
      const int pix = pix0 + j;
      T z = T(0);
      if (l < L && pix < N) {
        const size_t idx = (size_t)l * N + pix;
        if (a.pure) {
          z = xa[idx];
        } else {
          z = T(c1) * (T(2) * ta[idx] - xa[idx]);
          if (xb) z += T(c2) * (T(2) * tb[idx] - xb[idx]);
        }
      }
      Z[t] = z;
    }
  }
  __syncthreads();

  const int jcol = wave * 16 + lr;       // this lane's pixel column in the tile
  const int pix = pix0 + jcol;
  const T* C = a.C;
  acc_t acc[kDctMaxKt];
#pragma unroll
  for (int kt = 0; kt < kDctMaxKt; ++kt) acc[kt] = acc_t{0, 0, 0, 0};

  // ---- product 1 (or the transposed product for the pure adjoint) ----
  const bool trans1 = a.pure == 2;
  for (int l0 = 0; l0 < Lp; l0 += 4) {
    const T b = Z[(l0 + lk) * kDctPix + jcol];
#pragma unroll
    for (int kt = 0; kt < kDctMaxKt; ++kt) {
      if (kt < nkt) {
        const int row = kt * 16 + lr, col = l0 + lk;
        const T av = trans1 ? C[(size_t)col * Lp + row] : C[(size_t)row * Lp + col];
        acc[kt] = mfma16(av, b, acc[kt]);
      }
    }
  }

  if (a.pure) {
    T* out = a.V[set];
#pragma unroll
    for (int kt = 0; kt < kDctMaxKt; ++kt) {
      if (kt < nkt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = kt * 16 + out_row<T>(lk, r);
          if (k < L && pix < N) out[(size_t)k * N + pix] = acc[kt][r];
        }
      }
    }
    return;
  }

  // ---- v update, adjoint input into LDS (own columns only) ----
  const double al = a.alpha ? (pix < N ? a.alpha[pix] : 0.0) : 1.0;
  const T sa = T(dp->sigma * al);
  const T d1 = T(dct_coef(a.d1_sel[set], dp));
  const T d2 = T(dct_coef(a.d2_sel[set], dp));
  T* V = a.V[set];
  const T* Vb = a.Vb[set];
  uint8_t* M = a.mask[set];
#pragma unroll
  for (int kt = 0; kt < kDctMaxKt; ++kt) {
    if (kt < nkt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = kt * 16 + out_row<T>(lk, r);
        T bv = T(0);
        if (k < L && pix < N) {
          const size_t idx = (size_t)k * N + pix;
          const T vt = V[idx] + sa * acc[kt][r];
          T vn;
          if (a.role == ROLE_PRIMAL) {
            vn = vt < T(-1) ? T(-1) : (vt > T(1) ? T(1) : vt);
            if (M) M[idx] = (vt >= T(-1) && vt <= T(1)) ? 1 : 0;
          } else {
            vn = M[idx] ? vt : T(0);
          }
          V[idx] = vn;
          bv = d1 * vn;
          if (Vb) bv += d2 * Vb[idx];
        }
        Z[k * kDctPix + jcol] = bv;
      }
    }
  }
  // LDS reads and writes of one wave execute in order, and each wave only
  // touches its own 16 columns, so no block barrier is needed here.

  // ---- product 2: t = alpha C^T b ----
#pragma unroll
  for (int kt = 0; kt < kDctMaxKt; ++kt) acc[kt] = acc_t{0, 0, 0, 0};
  for (int k0 = 0; k0 < Lp; k0 += 4) {
    const T b = Z[(k0 + lk) * kDctPix + jcol];
#pragma unroll
    for (int lt = 0; lt < kDctMaxKt; ++lt) {
      if (lt < nkt) {
        const T av = C[(size_t)(k0 + lk) * Lp + lt * 16 + lr];  // C^T[l][k]
        acc[lt] = mfma16(av, b, acc[lt]);
      }
    }
  }
  const T ta = T(al);
  T* To = a.Tout[set];
#pragma unroll
  for (int lt = 0; lt < kDctMaxKt; ++lt) {
    if (lt < nkt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int l = lt * 16 + out_row<T>(lk, r);
        if (l < L && pix < N) To[(size_t)l * N + pix] = ta * acc[lt][r];
      }
    }
  }
}

template <typename T>
int dct_make_plan(DctPlan<T>& p, int L, int N, int kind) {
  if (L < 1 || L > 16 * kDctMaxKt) return -2;
  p.L = L;
  p.N = N;
  p.Lp = (L + 15) & ~15;
  p.kind = kind;
  std::vector<T> h((size_t)p.Lp * p.Lp, T(0));
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int k = 0; k < L; ++k) {
    const long double ck = k == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L);
    for (int l = 0; l < L; ++l)
      h[(size_t)k * p.Lp + l] = T(ck * cosl(pi * (2 * l + 1) * k / (2.0L * L)));
  }
  MUFFIN_HIP_CHECK(hipMalloc(&p.C, sizeof(T) * h.size()));
  MUFFIN_HIP_CHECK(hipMemcpy(p.C, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return 0;
}

template <typename T>
void dct_free_plan(DctPlan<T>& p) {
  if (p.C) (void)hipFree(p.C);
  if (p.Chi) (void)hipFree(p.Chi);
  if (p.Clo) (void)hipFree(p.Clo);
  p.C = nullptr;
  p.Chi = p.Clo = nullptr;
}

template <typename T>
int dct_update(const DctPlan<T>& p, const DctIO<T>& io, const DevParams* dp, hipStream_t s) {
  DctArgs<T> a{};
  for (int i = 0; i < io.nsets; ++i) {
    a.xt_a[i] = io.xt_a[i];
    a.x_a[i] = io.x_a[i];
    a.xt_b[i] = io.xt_b[i];
    a.x_b[i] = io.x_b[i];
    a.c1_sel[i] = io.c1_sel[i];
    a.c2_sel[i] = io.c2_sel[i];
    a.V[i] = io.V[i];
    a.Vb[i] = io.Vb[i];
    a.d1_sel[i] = io.d1_sel[i];
    a.d2_sel[i] = io.d2_sel[i];
    a.Tout[i] = io.Tout[i];
    a.mask[i] = io.mask[i];
  }
  a.C = p.C;
  a.alpha = io.alpha;
  a.dp = dp;
  a.L = p.L;
  a.Lp = p.Lp;
  a.N = p.N;
  a.role = io.role;
  a.pure = io.pure;
  constexpr int kDctPix = 16 * dct_waves<T>();
  const size_t shm = sizeof(T) * (size_t)p.Lp * kDctPix;
  dim3 grid((p.N + kDctPix - 1) / kDctPix, io.nsets);
  MUFFIN_ALLOW_BIG_LDS(dct_kernel<T>);
  dct_kernel<T><<<grid, 64 * dct_waves<T>(), shm, s>>>(a);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template int dct_make_plan<double>(DctPlan<double>&, int, int, int);
template int dct_make_plan<float>(DctPlan<float>&, int, int, int);
template void dct_free_plan<double>(DctPlan<double>&);
template void dct_free_plan<float>(DctPlan<float>&);
template int dct_update<double>(const DctPlan<double>&, const DctIO<double>&,
                                const DevParams*, hipStream_t);
template int dct_update<float>(const DctPlan<float>&, const DctIO<float>&,
                               const DevParams*, hipStream_t);

}  // namespace muffin
