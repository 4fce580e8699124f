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
// A block owns 64 (FP32) or 32 (FP64) pixels and all bands, staged in LDS;
// its 8 waves split the output rows and run the two products on MFMA
// 16x16x4 tiles (FP64 or FP32) with the v update in registers between them.
// The DCT matrix is stored in MFMA fragment order so every operand load is one
// coalesced 64-lane read.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
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
  const T* z_a[kMaxSets];    // input z = c1 z_a + c2 z_b
  const T* z_b[kMaxSets];
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  T* V[kMaxSets];
  const T* Vb[kMaxSets];
  int d1_sel[kMaxSets], d2_sel[kMaxSets];
  T* Tout[kMaxSets];
  uint8_t* mask[kMaxSets];
  const T* Cf1;        // C in MFMA A-fragment order:   [kt][ks][lane]
  const T* Cf2;        // C^T in MFMA A-fragment order: [lt][ks][lane]
  const double* alpha; // [N] or null
  const DevParams* dp;
  int L, Lp, N;
  int role, pure;
};

#ifndef MUFFIN_DCT_WAVES
#define MUFFIN_DCT_WAVES 8
#endif
constexpr int kDctWaves = MUFFIN_DCT_WAVES;  // waves per block of the FP32/FP64 kernel
constexpr int kDctMaxKt = 16;  // Lp <= 256
constexpr int kDctKtPerWave = kDctMaxKt / kDctWaves;
static_assert(4 * 4 * kDctKtPerWave <= 32, "a thread's DCT mask bits fit one word");

// Column groups (16 pixels each) per block: the LDS tile Lp x pixels is
// 64 KB at L = 256 in both precisions.
template <typename T>
constexpr int dct_groups() { return sizeof(T) == 8 ? 2 : 4; }

// MFMA 16x16x4 operand layout (64 lanes): A[i][k] with i = lane % 16,
// k = lane / 16; B[k][j] with k = lane / 16, j = lane % 16.  Result r of a
// lane is D[4 (lane / 16) + r][lane % 16] for the FP32 instruction and
// D[lane / 16 + 4 r][lane % 16] for the FP64 one (measured on gfx950).
template <typename T>
__device__ __forceinline__ int out_row(int lk, int r) {
  return sizeof(T) == 8 ? lk + 4 * r : 4 * lk + r;
}

// Block = kDctWaves waves x (16 * G) pixels.  Wave w owns the output row
// tiles w, w + kDctWaves, ... for every pixel group, so each A fragment
// (read coalesced from the fragment-ordered matrix) feeds G MFMAs.  Eight
// waves (two output tiles each) rather than four: the block's 64 KB of LDS
// allows two blocks per CU, and the per-wave accumulators then fit in 128
// VGPRs, so a SIMD holds four waves instead of two to cover the latency of
// the operand loads.
template <typename T>
__global__ void __launch_bounds__(64 * kDctWaves, 2) dct_kernel(DctArgs<T> a) {
  typedef typename Acc4<T>::type acc_t;
  constexpr int G = dct_groups<T>();
  constexpr int PIX = 16 * G;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Z = reinterpret_cast<T*>(smem_raw);  // [Lp][PIX]
  const int set = blockIdx.y;
  const int pix0 = blockIdx.x * PIX;
  const int L = a.L, Lp = a.Lp, N = a.N;
  const int nkt = Lp >> 4, nks = Lp >> 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const DevParams* dp = a.dp;

  // ---- stage z = c1 z_a + c2 z_b (the operand itself for pure), zero padded ----
  {
    const double c1 = a.pure ? 1.0 : dct_coef(a.c1_sel[set], dp);
    const double c2 = a.pure ? 0.0 : dct_coef(a.c2_sel[set], dp);
    // Operands of U items are loaded unconditionally (indices clamped into
    // the cube; out-of-range items are zeroed afterwards) before any is
    // used, so they are all in flight together.
    const T* za = a.z_a[set];
    const bool has_b = !a.pure && a.z_b[set] != nullptr;
    const T* zb = has_b ? a.z_b[set] : za;
    constexpr int U = 8;
    constexpr int NT = 64 * kDctWaves;
    const int total = Lp * PIX;
    for (int t0 = threadIdx.x; t0 < total; t0 += U * NT) {
      T va[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = min(t0 + u * NT, total - 1);
        const int l = t / PIX, j = t - l * PIX;
        const size_t idx = (size_t)min(l, L - 1) * N + min(pix0 + j, N - 1);
        va[u] = za[idx];
        if (has_b) vb[u] = zb[idx];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * NT;
        if (t < total) {
          const int l = t / PIX, j = t - l * PIX;
          T z = T(0);
          if (l < L && pix0 + j < N) {
            z = T(c1) * va[u];
            if (has_b) z += T(c2) * vb[u];
          }
          Z[t] = z;
        }
      }
    }
  }
  lds_barrier();

  acc_t acc[kDctKtPerWave][G];
#pragma unroll
  for (int i = 0; i < kDctKtPerWave; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[i][g] = acc_t{0, 0, 0, 0};

  // ---- product 1: C Z (pure == 2: C^T Z) ----
  const T* A1 = a.pure == 2 ? a.Cf2 : a.Cf1;
  for (int ks = 0; ks < nks; ++ks) {
    T b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) b[g] = Z[(4 * ks + lk) * PIX + 16 * g + lr];
#pragma unroll
    for (int i = 0; i < kDctKtPerWave; ++i) {
      const int kt = wave + kDctWaves * i;
      if (kt < nkt) {
        const T av = A1[((size_t)kt * nks + ks) * 64 + lane];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[i][g] = mfma16(av, b[g], acc[i][g]);
      }
    }
  }

  if (a.pure) {
    T* out = a.V[set];
#pragma unroll
    for (int i = 0; i < kDctKtPerWave; ++i) {
      const int kt = wave + kDctWaves * i;
      if (kt < nkt) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int pix = pix0 + 16 * g + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = kt * 16 + out_row<T>(lk, r);
            if (k < L && pix < N) out[(size_t)k * N + pix] = acc[i][g][r];
          }
        }
      }
    }
    return;
  }

  // ---- v update; the adjoint input d1 v + d2 v_b replaces Z ----
  lds_barrier();  // every wave is done reading Z
  const T sg = T(dp->sigma);
  const T d1 = T(dct_coef(a.d1_sel[set], dp));
  const T d2 = T(dct_coef(a.d2_sel[set], dp));
  T* __restrict__ V = a.V[set];
  const T* __restrict__ Vb = a.Vb[set];
  // masks 1[|v~| <= 1] as bits of one 32-bit word per thread and block (bit
  // 4 (G i + g) + r), written by the primal role, read by the derivative
  // role (same launch shape)
  uint32_t* __restrict__ MW =
      a.mask[set] ? reinterpret_cast<uint32_t*>(a.mask[set]) + (size_t)blockIdx.x * blockDim.x +
                        threadIdx.x
                  : nullptr;
  const bool has_vb = Vb != nullptr;
  uint32_t mw = (a.role != ROLE_PRIMAL && MW) ? *MW : 0u;
  T al[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int pix = pix0 + 16 * g + lr;
    al[g] = a.alpha ? (pix < N ? T(a.alpha[pix]) : T(0)) : T(1);
  }
#pragma unroll
  for (int i = 0; i < kDctKtPerWave; ++i) {
    const int kt = wave + kDctWaves * i;
    if (kt < nkt) {
      // every operand of this k-tile in flight at once: clamped,
      // unconditional loads (values outside the cube are not used)
      T vold[G][4], vbv[G][4];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int pix = min(pix0 + 16 * g + lr, N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = min(kt * 16 + out_row<T>(lk, r), L - 1);
          const size_t idx = (size_t)k * N + pix;
          vold[g][r] = V[idx];
          if (has_vb) vbv[g][r] = Vb[idx];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int pix = pix0 + 16 * g + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = kt * 16 + out_row<T>(lk, r);
          T bv = T(0);
          if (k < L && pix < N) {
            const size_t idx = (size_t)k * N + pix;
            const T vt = vold[g][r] + sg * al[g] * acc[i][g][r];
            T vn;
            const uint32_t bit = 1u << (4 * (G * i + g) + r);
            if (a.role == ROLE_PRIMAL) {
              vn = vt < T(-1) ? T(-1) : (vt > T(1) ? T(1) : vt);
              if (vt >= T(-1) && vt <= T(1)) mw |= bit;
            } else {
              vn = (mw & bit) ? vt : T(0);
            }
            V[idx] = vn;
            bv = d1 * vn;
            if (has_vb) bv += d2 * vbv[g][r];
          }
          Z[k * PIX + 16 * g + lr] = bv;
        }
      }
    }
  }
  if (a.role == ROLE_PRIMAL && MW) *MW = mw;
  lds_barrier();

  // ---- product 2: t = alpha C^T b ----
#pragma unroll
  for (int i = 0; i < kDctKtPerWave; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[i][g] = acc_t{0, 0, 0, 0};
  for (int ks = 0; ks < nks; ++ks) {
    T b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) b[g] = Z[(4 * ks + lk) * PIX + 16 * g + lr];
#pragma unroll
    for (int i = 0; i < kDctKtPerWave; ++i) {
      const int lt = wave + kDctWaves * i;
      if (lt < nkt) {
        const T av = a.Cf2[((size_t)lt * nks + ks) * 64 + lane];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[i][g] = mfma16(av, b[g], acc[i][g]);
      }
    }
  }
  T* To = a.Tout[set];
#pragma unroll
  for (int i = 0; i < kDctKtPerWave; ++i) {
    const int lt = wave + kDctWaves * i;
    if (lt < nkt) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int pix = pix0 + 16 * g + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = lt * 16 + out_row<T>(lk, r);
          if (l < L && pix < N) To[(size_t)l * N + pix] = al[g] * acc[i][g][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 split form: every FP32 operand is x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi); a product is hi_a hi_b + lo_a hi_b + hi_a lo_b (the
// lo lo term, ~2^-18 relative, is dropped) on the 16x16x32 bf16 MFMA with
// FP32 accumulation.  Operand layout of that instruction (measured on
// gfx950): A[i][k] with i = lane % 16, k = 8 (lane / 16) + e for the lane's 8
// values e; B[k][j] with k = 8 (lane / 16) + e, j = lane % 16; result r is
// D[4 (lane / 16) + r][lane % 16].  The pixel tile is kept in LDS as
// [pixel][band] (bands contiguous) so a lane's 8 B-operand values are one
// 16-byte read.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

struct DctBfArgs {
  const float* z_a[kMaxSets];  // input z = c1 z_a + c2 z_b
  const float* z_b[kMaxSets];
  int c1_sel[kMaxSets], c2_sel[kMaxSets];
  float* V[kMaxSets];
  const float* Vb[kMaxSets];
  int d1_sel[kMaxSets], d2_sel[kMaxSets];
  float* Tout[kMaxSets];
  uint8_t* mask[kMaxSets];
  const bf16x8* Ah1;  // C hi,   [kt][ks][lane]
  const bf16x8* Al1;  // C lo
  const bf16x8* Ah2;  // C^T hi
  const bf16x8* Al2;  // C^T lo
  const double* alpha;
  const DevParams* dp;
  int L, Lp, N;
  int role, pure;
};

constexpr int kBfPix = 64;   // pixels per block (4 groups of 16)
constexpr int kBfG = 4;
// waves per block; each takes kDctMaxKt / kBfWaves of the 16-band output tiles
#ifndef MUFFIN_BF_WAVES
#define MUFFIN_BF_WAVES 8
#endif
constexpr int kBfWaves = MUFFIN_BF_WAVES;
constexpr int kBfKtPerWave = kDctMaxKt / kBfWaves;
static_assert(4 * 4 * kBfKtPerWave <= 32, "a thread's DCT mask bits fit one word");

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__global__ void __launch_bounds__(64 * kBfWaves, 2) dct_bf16_kernel(DctBfArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L, Lp = a.Lp, N = a.N;
  const int LpS = Lp + 8;  // padded band stride of the [pixel][band] tile
  __bf16* Zh = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* Zl = Zh + kBfPix * LpS;
  const int set = blockIdx.y;
  const int pix0 = blockIdx.x * kBfPix;
  const int nkt = Lp >> 4, nks = Lp >> 5;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const DevParams* dp = a.dp;
  {
    const double c1 = a.pure ? 1.0 : dct_coef(a.c1_sel[set], dp);
    const double c2 = a.pure ? 0.0 : dct_coef(a.c2_sel[set], dp);
    const float* za = a.z_a[set];
    const bool has_b = !a.pure && a.z_b[set] != nullptr;
    const float* zb = has_b ? a.z_b[set] : za;
    // each thread converts 8 consecutive bands of one pixel and stores them
    // as one 16-byte hi and one 16-byte lo vector; the operands of the 8
    // bands are loaded unconditionally (clamped indices) before any is used
    const int total = (Lp / 8) * kBfPix;
    for (int t = threadIdx.x; t < total; t += 64 * kBfWaves) {
      const int lg = t / kBfPix, j = t - lg * kBfPix;
      const int pix = pix0 + j;
      const int pc = min(pix, N - 1);
      float va[8], vb[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const size_t idx = (size_t)min(8 * lg + e, L - 1) * N + pc;
        va[e] = za[idx];
        if (has_b) vb[e] = zb[idx];
      }
      bf16x8 vh, vl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int l = 8 * lg + e;
        float z = 0.f;
        if (l < L && pix < N) {
          z = float(c1) * va[e];
          if (has_b) z += float(c2) * vb[e];
        }
        __bf16 h, lo;
        split_bf16(z, h, lo);
        vh[e] = h;
        vl[e] = lo;
      }
      *reinterpret_cast<bf16x8*>(Zh + j * LpS + 8 * lg) = vh;
      *reinterpret_cast<bf16x8*>(Zl + j * LpS + 8 * lg) = vl;
    }
  }
  lds_barrier();
  flt4 acc[kBfKtPerWave][kBfG];
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i)
#pragma unroll
    for (int g = 0; g < kBfG; ++g) acc[i][g] = flt4{0, 0, 0, 0};
  const bf16x8* Ah = a.pure == 2 ? a.Ah2 : a.Ah1;
  const bf16x8* Al = a.pure == 2 ? a.Al2 : a.Al1;
  for (int ks = 0; ks < nks; ++ks) {
    bf16x8 bh[kBfG], bl[kBfG];
#pragma unroll
    for (int g = 0; g < kBfG; ++g) {
      const int o = (16 * g + lr) * LpS + 32 * ks + 8 * lk;
      bh[g] = *reinterpret_cast<const bf16x8*>(Zh + o);
      bl[g] = *reinterpret_cast<const bf16x8*>(Zl + o);
    }
#pragma unroll
    for (int i = 0; i < kBfKtPerWave; ++i) {
      const int kt = wave + kBfWaves * i;
      if (kt < nkt) {
        const size_t f = ((size_t)kt * nks + ks) * 64 + lane;
        const bf16x8 ah = Ah[f], al = Al[f];
#pragma unroll
        for (int g = 0; g < kBfG; ++g) {
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[g], acc[i][g], 0, 0, 0);
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[g], acc[i][g], 0, 0, 0);
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[g], acc[i][g], 0, 0, 0);
        }
      }
    }
  }
  if (a.pure) {
    float* out = a.V[set];
#pragma unroll
    for (int i = 0; i < kBfKtPerWave; ++i) {
      const int kt = wave + kBfWaves * i;
      if (kt < nkt) {
#pragma unroll
        for (int g = 0; g < kBfG; ++g) {
          const int pix = pix0 + 16 * g + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = kt * 16 + 4 * lk + r;
            if (k < L && pix < N) out[(size_t)k * N + pix] = acc[i][g][r];
          }
        }
      }
    }
    return;
  }
  lds_barrier();
  const float sg = float(dp->sigma);
  const float d1 = float(dct_coef(a.d1_sel[set], dp));
  const float d2 = float(dct_coef(a.d2_sel[set], dp));
  float* __restrict__ V = a.V[set];
  const float* __restrict__ Vb = a.Vb[set];
  // mask bits as in dct_kernel: bit 4 (kBfG i + g) + r of the thread's word
  uint32_t* __restrict__ MW =
      a.mask[set] ? reinterpret_cast<uint32_t*>(a.mask[set]) + (size_t)blockIdx.x * blockDim.x +
                        threadIdx.x
                  : nullptr;
  const bool has_vb = Vb != nullptr;
  uint32_t mw = (a.role != ROLE_PRIMAL && MW) ? *MW : 0u;
  float al[kBfG];
#pragma unroll
  for (int g = 0; g < kBfG; ++g) {
    const int pix = pix0 + 16 * g + lr;
    al[g] = a.alpha ? (pix < N ? float(a.alpha[pix]) : 0.f) : 1.f;
  }
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i) {
    const int kt = wave + kBfWaves * i;
    if (kt < nkt) {
      // phase 1: every operand of this k-tile in flight at once
      float vold[kBfG][4], vbv[kBfG][4];
#pragma unroll
      for (int g = 0; g < kBfG; ++g) {
        const int pix = min(pix0 + 16 * g + lr, N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = min(kt * 16 + 4 * lk + r, L - 1);
          const size_t idx = (size_t)k * N + pix;
          vold[g][r] = V[idx];
          if (has_vb) vbv[g][r] = Vb[idx];
        }
      }
#pragma unroll
      for (int g = 0; g < kBfG; ++g) {
        const int pix = pix0 + 16 * g + lr;
        bf16x4 qh, ql;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = kt * 16 + 4 * lk + r;
          float bv = 0.f;
          if (k < L && pix < N) {
            const size_t idx = (size_t)k * N + pix;
            const float vt = vold[g][r] + sg * al[g] * acc[i][g][r];
            float vn;
            const uint32_t bit = 1u << (4 * (kBfG * i + g) + r);
            if (a.role == ROLE_PRIMAL) {
              vn = vt < -1.f ? -1.f : (vt > 1.f ? 1.f : vt);
              if (vt >= -1.f && vt <= 1.f) mw |= bit;
            } else {
              vn = (mw & bit) ? vt : 0.f;
            }
            V[idx] = vn;
            bv = d1 * vn;
            if (has_vb) bv += d2 * vbv[g][r];
          }
          __bf16 h, lo;
          split_bf16(bv, h, lo);
          qh[r] = h;
          ql[r] = lo;
        }
        // the 4 results of a lane are 4 consecutive bands of one pixel
        *reinterpret_cast<bf16x4*>(Zh + (16 * g + lr) * LpS + kt * 16 + 4 * lk) = qh;
        *reinterpret_cast<bf16x4*>(Zl + (16 * g + lr) * LpS + kt * 16 + 4 * lk) = ql;
      }
    }
  }
  if (a.role == ROLE_PRIMAL && MW) *MW = mw;
  lds_barrier();
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i)
#pragma unroll
    for (int g = 0; g < kBfG; ++g) acc[i][g] = flt4{0, 0, 0, 0};
  for (int ks = 0; ks < nks; ++ks) {
    bf16x8 bh[kBfG], bl[kBfG];
#pragma unroll
    for (int g = 0; g < kBfG; ++g) {
      const int o = (16 * g + lr) * LpS + 32 * ks + 8 * lk;
      bh[g] = *reinterpret_cast<const bf16x8*>(Zh + o);
      bl[g] = *reinterpret_cast<const bf16x8*>(Zl + o);
    }
#pragma unroll
    for (int i = 0; i < kBfKtPerWave; ++i) {
      const int lt = wave + kBfWaves * i;
      if (lt < nkt) {
        const size_t f = ((size_t)lt * nks + ks) * 64 + lane;
        const bf16x8 ah = a.Ah2[f], al2 = a.Al2[f];
#pragma unroll
        for (int g = 0; g < kBfG; ++g) {
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[g], acc[i][g], 0, 0, 0);
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al2, bh[g], acc[i][g], 0, 0, 0);
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[g], acc[i][g], 0, 0, 0);
        }
      }
    }
  }
  float* To = a.Tout[set];
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i) {
    const int lt = wave + kBfWaves * i;
    if (lt < nkt) {
#pragma unroll
      for (int g = 0; g < kBfG; ++g) {
        const int pix = pix0 + 16 * g + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = lt * 16 + 4 * lk + r;
          if (l < L && pix < N) To[(size_t)l * N + pix] = al[g] * acc[i][g][r];
        }
      }
    }
  }
}

size_t dct_mask_words(int N) {
  // blocks of 32 (FP64) or 64 pixels; 64 threads per wave
  const size_t threads = 64 * (size_t)std::max(kDctWaves, kBfWaves);
  return (size_t)((N + 31) / 32) * threads;
}

// host: round-to-nearest-even float -> bf16 bits
static uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
static float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

size_t dct_plan_bytes(int L, int kind, int elem_bytes) {
  const size_t Lp = kind == DCT_BF16X3 ? (L + 31) & ~31 : (L + 15) & ~15;
  size_t b = region_round((size_t)elem_bytes * 2 * Lp * Lp);
  if (kind == DCT_BF16X3) b += region_round(sizeof(uint16_t) * 4 * (Lp / 16) * (Lp / 32) * 64 * 8);
  return b;
}

template <typename T>
int dct_make_plan(DctPlan<T>& p, int L, int N, int kind, Region* r) {
  if (L < 1 || L > 16 * kDctMaxKt) return -2;
  p.L = L;
  p.N = N;
  p.Lp = kind == DCT_BF16X3 ? (L + 31) & ~31 : (L + 15) & ~15;
  p.kind = kind;
  const int Lp = p.Lp, nkt = Lp / 16, nks = Lp / 4;
  std::vector<long double> c((size_t)Lp * Lp, 0.0L);  // C[k][l], zero padded
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int k = 0; k < L; ++k) {
    const long double ck = k == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L);
    for (int l = 0; l < L; ++l) c[(size_t)k * Lp + l] = ck * cosl(pi * (2 * l + 1) * k / (2.0L * L));
  }
  // fragment order: lane = i + 16 k holds A[i][k] of tile (t, ks)
  std::vector<T> f1((size_t)Lp * Lp), f2((size_t)Lp * Lp);
  for (int t = 0; t < nkt; ++t)
    for (int ks = 0; ks < nks; ++ks)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane % 16, k = lane / 16;
        const size_t o = ((size_t)t * nks + ks) * 64 + lane;
        f1[o] = T(c[(size_t)(t * 16 + i) * Lp + ks * 4 + k]);   // C[row][col]
        f2[o] = T(c[(size_t)(ks * 4 + k) * Lp + t * 16 + i]);   // C^T[row][col]
      }
  p.borrowed = r != nullptr;
  p.C = static_cast<T*>(region_alloc(r, sizeof(T) * 2 * f1.size()));
  if (!p.C) return -3; /* E_NOMEM */
  MUFFIN_HIP_CHECK(hipMemcpy(p.C, f1.data(), sizeof(T) * f1.size(), hipMemcpyHostToDevice));
  MUFFIN_HIP_CHECK(hipMemcpy(p.C + f1.size(), f2.data(), sizeof(T) * f2.size(),
                             hipMemcpyHostToDevice));
  if (kind == DCT_BF16X3) {
    // bf16 hi/lo fragments for the 16x16x32 instruction: [t][ks32][lane][8]
    const int nk32 = Lp / 32;
    const size_t cnt = (size_t)nkt * nk32 * 64 * 8;
    std::vector<uint16_t> h((size_t)4 * cnt);
    for (int t = 0; t < nkt; ++t)
      for (int ks = 0; ks < nk32; ++ks)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < 8; ++e) {
            const int i = lane % 16, k = 8 * (lane / 16) + e;
            const size_t o = (((size_t)t * nk32 + ks) * 64 + lane) * 8 + e;
            const long double v1 = c[(size_t)(t * 16 + i) * Lp + ks * 32 + k];
            const long double v2 = c[(size_t)(ks * 32 + k) * Lp + t * 16 + i];
            const uint16_t h1 = bf16_bits((float)v1), h2 = bf16_bits((float)v2);
            h[o] = h1;
            h[cnt + o] = bf16_bits((float)(v1 - (long double)bf16_value(h1)));
            h[2 * cnt + o] = h2;
            h[3 * cnt + o] = bf16_bits((float)(v2 - (long double)bf16_value(h2)));
          }
    p.Chi = static_cast<uint16_t*>(region_alloc(r, sizeof(uint16_t) * h.size()));
    if (!p.Chi) return -3; /* E_NOMEM */
    MUFFIN_HIP_CHECK(hipMemcpy(p.Chi, h.data(), sizeof(uint16_t) * h.size(), hipMemcpyHostToDevice));
    p.Clo = p.Chi + cnt;
  }
  return 0;
}

template <typename T>
void dct_free_plan(DctPlan<T>& p) {
  if (p.C && !p.borrowed) (void)hipFree(p.C);
  if (p.Chi && !p.borrowed) (void)hipFree(p.Chi);
  p.C = nullptr;
  p.Chi = p.Clo = nullptr;
}

static int dct_update_bf16(const DctPlan<float>& p, const DctIO<float>& io, const DevParams* dp,
                           hipStream_t s) {
  DctBfArgs a{};
  for (int i = 0; i < io.nsets; ++i) {
    a.z_a[i] = io.z_a[i];
    a.z_b[i] = io.z_b[i];
    a.c1_sel[i] = io.c1_sel[i];
    a.c2_sel[i] = io.c2_sel[i];
    a.V[i] = io.V[i];
    a.Vb[i] = io.Vb[i];
    a.d1_sel[i] = io.d1_sel[i];
    a.d2_sel[i] = io.d2_sel[i];
    a.Tout[i] = io.Tout[i];
    a.mask[i] = io.mask[i];
  }
  const int nkt = p.Lp / 16, nk32 = p.Lp / 32;
  const size_t cnt = (size_t)nkt * nk32 * 64;  // bf16x8 per table
  const bf16x8* base = reinterpret_cast<const bf16x8*>(p.Chi);
  a.Ah1 = base;
  a.Al1 = base + cnt;
  a.Ah2 = base + 2 * cnt;
  a.Al2 = base + 3 * cnt;
  a.alpha = io.alpha;
  a.dp = dp;
  a.L = p.L;
  a.Lp = p.Lp;
  a.N = p.N;
  a.role = io.role;
  a.pure = io.pure;
  const size_t shm = 2 * sizeof(__bf16) * (size_t)kBfPix * (p.Lp + 8);
  dim3 grid((p.N + kBfPix - 1) / kBfPix, io.nsets);
  MUFFIN_ALLOW_BIG_LDS(dct_bf16_kernel);
  dct_bf16_kernel<<<grid, 64 * kBfWaves, shm, s>>>(a);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template <typename T>
int dct_update(const DctPlan<T>& p, const DctIO<T>& io, const DevParams* dp, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (p.kind == DCT_BF16X3) return dct_update_bf16(p, io, dp, s);
  }
  DctArgs<T> a{};
  for (int i = 0; i < io.nsets; ++i) {
    a.z_a[i] = io.z_a[i];
    a.z_b[i] = io.z_b[i];
    a.c1_sel[i] = io.c1_sel[i];
    a.c2_sel[i] = io.c2_sel[i];
    a.V[i] = io.V[i];
    a.Vb[i] = io.Vb[i];
    a.d1_sel[i] = io.d1_sel[i];
    a.d2_sel[i] = io.d2_sel[i];
    a.Tout[i] = io.Tout[i];
    a.mask[i] = io.mask[i];
  }
  a.Cf1 = p.C;
  a.Cf2 = p.C + (size_t)p.Lp * p.Lp;
  a.alpha = io.alpha;
  a.dp = dp;
  a.L = p.L;
  a.Lp = p.Lp;
  a.N = p.N;
  a.role = io.role;
  a.pure = io.pure;
  constexpr int PIX = 16 * dct_groups<T>();
  const size_t shm = sizeof(T) * (size_t)p.Lp * PIX;
  dim3 grid((p.N + PIX - 1) / PIX, io.nsets);
  MUFFIN_ALLOW_BIG_LDS(dct_kernel<T>);
  dct_kernel<T><<<grid, 64 * kDctWaves, shm, s>>>(a);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template int dct_make_plan<double>(DctPlan<double>&, int, int, int, Region*);
template int dct_make_plan<float>(DctPlan<float>&, int, int, int, Region*);
template void dct_free_plan<double>(DctPlan<double>&);
template void dct_free_plan<float>(DctPlan<float>&);
template int dct_update<double>(const DctPlan<double>&, const DctIO<double>&,
                                const DevParams*, hipStream_t);
template int dct_update<float>(const DctPlan<float>&, const DctIO<float>&,
                               const DevParams*, hipStream_t);

}  // namespace muffin
