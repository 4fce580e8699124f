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
#include <type_traits>
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

// One product of a block: acc[i][g] += A(tile wave + kDctWaves i) B(g),
// summed over the nks k-steps of 4 bands, B from the LDS tile Z ([band][pixel]).
// The A fragments (one value per lane, from the fragment-ordered table in
// global memory) are fetched kDctAhead k-steps before their use, in two
// alternating register buffers, so the table's L2 latency overlaps the
// MFMAs of the previous k-steps instead of stalling every k-step.
constexpr int kDctAhead = 4;
template <typename T, int G, typename Acc>
__device__ __forceinline__ void dct_product(Acc (&acc)[kDctKtPerWave][G], const T* __restrict__ A,
                                            const T* Z, int nkt, int nks, int wave, int lane,
                                            int lr, int lk) {
  constexpr int PIX = 16 * G;
  auto fetch = [&](T (&av)[kDctAhead][kDctKtPerWave], int ks0) {
#pragma unroll
    for (int d = 0; d < kDctAhead; ++d) {
      const int ks = min(ks0 + d, nks - 1);  // clamped: the tail re-reads the last step
#pragma unroll
      for (int i = 0; i < kDctKtPerWave; ++i) {
        const int kt = min(wave + kDctWaves * i, nkt - 1);
        av[d][i] = A[((size_t)kt * nks + ks) * 64 + lane];
      }
    }
  };
  auto use = [&](const T (&av)[kDctAhead][kDctKtPerWave], int ks0) {
#pragma unroll
    for (int d = 0; d < kDctAhead; ++d) {
      const int ks = ks0 + d;
      if (ks < nks) {
        T b[G];
#pragma unroll
        for (int g = 0; g < G; ++g) b[g] = Z[(4 * ks + lk) * PIX + 16 * g + lr];
#pragma unroll
        for (int i = 0; i < kDctKtPerWave; ++i) {
          if (wave + kDctWaves * i < nkt) {
#pragma unroll
            for (int g = 0; g < G; ++g) acc[i][g] = mfma16(av[d][i], b[g], acc[i][g]);
          }
        }
      }
    }
  };
  T a0[kDctAhead][kDctKtPerWave], a1[kDctAhead][kDctKtPerWave];
  fetch(a0, 0);
  for (int ks0 = 0; ks0 < nks; ks0 += 2 * kDctAhead) {
    fetch(a1, ks0 + kDctAhead);
    use(a0, ks0);
    if (ks0 + kDctAhead < nks) {
      fetch(a0, ks0 + 2 * kDctAhead);
      use(a1, ks0 + kDctAhead);
    }
  }
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
    constexpr int U = 16;
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

  // the pixels' weights alpha_n and (derivative role) the mask word are
  // fetched before the first product, which hides their latency.  Masks
  // 1[|v~| <= 1] are bits of one 32-bit word per thread and block (bit
  // 4 (G i + g) + r), written by the primal role, read by the derivative
  // role (same launch shape).  Lanes past the last pixel read a clamped
  // weight and store nothing.
  T al[G];
  uint32_t* __restrict__ MW =
      (!a.pure && a.mask[set]) ? reinterpret_cast<uint32_t*>(a.mask[set]) +
                                     (size_t)blockIdx.x * blockDim.x + threadIdx.x
                               : nullptr;
  uint32_t mw = (a.role != ROLE_PRIMAL && MW) ? *MW : 0u;
#pragma unroll
  for (int g = 0; g < G; ++g) al[g] = a.alpha ? T(a.alpha[min(pix0 + 16 * g + lr, N - 1)]) : T(1);

  acc_t acc[kDctKtPerWave][G];
#pragma unroll
  for (int i = 0; i < kDctKtPerWave; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[i][g] = acc_t{0, 0, 0, 0};

  // ---- product 1: C Z (pure == 2: C^T Z) ----
  dct_product<T, G>(acc, a.pure == 2 ? a.Cf2 : a.Cf1, Z, nkt, nks, wave, lane, lr, lk);

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
  const bool has_vb = Vb != nullptr;
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
  dct_product<T, G>(acc, a.Cf2, Z, nkt, nks, wave, lane, lr, lk);
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

// One product of a block in the split form: acc[i][g] += A(tile wave +
// kBfWaves i) B(g) over the nks k-steps of 32 bands, each as the three bf16
// products hi hi + lo hi + hi lo.  The A fragments (hi and lo, one 16-byte
// vector each per lane) are fetched one k-step ahead of their use, in two
// alternating register buffers, so their L2 latency overlaps the MFMAs of
// the step before; B comes from the LDS tile ([pixel][band], row pitch LpS).
__device__ __forceinline__ void bf_product(flt4 (&acc)[kBfKtPerWave][kBfG],
                                           const bf16x8* __restrict__ Ah,
                                           const bf16x8* __restrict__ Al, const __bf16* Zh,
                                           const __bf16* Zl, int LpS, int nkt, int nks, int wave,
                                           int lane, int lr, int lk) {
  auto fetch = [&](bf16x8 (&h)[kBfKtPerWave], bf16x8 (&l)[kBfKtPerWave], int ks) {
    ks = min(ks, nks - 1);  // clamped: the tail re-reads the last step
#pragma unroll
    for (int i = 0; i < kBfKtPerWave; ++i) {
      const int kt = min(wave + kBfWaves * i, nkt - 1);
      const size_t f = ((size_t)kt * nks + ks) * 64 + lane;
      h[i] = Ah[f];
      l[i] = Al[f];
    }
  };
  auto use = [&](const bf16x8 (&h)[kBfKtPerWave], const bf16x8 (&l)[kBfKtPerWave], int ks) {
    bf16x8 bh[kBfG], bl[kBfG];
#pragma unroll
    for (int g = 0; g < kBfG; ++g) {
      const int o = (16 * g + lr) * LpS + 32 * ks + 8 * lk;
      bh[g] = *reinterpret_cast<const bf16x8*>(Zh + o);
      bl[g] = *reinterpret_cast<const bf16x8*>(Zl + o);
    }
#pragma unroll
    for (int i = 0; i < kBfKtPerWave; ++i) {
      if (wave + kBfWaves * i < nkt) {
#pragma unroll
        for (int g = 0; g < kBfG; ++g) {
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h[i], bh[g], acc[i][g], 0, 0, 0);
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l[i], bh[g], acc[i][g], 0, 0, 0);
          acc[i][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h[i], bl[g], acc[i][g], 0, 0, 0);
        }
      }
    }
  };
  bf16x8 h0[kBfKtPerWave], l0[kBfKtPerWave], h1[kBfKtPerWave], l1[kBfKtPerWave];
  fetch(h0, l0, 0);
  for (int ks = 0; ks < nks; ks += 2) {
    fetch(h1, l1, ks + 1);
    use(h0, l0, ks);
    if (ks + 1 < nks) {
      fetch(h0, l0, ks + 2);
      use(h1, l1, ks + 1);
    }
  }
}

__global__ void __launch_bounds__(64 * kBfWaves, 4) dct_bf16_kernel(DctBfArgs a) {
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
    // each thread converts 8 consecutive bands of one pixel per item and
    // stores them as one 16-byte hi and one 16-byte lo vector; the operands
    // of all the thread's items (at most kBfItems) are loaded unconditionally
    // (clamped indices) before any is used, so the whole tile is in flight
    // at once
    constexpr int NT = 64 * kBfWaves;
    constexpr int kBfItems = (256 / 8) * kBfPix / NT;
    const int total = (Lp / 8) * kBfPix;
    auto stage = [&](auto two) {
      constexpr bool B = decltype(two)::value;
      float va[kBfItems][8], vb[B ? kBfItems : 1][8];
#pragma unroll
      for (int it = 0; it < kBfItems; ++it) {
        const int t = min((int)threadIdx.x + it * NT, total - 1);
        const int lg = t / kBfPix, j = t - lg * kBfPix;
        const int pc = min(pix0 + j, N - 1);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const size_t idx = (size_t)min(8 * lg + e, L - 1) * N + pc;
          va[it][e] = za[idx];
          if constexpr (B) vb[it][e] = zb[idx];
        }
      }
#pragma unroll
      for (int it = 0; it < kBfItems; ++it) {
        const int t = threadIdx.x + it * NT;
        if (t < total) {
          const int lg = t / kBfPix, j = t - lg * kBfPix;
          const int pix = pix0 + j;
          bf16x8 vh, vl;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int l = 8 * lg + e;
            float z = 0.f;
            if (l < L && pix < N) {
              z = float(c1) * va[it][e];
              if constexpr (B) z += float(c2) * vb[it][e];
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
    };
    if (has_b)
      stage(std::true_type{});
    else
      stage(std::false_type{});
  }
  lds_barrier();
  // the pixels' weights alpha_n and (derivative role) the mask word are
  // fetched before the first product, which hides their latency; mask bits
  // as in dct_kernel: bit 4 (kBfG i + g) + r of the thread's word.  Lanes
  // past the last pixel read a clamped weight and store nothing.
  float al[kBfG];
  uint32_t* __restrict__ MW =
      (!a.pure && a.mask[set]) ? reinterpret_cast<uint32_t*>(a.mask[set]) +
                                     (size_t)blockIdx.x * blockDim.x + threadIdx.x
                               : nullptr;
  uint32_t mw = (a.role != ROLE_PRIMAL && MW) ? *MW : 0u;
#pragma unroll
  for (int g = 0; g < kBfG; ++g)
    al[g] = a.alpha ? float(a.alpha[min(pix0 + 16 * g + lr, N - 1)]) : 1.f;
  flt4 acc[kBfKtPerWave][kBfG];
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i)
#pragma unroll
    for (int g = 0; g < kBfG; ++g) acc[i][g] = flt4{0, 0, 0, 0};
  bf_product(acc, a.pure == 2 ? a.Ah2 : a.Ah1, a.pure == 2 ? a.Al2 : a.Al1, Zh, Zl, LpS, nkt, nks,
             wave, lane, lr, lk);
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
  const bool has_vb = Vb != nullptr;
  // phase 1: the operands of both of the wave's k-tiles in flight at once
  // (clamped, unconditional loads; values outside the cube are not used);
  // the second term v_b of the adjoint's input, when there is one, is
  // fetched per k-tile (one tile ahead) to stay within 128 registers
  float vold[kBfKtPerWave][kBfG][4], vbv[kBfG][4];
  auto load_vb = [&](int i) {
    const int kt = min(wave + kBfWaves * i, nkt - 1);
#pragma unroll
    for (int g = 0; g < kBfG; ++g) {
      const int pix = min(pix0 + 16 * g + lr, N - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = min(kt * 16 + 4 * lk + r, L - 1);
        vbv[g][r] = Vb[(size_t)k * N + pix];
      }
    }
  };
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i) {
    const int kt = min(wave + kBfWaves * i, nkt - 1);
#pragma unroll
    for (int g = 0; g < kBfG; ++g) {
      const int pix = min(pix0 + 16 * g + lr, N - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = min(kt * 16 + 4 * lk + r, L - 1);
        vold[i][g][r] = V[(size_t)k * N + pix];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kBfKtPerWave; ++i) {
    const int kt = wave + kBfWaves * i;
    if (has_vb) load_vb(i);
    if (kt < nkt) {
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
            const float vt = vold[i][g][r] + sg * al[g] * acc[i][g][r];
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
  bf_product(acc, a.Ah2, a.Al2, Zh, Zl, LpS, nkt, nks, wave, lane, lr, lk);
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
