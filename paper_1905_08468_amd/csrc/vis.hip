// Visibility-domain direct operator (Section 1: the same algorithm with the
// visibilities as data, only the direct operator changes).  Band l samples
// the sky's Fourier transform at K continuous positions (u_k, v_k), in
// cycles across the image, phases referred to the image centre c = n / 2:
//   (H x)_k = sum_{i,j} x[i, j] exp(-2 pi i (u_k (i - c) + v_k (j - c)) / n).
// For a real cube the gradient of 1/2 |v - H x|^2 is Re H^* H x - Re H^* v,
// and Re H^* H is the windowed linear convolution by the real point spread
// function psf[n + a][n + b] = sum_k cos(2 pi (u_k a + v_k b) / n): the
// iteration then runs on the image-domain machinery with that PSF, the
// back-projected ("dirty") cube Re H^* v and the back-projected probe.
//
// Kernels (FP64 arithmetic, exact sums, O(K) per output):
//   back-projection  out[l][i][j] = Re sum_k w_k e^{+2 pi i (u_k (i-o) + v_k (j-o)) / n}
//                    on an m x m grid with origin o (the dirty and probe cubes:
//                    m = n, o = n/2; the PSF: m = 2n, o = n, w = 1).  A block
//                    owns a 16 x 16 tile; per chunk of 64 samples it computes
//                    the tile's 16 row and 16 column phase factors of each
//                    sample once (separability), then every output costs one
//                    complex product per sample.
//   degridding       the forward sums, one block per 64 samples, the image
//                    streamed row by row through LDS, the column phases by
//                    a rotation recurrence along each row.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "muffin.h"
#include "internal.hpp"

namespace muffin {
namespace {

constexpr int kVT = 16;      // tile side (outputs)
constexpr int kVChunk = 64;  // samples per LDS chunk
constexpr int kVNT = 256;

// e^{+2 pi i u a / n} with the argument reduced to [-1/2, 1/2] turns first
__device__ __forceinline__ double2 phase(double u, double a, double inv_n) {
  double t = u * a * inv_n;
  t -= rint(t);
  double s, c;
  sincospi(2.0 * t, &s, &c);
  return make_double2(c, s);
}

template <typename T>
__global__ void __launch_bounds__(kVNT) backproject_kernel(const double* __restrict__ uv,
                                                           const double* __restrict__ w, int K,
                                                           int n, int m, int o, T* __restrict__ out) {
  __shared__ double2 er[kVChunk][kVT];
  __shared__ double2 ec[kVChunk][kVT];
  __shared__ double2 ws[kVChunk];
  const int band = blockIdx.y;
  const int tiles = (m + kVT - 1) / kVT;
  const int i0 = (blockIdx.x / tiles) * kVT, j0 = (blockIdx.x % tiles) * kVT;
  const int ti = threadIdx.x / kVT, tj = threadIdx.x % kVT;
  const double inv_n = 1.0 / n;
  const double* ub = uv + (size_t)band * K * 2;
  const double* wb = w ? w + (size_t)band * K * 2 : nullptr;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += kVChunk) {
    const int kc = min(kVChunk, K - k0);
    for (int t = threadIdx.x; t < 2 * kVChunk * kVT; t += kVNT) {
      const int which = t / (kVChunk * kVT), rem = t - which * (kVChunk * kVT);
      const int k = rem / kVT, q = rem - k * kVT;
      double2 f = make_double2(0.0, 0.0);
      if (k < kc) {
        const double u = ub[2 * (k0 + k) + which];
        f = phase(u, double((which ? j0 : i0) + q - o), inv_n);
      }
      if (which) ec[k][q] = f;
      else er[k][q] = f;
    }
    for (int k = threadIdx.x; k < kVChunk; k += kVNT)
      ws[k] = k < kc ? (wb ? make_double2(wb[2 * (k0 + k)], wb[2 * (k0 + k) + 1])
                           : make_double2(1.0, 0.0))
                     : make_double2(0.0, 0.0);
    lds_barrier();
    for (int k = 0; k < kc; ++k) {
      const double2 r = er[k][ti], c = ec[k][tj], wk = ws[k];
      const double zr = r.x * c.x - r.y * c.y, zi = r.x * c.y + r.y * c.x;
      acc = fma(wk.x, zr, acc);
      acc = fma(-wk.y, zi, acc);
    }
    lds_barrier();
  }
  const int i = i0 + ti, j = j0 + tj;
  if (i < m && j < m) out[((size_t)band * m + i) * m + j] = T(acc);
}

template <typename T>
__global__ void __launch_bounds__(kVNT) degrid_kernel(const double* __restrict__ uv,
                                                      const T* __restrict__ x, int K, int n,
                                                      double* __restrict__ vis) {
  constexpr int RG = kVNT / kVChunk;  // row groups
  extern __shared__ __align__(16) unsigned char vis_smem[];
  double2(*red)[kVChunk] = reinterpret_cast<double2(*)[kVChunk]>(vis_smem);
  double* xs0 = reinterpret_cast<double*>(vis_smem + sizeof(double2) * RG * kVChunk);
  auto xs = [&](int r, int j) -> double& { return xs0[r * n + j]; };
  const int band = blockIdx.y;
  const int k = blockIdx.x * kVChunk + threadIdx.x % kVChunk;
  const int g = threadIdx.x / kVChunk;
  const bool on = k < K;
  const double* ub = uv + ((size_t)band * K + (on ? k : 0)) * 2;
  const double u = ub[0], v = ub[1];
  const double inv_n = 1.0 / n, c = n / 2.0;
  const T* xb = x + (size_t)band * n * n;
  // e^{-2 pi i v (j - c) / n}: start and step of the column recurrence
  const double2 s0 = phase(-v, -c, inv_n), st = phase(-v, 1.0, inv_n);
  double re = 0.0, im = 0.0;
  for (int i0 = 0; i0 < n; i0 += RG) {
    for (int t = threadIdx.x; t < RG * n; t += kVNT) {
      const int r = t / n, j = t - r * n;
      xs(r, j) = i0 + r < n ? double(xb[(size_t)(i0 + r) * n + j]) : 0.0;
    }
    lds_barrier();
    const int i = i0 + g;
    if (i < n) {
      double sr = 0.0, si = 0.0, cr = s0.x, ci = s0.y;
      for (int j = 0; j < n; ++j) {
        const double xv = xs(g, j);
        sr = fma(xv, cr, sr);
        si = fma(xv, ci, si);
        const double nr = cr * st.x - ci * st.y;
        ci = cr * st.y + ci * st.x;
        cr = nr;
      }
      const double2 rp = phase(-u, double(i) - c, inv_n);
      re += rp.x * sr - rp.y * si;
      im += rp.x * si + rp.y * sr;
    }
    lds_barrier();
  }
  red[g][threadIdx.x % kVChunk] = make_double2(re, im);
  lds_barrier();
  if (g == 0 && on) {
    double2 s = red[0][threadIdx.x];
    for (int q = 1; q < RG; ++q) {
      s.x += red[q][threadIdx.x].x;
      s.y += red[q][threadIdx.x].y;
    }
    vis[((size_t)band * K + k) * 2] = s.x;
    vis[((size_t)band * K + k) * 2 + 1] = s.y;
  }
}

__global__ void __launch_bounds__(1024) sumsq_kernel(const double* a, size_t count, double* out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < count; i += 1024) acc = fma(a[i], a[i], acc);
  sh[threadIdx.x] = acc;
  lds_barrier();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    lds_barrier();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

template <typename T>
int backproject(const double* uv, const double* w, int L, int K, int n, int m, int o, T* out,
                hipStream_t s) {
  const int tiles = (m + kVT - 1) / kVT;
  backproject_kernel<T><<<dim3(tiles * tiles, L), kVNT, 0, s>>>(uv, w, K, n, m, o, out);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace
}  // namespace muffin

using namespace muffin;

extern "C" {

int muffin_vis_prepare(const double* uv, const double* vis, const double* delta, int32_t L,
                       int32_t K, int32_t n, int32_t mode, void* dirty_out, void* psf_out,
                       void* delta_out, double* vis_norm2, void* stream) {
  if (!uv || !vis || !dirty_out || !psf_out || L < 1 || K < 1 || n < 8 || n > 2048)
    return MUFFIN_E_INVAL;
  if ((delta == nullptr) != (delta_out == nullptr)) return MUFFIN_E_INVAL;
  if (mode != MUFFIN_F64 && mode != MUFFIN_F32 && mode != MUFFIN_F32_BF16DCT)
    return MUFFIN_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int c = n / 2;
  auto run = [&](auto* dirty, auto* psf, auto* dout) -> int {
    int rc = backproject(uv, vis, L, K, n, n, c, dirty, s);
    if (!rc) rc = backproject(uv, (const double*)nullptr, L, K, n, 2 * n, n, psf, s);
    if (!rc && delta) rc = backproject(uv, delta, L, K, n, n, c, dout, s);
    return rc;
  };
  int rc = mode == MUFFIN_F64
               ? run(static_cast<double*>(dirty_out), static_cast<double*>(psf_out),
                     static_cast<double*>(delta_out))
               : run(static_cast<float*>(dirty_out), static_cast<float*>(psf_out),
                     static_cast<float*>(delta_out));
  if (rc) return rc;
  if (vis_norm2) {
    double* d = nullptr;
    MUFFIN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&d), sizeof(double), s));
    sumsq_kernel<<<1, 1024, 0, s>>>(vis, (size_t)L * K * 2, d);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipMemcpyAsync(vis_norm2, d, sizeof(double), hipMemcpyDeviceToHost, s);
    const hipError_t e3 = hipStreamSynchronize(s);
    (void)hipFreeAsync(d, s);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return MUFFIN_E_HIP;
  }
  return MUFFIN_OK;
}

int muffin_vis_degrid(const double* uv, int32_t L, int32_t K, int32_t n, int32_t mode,
                      const void* x, double* vis_out, void* stream) {
  if (!uv || !x || !vis_out || L < 1 || K < 1 || n < 8 || n > 2048) return MUFFIN_E_INVAL;
  if (mode != MUFFIN_F64 && mode != MUFFIN_F32 && mode != MUFFIN_F32_BF16DCT)
    return MUFFIN_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid((K + kVChunk - 1) / kVChunk, L);
  const size_t shm = sizeof(double2) * (kVNT / kVChunk) * kVChunk +
                     sizeof(double) * (kVNT / kVChunk) * (size_t)n;
  if (mode == MUFFIN_F64) {
    MUFFIN_ALLOW_BIG_LDS((degrid_kernel<double>));
    degrid_kernel<double><<<grid, kVNT, shm, s>>>(uv, static_cast<const double*>(x), K, n, vis_out);
  } else {
    MUFFIN_ALLOW_BIG_LDS((degrid_kernel<float>));
    degrid_kernel<float><<<grid, kVNT, shm, s>>>(uv, static_cast<const float*>(x), K, n, vis_out);
  }
  MUFFIN_HIP_CHECK(hipGetLastError());
  return MUFFIN_OK;
}

}  // extern "C"
