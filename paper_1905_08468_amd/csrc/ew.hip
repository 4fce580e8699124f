// Element-wise and reduction kernels of the MUFFIN iteration:
//  * primal step with positivity (eqs. `stpm`, `stpx`) and its weak
//    derivative (Algorithms 3-4: x~' = U(m) m'), all sets of one trajectory
//    in one thread so the derivative mask never leaves registers;
//  * deterministic FP64 dot products (fixed block partials + one ordered
//    final sum) for PSURE-FDMC (eq. `PSURE0`) and SUGAR-FDMC (eq. `SUGAR`);
//  * the ADA-PT parameter update (eq. `adaptgrad`) and the step-size rule of
//    Section 2.2, as one-thread kernels on device-resident scalars;
//  * weights alpha_n, beta_l of Section 2.1 (norms of the initial estimate;
//    both dictionaries preserve norms, so ||W x|| = ||x||);
//  * power-iteration helpers for the Lipschitz constant (FP64).
#include "internal.hpp"

namespace muffin {

constexpr int kEwNT = 256;
constexpr int kDotBlocks = 1024;

template <int NT>
__device__ double block_sum_all(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s += sh[i];
  return s;  // thread 0
}

// ------------------------------------------------------------ primal step --
template <typename T>
__global__ void __launch_bounds__(kEwNT) primal_kernel(PrimalIO<T> io, size_t count,
                                                       const DevParams* dp) {
  const int tr = blockIdx.y;
  const T tau = T(dp->tau);
  const T mu = T(dp->mu);
  const T* __restrict__ x0 = io.x[tr][0];
  const T* __restrict__ g0 = io.g[tr][0];
  const T* __restrict__ hy = io.hty[tr];
  const T* __restrict__ s0 = io.s[tr][0];
  const T* __restrict__ t0 = io.t[tr][0];
  T* __restrict__ o0 = io.xt[tr][0];
  T* __restrict__ z0 = io.z[tr][0];
  const int nd = io.nderiv;
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT) {
    // all loads of this element first (primal and both derivative sets)
    T xd[2], gd[2], sd[2], td[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (d < nd) {
        xd[d] = io.x[tr][d + 1][i];
        gd[d] = io.g[tr][d + 1][i];
        sd[d] = io.s[tr][d + 1][i];
        td[d] = io.t[tr][d + 1][i];
      }
    }
    // s arrays hold beta_l / sqrt(P) W_s^T u of their own set; the spatial
    // term of the primal update is mu s, and its mu-derivative
    // s + mu s' (the primal's s is in registers already)
    const T sp = s0[i];
    const T xp = x0[i];
    const T m = xp - tau * ((g0[i] - hy[i]) + mu * sp + t0[i]);
    const bool pos = m > T(0);
    const T op = pos ? m : T(0);
    o0[i] = op;
    z0[i] = T(2) * op - xp;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (d < nd) {
        T sterm = mu * sd[d];
        if (d == 0) sterm += sp;  // d/dmu set
        const T md = xd[d] - tau * (gd[d] + sterm + td[d]);
        const T od = pos ? md : T(0);
        io.xt[tr][d + 1][i] = od;
        io.z[tr][d + 1][i] = T(2) * od - xd[d];
      }
    }
  }
}

template <typename T>
int primal_step(const PrimalIO<T>& io, size_t count, const DevParams* dp, hipStream_t s) {
  const size_t need = (count + kEwNT - 1) / kEwNT;
  const int bx = (int)std::min<size_t>(need, 8192);
  primal_kernel<T><<<dim3(bx, io.ntraj), kEwNT, 0, s>>>(io, count, dp);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------- dots ----
template <typename T>
__global__ void __launch_bounds__(kEwNT) dot_kernel(const T* a, const T* b, const T* c,
                                                    size_t count, double* partials) {
  __shared__ double sh[kEwNT / 64];
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT) {
    double v = double(a[i]);
    if (b) v -= double(b[i]);
    acc += v * double(c[i]);
  }
  const double s = block_sum_all<kEwNT>(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int dot_blocks() { return kDotBlocks; }

template <typename T>
int dot_partials(const T* a, const T* b, const T* c, size_t count, double* partials,
                 int nblocks, hipStream_t s) {
  dot_kernel<T><<<nblocks, kEwNT, 0, s>>>(a, b, c, count, partials);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ void __launch_bounds__(kEwNT) reduce_kernel(const double* partials, int count,
                                                       double* out) {
  __shared__ double sh[kEwNT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += kEwNT) acc += partials[i];
  const double s = block_sum_all<kEwNT>(acc, sh);
  if (threadIdx.x == 0) *out = s;
}

int reduce_to_slot(const double* partials, int count, DevParams* dp, int slot, hipStream_t s) {
  reduce_kernel<<<1, kEwNT, 0, s>>>(partials, count, dp->sums + slot);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

int reduce_to_buffer(const double* partials, int count, double* out, hipStream_t s) {
  reduce_kernel<<<1, kEwNT, 0, s>>>(partials, count, out);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------- theta and tau ----
__device__ void tau_from_rule(DevParams* dp) {
  if (dp->tau_rule < 0) return;  // fixed step
  const double mu2 = dp->mu * dp->mu, ga2 = dp->gamma * dp->gamma;
  const double k = dp->tau_rule == 0
                       ? dp->ws_norm2 * mu2 * dp->max_beta2 + ga2 * dp->max_alpha2
                       : dp->ws_norm2 * mu2 * dp->sum_beta2 + ga2 * dp->sum_alpha2;
  dp->tau = dp->rho / (0.5 * dp->beta_H + dp->sigma * k);
}

// The history row and its iteration number follow from the device's update
// counter (updates happen after every `period` iterations), so the kernel
// can be replayed from a captured graph.
__global__ void theta_kernel(DevParams* dp, double* hist, int max_hist, int period,
                             int apply) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int q = dp->n_updates;  // this update's index
  double* hist_row = (hist && q < max_hist) ? hist + (size_t)q * kHistCols : nullptr;
  const long long k = (long long)(q + 1) * period;
  const double c = 2.0 * dp->sigma_w * dp->sigma_w / dp->eps_fd;
  const double s_mu = 2.0 * dp->sums[SLOT_GX_MU] + c * dp->sums[SLOT_FD_MU];
  const double s_ga = 2.0 * dp->sums[SLOT_GX_GA] + c * dp->sums[SLOT_FD_GA];
  // ||Y - H X||^2: from the FFT chain (dirty images), or for visibilities
  // |v|^2 + <X, psf * X - 2 Re H^* v> (two dot products)
  const double res2 = dp->vis ? dp->res_const + dp->sums[SLOT_RES2] - dp->sums[SLOT_AUX0]
                              : dp->sums[SLOT_RES2];
  const double psure = res2 - dp->n_meas * dp->sigma_w * dp->sigma_w + c * dp->sums[SLOT_FD_X];
  if (apply) {
    const double mu = dp->mu - dp->eta_mu * s_mu;
    const double ga = dp->gamma - dp->eta_gamma * s_ga;
    dp->mu = mu > 0.0 ? mu : 0.0;
    dp->gamma = ga > 0.0 ? ga : 0.0;
    tau_from_rule(dp);
    dp->n_updates += 1;
  }
  if (hist_row) {
    hist_row[0] = double(k);
    hist_row[1] = dp->mu;
    hist_row[2] = dp->gamma;
    hist_row[3] = dp->tau;
    hist_row[4] = s_mu;
    hist_row[5] = s_ga;
    hist_row[6] = psure;
    hist_row[7] = res2;
  }
}

int theta_update(DevParams* dp, double* hist, int max_hist, int period, int apply,
                 hipStream_t s) {
  theta_kernel<<<1, 64, 0, s>>>(dp, hist, max_hist, period, apply);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ void tau_kernel(DevParams* dp) {
  if (threadIdx.x == 0 && blockIdx.x == 0) tau_from_rule(dp);
}

int tau_refresh(DevParams* dp, hipStream_t s) {
  tau_kernel<<<1, 64, 0, s>>>(dp);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------- small utils ----
template <typename T>
__global__ void fill_kernel(T* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT)
    p[i] = T(0);
}

template <typename T>
int fill_zero(T* p, size_t count, hipStream_t s) {
  if (count == 0) return 0;
  const int bx = (int)std::min<size_t>((count + kEwNT - 1) / kEwNT, 8192);
  fill_kernel<T><<<bx, kEwNT, 0, s>>>(p, count);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template <typename T>
__global__ void axpy_kernel(T* out, const T* a, const T* b, double beta, size_t count) {
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT)
    out[i] = a[i] + T(beta) * b[i];
}

template <typename T>
int axpy_copy(T* out, const T* a, const T* b, double beta, size_t count, hipStream_t s) {
  const int bx = (int)std::min<size_t>((count + kEwNT - 1) / kEwNT, 8192);
  axpy_kernel<T><<<bx, kEwNT, 0, s>>>(out, a, b, beta, count);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template <typename T>
__global__ void copy_kernel(T* out, const T* in, size_t count) {
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT)
    out[i] = in[i];
}

template <typename T>
int copy_dev(T* out, const T* in, size_t count, hipStream_t s) {
  if (count == 0) return 0;
  const int bx = (int)std::min<size_t>((count + kEwNT - 1) / kEwNT, 8192);
  copy_kernel<T><<<bx, kEwNT, 0, s>>>(out, in, count);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// Per block: sum (a - b)^2 and sum a^2 in FP64 (fixed order: deterministic).
template <typename T>
__global__ void __launch_bounds__(kEwNT) diffsq_kernel(const T* a, const T* b, size_t count,
                                                       double* partials) {
  __shared__ double sh[kEwNT / 64];
  double d2 = 0.0, a2 = 0.0;
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT) {
    const double av = double(a[i]), dv = av - double(b[i]);
    d2 += dv * dv;
    a2 += av * av;
  }
  const double sd = block_sum_all<kEwNT>(d2, sh);
  const double sa = block_sum_all<kEwNT>(a2, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sd;
    partials[2 * blockIdx.x + 1] = sa;
  }
}

__global__ void __launch_bounds__(kEwNT) reduce2_kernel(const double* partials, int count,
                                                        double* out) {
  __shared__ double sh[kEwNT / 64];
  double d = 0.0, a = 0.0;
  for (int i = threadIdx.x; i < count; i += kEwNT) {
    d += partials[2 * i];
    a += partials[2 * i + 1];
  }
  const double sd = block_sum_all<kEwNT>(d, sh);
  const double sa = block_sum_all<kEwNT>(a, sh);
  if (threadIdx.x == 0) {
    out[0] = sd;
    out[1] = sa;
  }
}

template <typename T>
int diff_sq(const T* a, const T* b, size_t count, double* partials, int nblocks, double* out,
            hipStream_t s) {
  diffsq_kernel<T><<<nblocks, kEwNT, 0, s>>>(a, b, count, partials);
  MUFFIN_HIP_CHECK(hipGetLastError());
  reduce2_kernel<<<1, kEwNT, 0, s>>>(partials, nblocks, out);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template <typename T>
__global__ void nonfinite_kernel(const T* p, size_t count, int* flag) {
  int bad = 0;
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT)
    bad |= !isfinite(p[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

template <typename T>
int count_nonfinite(const T* p, size_t count, int* flag, hipStream_t s) {
  const int bx = (int)std::min<size_t>((count + kEwNT - 1) / kEwNT, 4096);
  nonfinite_kernel<T><<<bx, kEwNT, 0, s>>>(p, count, flag);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

template <typename T, typename U>
__global__ void convert_kernel(U* out, const T* in, size_t count) {
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT)
    out[i] = U(in[i]);
}

template <typename T, typename U>
int convert(U* out, const T* in, size_t count, hipStream_t s) {
  const int bx = (int)std::min<size_t>((count + kEwNT - 1) / kEwNT, 8192);
  convert_kernel<T, U><<<bx, kEwNT, 0, s>>>(out, in, count);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------- weights ----
template <typename T>
__global__ void alpha_kernel(const T* x0, int L, int N, double eps, double* alpha) {
  const int p = blockIdx.x * kEwNT + threadIdx.x;
  if (p >= N) return;
  double s = 0.0;
  for (int l = 0; l < L; ++l) {
    const double v = double(x0[(size_t)l * N + p]);
    s += v * v;
  }
  alpha[p] = 1.0 / (sqrt(s) + eps);
}

template <typename T>
__global__ void band_sq_kernel(const T* x0, int N, double* partials, int bpb) {
  __shared__ double sh[kEwNT / 64];
  const int band = blockIdx.y;
  const T* x = x0 + (size_t)band * N;
  double acc = 0.0;
  for (int i = blockIdx.x * kEwNT + threadIdx.x; i < N; i += bpb * kEwNT) {
    const double v = double(x[i]);
    acc += v * v;
  }
  const double s = block_sum_all<kEwNT>(acc, sh);
  if (threadIdx.x == 0) partials[(size_t)band * bpb + blockIdx.x] = s;
}

__global__ void beta_kernel(const double* partials, int L, int bpb, double eps, double* beta) {
  const int band = blockIdx.x * kEwNT + threadIdx.x;
  if (band >= L) return;
  double s = 0.0;
  for (int i = 0; i < bpb; ++i) s += partials[(size_t)band * bpb + i];
  beta[band] = 1.0 / (sqrt(s) + eps);
}

template <typename T>
int weights_from(const T* x0, int L, int N, double eps, double* alpha, double* beta,
                 double* partials, hipStream_t s) {
  alpha_kernel<T><<<(N + kEwNT - 1) / kEwNT, kEwNT, 0, s>>>(x0, L, N, eps, alpha);
  MUFFIN_HIP_CHECK(hipGetLastError());
  const int bpb = 64;
  band_sq_kernel<T><<<dim3(bpb, L), kEwNT, 0, s>>>(x0, N, partials, bpb);
  MUFFIN_HIP_CHECK(hipGetLastError());
  beta_kernel<<<(L + kEwNT - 1) / kEwNT, kEwNT, 0, s>>>(partials, L, bpb, eps, beta);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// beta_l = 1 / (||w_l|| + eps) from per-band coefficient blocks w_l of
// `per_band` values (a redundant dictionary's analysis of the dirty cube)
template <typename T>
int beta_from(const T* w, int L, int per_band, double eps, double* beta, double* partials,
              hipStream_t s) {
  const int bpb = 64;
  band_sq_kernel<T><<<dim3(bpb, L), kEwNT, 0, s>>>(w, per_band, partials, bpb);
  MUFFIN_HIP_CHECK(hipGetLastError());
  beta_kernel<<<(L + kEwNT - 1) / kEwNT, kEwNT, 0, s>>>(partials, L, bpb, eps, beta);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}
template int beta_from<double>(const double*, int, int, double, double*, double*, hipStream_t);
template int beta_from<float>(const float*, int, int, double, double*, double*, hipStream_t);

// --------------------------------------------------------- power iteration --
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void pi_init_kernel(double* v, size_t count, unsigned long long seed) {
  for (size_t i = blockIdx.x * (size_t)kEwNT + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kEwNT) {
    const unsigned long long r = splitmix64(seed ^ (i * 0xD1B54A32D192ED03ull));
    v[i] = double(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

int pi_init(double* v, size_t count, unsigned long long seed, hipStream_t s) {
  const int bx = (int)std::min<size_t>((count + kEwNT - 1) / kEwNT, 8192);
  pi_init_kernel<<<bx, kEwNT, 0, s>>>(v, count, seed);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ void pi_dots_kernel(const double* v, const double* w, int N, double* partials,
                               int bpb) {
  __shared__ double sh[kEwNT / 64];
  const int band = blockIdx.y;
  const double* vb = v + (size_t)band * N;
  const double* wb = w + (size_t)band * N;
  double vw = 0.0, ww = 0.0, vv = 0.0;
  for (int i = blockIdx.x * kEwNT + threadIdx.x; i < N; i += bpb * kEwNT) {
    const double a = vb[i], b = wb[i];
    vw += a * b;
    ww += b * b;
    vv += a * a;
  }
  const double s0 = block_sum_all<kEwNT>(vw, sh);
  const double s1 = block_sum_all<kEwNT>(ww, sh);
  const double s2 = block_sum_all<kEwNT>(vv, sh);
  if (threadIdx.x == 0) {
    double* o = partials + ((size_t)band * bpb + blockIdx.x) * 3;
    o[0] = s0;
    o[1] = s1;
    o[2] = s2;
  }
}

int pi_band_dots(const double* v, const double* w, int L, int N, double* partials, int bpb,
                 hipStream_t s) {
  pi_dots_kernel<<<dim3(bpb, L), kEwNT, 0, s>>>(v, w, N, partials, bpb);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ void pi_finish_kernel(const double* partials, int L, int bpb, double* stats) {
  const int band = blockIdx.x * kEwNT + threadIdx.x;
  if (band >= L) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = 0; i < bpb; ++i) {
    const double* p = partials + ((size_t)band * bpb + i) * 3;
    a += p[0];
    b += p[1];
    c += p[2];
  }
  stats[band * 3 + 0] = a;
  stats[band * 3 + 1] = b;
  stats[band * 3 + 2] = c;
}

int pi_band_finish(const double* partials, int L, int bpb, double* stats, hipStream_t s) {
  pi_finish_kernel<<<(L + kEwNT - 1) / kEwNT, kEwNT, 0, s>>>(partials, L, bpb, stats);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ void pi_norm_kernel(double* v, const double* w, const double* stats, int N) {
  const int band = blockIdx.y;
  const double ww = stats[band * 3 + 1];
  const double inv = ww > 0.0 ? 1.0 / sqrt(ww) : 0.0;
  for (int i = blockIdx.x * kEwNT + threadIdx.x; i < N; i += gridDim.x * kEwNT)
    v[(size_t)band * N + i] = w[(size_t)band * N + i] * inv;
}

int pi_normalise(double* v, const double* w, const double* stats, int L, int N,
                 hipStream_t s) {
  const int bx = std::min(64, (N + kEwNT - 1) / kEwNT);
  pi_norm_kernel<<<dim3(bx, L), kEwNT, 0, s>>>(v, w, stats, N);
  MUFFIN_HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------- instantiations ----
template int primal_step<double>(const PrimalIO<double>&, size_t, const DevParams*, hipStream_t);
template int primal_step<float>(const PrimalIO<float>&, size_t, const DevParams*, hipStream_t);
template int dot_partials<double>(const double*, const double*, const double*, size_t, double*,
                                  int, hipStream_t);
template int dot_partials<float>(const float*, const float*, const float*, size_t, double*, int,
                                 hipStream_t);
template int fill_zero<double>(double*, size_t, hipStream_t);
template int fill_zero<float>(float*, size_t, hipStream_t);
template int fill_zero<uint8_t>(uint8_t*, size_t, hipStream_t);
template int copy_dev<double>(double*, const double*, size_t, hipStream_t);
template int copy_dev<float>(float*, const float*, size_t, hipStream_t);
template int diff_sq<double>(const double*, const double*, size_t, double*, int, double*,
                             hipStream_t);
template int diff_sq<float>(const float*, const float*, size_t, double*, int, double*,
                            hipStream_t);
template int axpy_copy<double>(double*, const double*, const double*, double, size_t, hipStream_t);
template int axpy_copy<float>(float*, const float*, const float*, double, size_t, hipStream_t);
template int count_nonfinite<double>(const double*, size_t, int*, hipStream_t);
template int count_nonfinite<float>(const float*, size_t, int*, hipStream_t);
template int convert<float, double>(double*, const float*, size_t, hipStream_t);
template int convert<double, double>(double*, const double*, size_t, hipStream_t);
template int weights_from<double>(const double*, int, int, double, double*, double*, double*,
                                  hipStream_t);
template int weights_from<float>(const float*, int, int, double, double*, double*, double*,
                                 hipStream_t);

}  // namespace muffin
