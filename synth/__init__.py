"""Seeded synthetic wideband radio-imaging inputs.

This module is shared by the CPU oracle, the GPU tests and the benchmark.
It holds no step of the deconvolution method itself: it only draws a sky
cube, a per-band point spread function and a noisy dirty cube, the way the
paper's experiments build their data (Section 4.1: sky convolved band by
band with a wavelength-dependent PSF, plus white Gaussian noise at a given
SNR).  The paper's own cubes (an M31 image, a cluster simulation) and its
SKA1-MID PSFs are not available, so the recipe below stands in for them:

* frequencies  nu_l = 1 + l/(L-1) GHz (linear 1-2 GHz), reference nu0 = 1 GHz;
* sky          K_p point sources at integer pixels, flux LogNormal(0, 1),
               spectrum f (nu/nu0)^a with a ~ U(-1, 0.5); K_b round Gaussian
               blobs, centre uniform, width U(2, 5) px, peak LogNormal(0, 1),
               same spectral law;
* PSF          B baselines uniform in a disc of radius 0.45 n uv cells at nu0,
               scaled by nu_l/nu0, rounded to a 2n x 2n uv grid, each cell
               added with its Hermitian mirror; psf_l is the real inverse FFT
               of that gridded mask, centred at (n, n) and normalised to a peak
               of 1 (a point-symmetric radio "dirty beam");
* dirty cube   y_l = (psf_l * x_l) cropped to the image window, plus noise of
               variance sigma_w^2 = ||H X*||^2 / (N L 10^(SNR/10));
* probe        delta ~ N(0, I), the Monte-Carlo direction of SURE-FDMC.

Visibility data (make_vis_problem), the same sky observed in the visibility
domain: B baselines uniform in a disc of radius 0.22 n cycles across the
image at nu0, scaled by nu_l/nu0 (continuous positions, below the n/2
Nyquist limit in every band); complex visibilities are the exact Fourier
sums of the sky at those positions (phases referred to the image centre
n/2), plus complex noise of variance sigma_w^2 per real component at the
given SNR; the probe is complex N(0, 1) per component.

All draws come from one numpy PCG64 stream per seed in a fixed order, so the
CPU oracle and the GPU path always see bit-identical inputs.  The smoothing
(PSF synthesis and the observation convolution) uses library FFT routines
(scipy.fft / scipy.signal) only.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
import scipy.fft
import scipy.signal

# The named workloads.  Sizes follow the paper's wideband cubes (256 x 256 px
# x 256 bands in Section 4.1) scaled down and up.
CONFIGS = {
    # 64^2 x 8 bands, PSF 128^2 -- small plain-FP64 case
    "c0": dict(n=64, L=8, n_src=20, n_blob=3, n_base=500),
    # 256^2 x 64 bands, PSF 512^2 -- SURE tuning on
    "c1": dict(n=256, L=64, n_src=200, n_blob=10, n_base=4000),
    # 1024^2 x 256 bands, PSF 2048^2 -- precision form / benchmark workload
    "c2": dict(n=1024, L=256, n_src=20000, n_blob=200, n_base=50000),
}


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


@dataclass
class Problem:
    n: int
    L: int
    nu: np.ndarray        # (L,) GHz
    sky: np.ndarray       # (L, n, n) true sky X*
    psf: np.ndarray       # (L, 2n, 2n), centre (n, n), peak 1
    dirty: np.ndarray     # (L, n, n) Y
    sigma_w: float        # noise standard deviation
    delta: np.ndarray     # (L, n, n) N(0, 1) probe
    seed: int


def frequencies(L: int) -> np.ndarray:
    if L == 1:
        return np.array([1.0])
    return 1.0 + np.arange(L, dtype=np.float64) / (L - 1)


def make_sky(rng: np.random.Generator, n: int, nu: np.ndarray, n_src: int,
             n_blob: int) -> np.ndarray:
    L = nu.size
    sky = np.zeros((L, n, n))
    ratio = nu / nu[0]
    # point sources
    pi = rng.integers(0, n, size=n_src)
    pj = rng.integers(0, n, size=n_src)
    flux = rng.lognormal(0.0, 1.0, size=n_src)
    idx = rng.uniform(-1.0, 0.5, size=n_src)
    spec = flux[None, :] * ratio[:, None] ** idx[None, :]          # (L, n_src)
    for l in range(L):
        np.add.at(sky[l], (pi, pj), spec[l])
    # Gaussian blobs, evaluated on a window of +-4 widths (periodic edges are
    # not used: the window is clipped to the image)
    cy = rng.uniform(0, n, size=n_blob)
    cx = rng.uniform(0, n, size=n_blob)
    wid = rng.uniform(2.0, 5.0, size=n_blob)
    peak = rng.lognormal(0.0, 1.0, size=n_blob)
    bidx = rng.uniform(-1.0, 0.5, size=n_blob)
    for b in range(n_blob):
        r = int(np.ceil(4 * wid[b]))
        i0, i1 = max(0, int(cy[b]) - r), min(n, int(cy[b]) + r + 1)
        j0, j1 = max(0, int(cx[b]) - r), min(n, int(cx[b]) + r + 1)
        ii = np.arange(i0, i1)[:, None]
        jj = np.arange(j0, j1)[None, :]
        g = np.exp(-((ii - cy[b]) ** 2 + (jj - cx[b]) ** 2) / (2 * wid[b] ** 2))
        s = peak[b] * ratio ** bidx[b]
        sky[:, i0:i1, j0:j1] += s[:, None, None] * g[None]
    return sky


def _uv_draws(rng: np.random.Generator, n: int, n_base: int):
    rad = 0.45 * n * np.sqrt(rng.uniform(0.0, 1.0, size=n_base))
    ang = rng.uniform(0.0, 2 * np.pi, size=n_base)
    return rad * np.cos(ang), rad * np.sin(ang)


def _uv_mask(u0, v0, n: int, scale: float) -> np.ndarray:
    m = 2 * n
    u = np.rint(u0 * scale).astype(np.int64)
    v = np.rint(v0 * scale).astype(np.int64)
    mask = np.zeros((m, m))
    # centred grid: cell (v, u) sits at (n + v, n + u); Hermitian mirror
    np.add.at(mask, ((n + v) % m, (n + u) % m), 1.0)
    np.add.at(mask, ((n - v) % m, (n - u) % m), 1.0)
    return mask


def make_psf(rng: np.random.Generator, n: int, nu: np.ndarray, n_base: int,
             device=None) -> np.ndarray:
    L = nu.size
    m = 2 * n
    u0, v0 = _uv_draws(rng, n, n_base)
    if device is not None:
        return _torch_psf(lambda l: _uv_mask(u0, v0, n, nu[l] / nu[0]), L, n, device)
    psf = np.empty((L, m, m))
    for l in range(L):
        mask = _uv_mask(u0, v0, n, nu[l] / nu[0])
        beam = np.real(scipy.fft.ifft2(scipy.fft.ifftshift(mask), workers=_workers()))
        beam = scipy.fft.fftshift(beam)
        psf[l] = beam / beam[n, n]
    return psf


def observe(psf: np.ndarray, sky: np.ndarray) -> np.ndarray:
    """Noise-free dirty cube: full linear convolution psf_l * x_l, keeping the
    image window [n, 2n) x [n, 2n) of the full result (centre of the PSF at
    (n, n))."""
    L, n, _ = sky.shape
    out = np.empty_like(sky)
    with scipy.fft.set_workers(_workers()):
        for l in range(L):
            full = scipy.signal.fftconvolve(psf[l], sky[l], mode="full")
            out[l] = full[n:2 * n, n:2 * n]
    return out


def _torch_psf(masks_fn, L, n, device):
    """PSF cube from gridded uv masks with torch.fft on `device` (FP64)."""
    import torch
    m = 2 * n
    out = np.empty((L, m, m))
    for l in range(L):
        mk = torch.from_numpy(masks_fn(l)).to(device)
        beam = torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(mk)).real)
        out[l] = (beam / beam[n, n]).cpu().numpy()
    return out


def _torch_observe(psf: np.ndarray, sky: np.ndarray, device) -> np.ndarray:
    """Same as observe(), linear convolution by a zero-padded 4n FFT with
    torch.fft on `device` (FP64), a few bands at a time."""
    import torch
    L, n, _ = sky.shape
    s = (4 * n, 4 * n)
    out = np.empty_like(sky)
    chunk = max(1, int(2 ** 31 // (16 * s[0] * s[1])))
    for l0 in range(0, L, chunk):
        l1 = min(L, l0 + chunk)
        P = torch.fft.rfft2(torch.from_numpy(psf[l0:l1]).to(device), s=s)
        X = torch.fft.rfft2(torch.from_numpy(sky[l0:l1]).to(device), s=s)
        full = torch.fft.irfft2(P * X, s=s)
        out[l0:l1] = full[:, n:2 * n, n:2 * n].cpu().numpy()
        del P, X, full
    return out


def make_problem(n: int, L: int, n_src: int, n_blob: int, n_base: int,
                 snr_db: float = 20.0, seed: int = 0, device=None) -> Problem:
    """device: None for scipy on the host, or a torch device on which the PSF
    synthesis and the observation convolution run (large cubes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nu = frequencies(L)
    sky = make_sky(rng, n, nu, n_src, n_blob)
    psf = make_psf(rng, n, nu, n_base, device)
    clean = observe(psf, sky) if device is None else _torch_observe(psf, sky, device)
    sigma_w = float(np.sqrt(np.sum(clean ** 2) / (clean.size * 10 ** (snr_db / 10))))
    noise = rng.standard_normal(size=sky.shape)
    dirty = clean + sigma_w * noise
    delta = rng.standard_normal(size=sky.shape)
    return Problem(n=n, L=L, nu=nu, sky=sky, psf=psf, dirty=dirty,
                   sigma_w=sigma_w, delta=delta, seed=seed)


@dataclass
class VisProblem:
    n: int
    L: int
    nu: np.ndarray
    sky: np.ndarray       # (L, n, n)
    uv: np.ndarray        # (L, K, 2) sample positions, cycles across the image
    vis: np.ndarray       # (L, K) complex visibilities
    sigma_w: float        # noise std per real component
    delta: np.ndarray     # (L, K) complex N(0, 1) probe
    seed: int


def _fourier_samples(sky_l: np.ndarray, uv_l: np.ndarray, device=None) -> np.ndarray:
    """sum_ij x[i, j] exp(-2 pi i (u (i - n/2) + v (j - n/2)) / n) at every
    (u, v) of one band."""
    n = sky_l.shape[0]
    idx = np.arange(n) - n / 2.0
    if device is not None:
        import torch
        t = lambda a: torch.from_numpy(a).to(device)
        er = torch.exp(-2j * np.pi * torch.outer(t(uv_l[:, 0]), t(idx)) / n)
        ec = torch.exp(-2j * np.pi * torch.outer(t(uv_l[:, 1]), t(idx)) / n)
        x = t(sky_l).to(torch.complex128)
        return ((er @ x) * ec).sum(dim=1).cpu().numpy()
    er = np.exp(-2j * np.pi * np.outer(uv_l[:, 0], idx) / n)
    ec = np.exp(-2j * np.pi * np.outer(uv_l[:, 1], idx) / n)
    return np.sum((er @ sky_l) * ec, axis=1)


def make_vis_problem(n: int, L: int, n_src: int, n_blob: int, n_base: int,
                     snr_db: float = 20.0, seed: int = 0, device=None) -> VisProblem:
    rng = np.random.Generator(np.random.PCG64(seed))
    nu = frequencies(L)
    sky = make_sky(rng, n, nu, n_src, n_blob)
    rad = 0.22 * n * np.sqrt(rng.uniform(0.0, 1.0, size=n_base))
    ang = rng.uniform(0.0, 2 * np.pi, size=n_base)
    base = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=-1)
    uv = np.stack([base * (nu[l] / nu[0]) for l in range(L)])
    clean = np.stack([_fourier_samples(sky[l], uv[l], device) for l in range(L)])
    power = np.sum(np.abs(clean) ** 2)
    sigma_w = float(np.sqrt(power / (2 * clean.size * 10 ** (snr_db / 10))))
    noise = rng.standard_normal(clean.shape) + 1j * rng.standard_normal(clean.shape)
    delta = rng.standard_normal(clean.shape) + 1j * rng.standard_normal(clean.shape)
    return VisProblem(n=n, L=L, nu=nu, sky=sky, uv=uv, vis=clean + sigma_w * noise,
                      sigma_w=sigma_w, delta=delta, seed=seed)


def make_config(name: str, seed: int = 0, **over) -> Problem:
    kw = dict(CONFIGS[name])
    kw.update(over)
    return make_problem(seed=seed, **kw)


def scaled_counts(n: int) -> dict:
    """Source/blob/baseline counts for an n x n image, interpolated in log
    space between the named anchors (64 -> 20/3/500, 256 -> 200/10/4000,
    1024 -> 20000/200/50000)."""
    xs = np.log2([64, 256, 1024])
    ys = np.log([[20, 3, 500], [200, 10, 4000], [20000, 200, 50000]])
    x = np.log2(n)
    vals = [np.exp(np.interp(x, xs, ys[:, k])) for k in range(3)]
    return dict(n_src=int(round(vals[0])), n_blob=max(1, int(round(vals[1]))),
                n_base=int(round(vals[2])))


def random_weights(L: int, n: int, seed: int = 1):
    """Positive per-band (beta_l) and per-pixel (alpha_n) weights drawn
    uniformly in [0.5, 1.5], for tests that bypass the weight rule."""
    rng = np.random.Generator(np.random.PCG64(seed))
    beta = rng.uniform(0.5, 1.5, size=L)
    alpha = rng.uniform(0.5, 1.5, size=n * n)
    return alpha, beta


def random_state(L: int, n: int, P: int, seed: int = 2, scale: float = 1.0):
    """A synthetic primal/dual state (X >= 0, |U| <= 1, |V| <= 1, T) for tests
    that start an iteration away from zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = scale * rng.exponential(1.0, size=(L, n, n))
    X[rng.uniform(size=X.shape) < 0.3] = 0.0
    U = np.clip(rng.normal(0.0, 0.7, size=(L, P, n, n)), -1.0, 1.0)
    V = np.clip(rng.normal(0.0, 0.7, size=(L, n, n)), -1.0, 1.0)
    T = rng.normal(0.0, 0.1 * scale, size=(L, n, n))
    return X, U, V, T
