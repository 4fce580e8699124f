"""Linear operators of the MUFFIN model (oracle, FP64, numpy).

Layouts: a cube is (L, n, n), band-major; x[l] is the image x_l of band l
and x[:, i, j] the spectrum x^n of pixel n = i*n + j (Section 2.1).

H_l  (measurement model, eq. `model`): convolution by the PSF of band l.
     The PSF cube is (L, 2n, 2n) with its centre at (n, n); H_l is the
     linear convolution restricted to the image window:
         (H_l x)[i, j] = sum_{a, b < n} psf_l[n + i - a, n + j - b] x[a, b].
W_s  (spatial analysis dictionary, eq. `RegAll`; Section 4.2): the union of
     the first P Daubechies bases, each a J-level 2-D separable periodised
     orthonormal DWT in the Mallat layout, stacked and scaled by 1/sqrt(P)
     so that W_s^T W_s = I.  Coefficients are (L, P, n, n).
W_lambda (spectral analysis dictionary): the orthonormal DCT-II along the
     band axis of every pixel spectrum; W_lambda^T is the DCT-III.
W_s, IUWT form (the other choice named in Section 2.1): the isotropic
     undecimated ("starlet") wavelet transform with J scales, coefficients
     (L, J + 1, n, n): planes 0..J-1 the wavelet scales, plane J the coarse
     approximation (see StarletDictionary).
"""
from __future__ import annotations

import numpy as np

from .daubechies import daubechies_bank

# --------------------------------------------------------------------------
# H_l and its adjoint
# --------------------------------------------------------------------------


def H_direct(x: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """Windowed linear convolution written out as the defining double sum
    (eq. `model`).  O(n^4) per band: tiny sizes only."""
    L, n, _ = x.shape
    out = np.zeros_like(x)
    for l in range(L):
        for i in range(n):
            for j in range(n):
                acc = 0.0
                for a in range(n):
                    for b in range(n):
                        acc += psf[l, n + i - a, n + j - b] * x[l, a, b]
                out[l, i, j] = acc
    return out


def HT_direct(r: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """Adjoint of H_direct, as a double sum."""
    L, n, _ = r.shape
    out = np.zeros_like(r)
    for l in range(L):
        for a in range(n):
            for b in range(n):
                acc = 0.0
                for i in range(n):
                    for j in range(n):
                        acc += psf[l, n + i - a, n + j - b] * r[l, i, j]
                out[l, a, b] = acc
    return out


def psf_spectrum(psf: np.ndarray) -> np.ndarray:
    """K_l = FFT2(ifftshift(psf_l)), the 2n x 2n transfer function.  Because
    psf indices n + i - a stay inside [1, 2n - 1] for i, a < n, the circular
    convolution of the 2n zero-padded image with ifftshift(psf) equals the
    windowed linear convolution on the image window."""
    return np.fft.fft2(np.fft.ifftshift(psf, axes=(1, 2)), axes=(1, 2))


def H(x: np.ndarray, K: np.ndarray) -> np.ndarray:
    """H_l x_l for every band, via the 2n zero-padded FFT (library FFT)."""
    L, n, _ = x.shape
    X = np.fft.fft2(x, s=(2 * n, 2 * n), axes=(1, 2))
    return np.real(np.fft.ifft2(K * X, axes=(1, 2)))[:, :n, :n]


def HT(r: np.ndarray, K: np.ndarray) -> np.ndarray:
    """H_l^T r_l for every band (conjugate transfer function)."""
    L, n, _ = r.shape
    R = np.fft.fft2(r, s=(2 * n, 2 * n), axes=(1, 2))
    return np.real(np.fft.ifft2(np.conj(K) * R, axes=(1, 2)))[:, :n, :n]


# --------------------------------------------------------------------------
# Periodised orthonormal DWT (one basis) and the union W_s
# --------------------------------------------------------------------------


def _analysis_1d(x: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """c[k] = sum_m h[m] x[(2k+m) mod M], d[k] = sum_m g[m] x[(2k+m) mod M],
    k < M/2, along `axis`."""
    x = np.moveaxis(x, axis, -1)
    M = x.shape[-1]
    k = np.arange(M // 2)
    c = np.zeros(x.shape[:-1] + (M // 2,))
    d = np.zeros_like(c)
    for m in range(h.size):
        xs = x[..., (2 * k + m) % M]
        c += h[m] * xs
        d += g[m] * xs
    return np.moveaxis(c, -1, axis), np.moveaxis(d, -1, axis)


def _synthesis_1d(c: np.ndarray, d: np.ndarray, h: np.ndarray, g: np.ndarray,
                  axis: int) -> np.ndarray:
    """Adjoint of _analysis_1d: x[(2k+m) mod M] += h[m] c[k] + g[m] d[k]."""
    c = np.moveaxis(c, axis, -1)
    d = np.moveaxis(d, axis, -1)
    half = c.shape[-1]
    M = 2 * half
    k = np.arange(half)
    x = np.zeros(c.shape[:-1] + (M,))
    for m in range(h.size):
        # for a fixed m the targets (2k+m) mod M are distinct
        x[..., (2 * k + m) % M] += h[m] * c + g[m] * d
    return np.moveaxis(x, -1, axis)


def dwt2(img: np.ndarray, h: np.ndarray, g: np.ndarray, J: int) -> np.ndarray:
    """J-level 2-D periodised DWT of the trailing two axes (square, side
    divisible by 2^J), Mallat layout: at each level the current top-left
    block is filtered along rows (low half left, high half right), then
    along columns (low half top, high half bottom)."""
    out = np.array(img, dtype=np.float64, copy=True)
    M = out.shape[-1]
    for _ in range(J):
        blk = out[..., :M, :M]
        lo, hi = _analysis_1d(blk, h, g, axis=-1)
        rows = np.concatenate([lo, hi], axis=-1)
        lo, hi = _analysis_1d(rows, h, g, axis=-2)
        out[..., :M, :M] = np.concatenate([lo, hi], axis=-2)
        M //= 2
    return out


def idwt2(coef: np.ndarray, h: np.ndarray, g: np.ndarray, J: int) -> np.ndarray:
    """Adjoint (= inverse) of dwt2."""
    out = np.array(coef, dtype=np.float64, copy=True)
    n = out.shape[-1]
    for lev in reversed(range(J)):
        M = n >> lev
        half = M // 2
        blk = out[..., :M, :M]
        cols = _synthesis_1d(blk[..., :half, :], blk[..., half:, :], h, g, axis=-2)
        img = _synthesis_1d(cols[..., :, :half], cols[..., :, half:], h, g, axis=-1)
        out[..., :M, :M] = img
    return out


class SpatialDictionary:
    """W_s = P^{-1/2} [Psi_1; ...; Psi_P] (union of db1..dbP bases)."""

    norm2 = 1.0   # ||W_s||^2: the union of orthonormal bases is a Parseval frame

    def __init__(self, P: int = 8, J: int = 3):
        self.P, self.J = P, J
        self.bank = daubechies_bank(P)

    def forward(self, x: np.ndarray) -> np.ndarray:
        """W_s x_l for every band: (L, n, n) -> (L, P, n, n)."""
        s = 1.0 / np.sqrt(self.P)
        return np.stack([s * dwt2(x, h, g, self.J) for (h, g) in self.bank], axis=1)

    def adjoint(self, u: np.ndarray) -> np.ndarray:
        """W_s^T u_l for every band: (L, P, n, n) -> (L, n, n)."""
        s = 1.0 / np.sqrt(self.P)
        acc = np.zeros(u.shape[:1] + u.shape[2:])
        for p, (h, g) in enumerate(self.bank):
            acc += s * idwt2(u[:, p], h, g, self.J)
        return acc


# --------------------------------------------------------------------------
# W_s, IUWT form: the starlet transform
# --------------------------------------------------------------------------

B3 = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0   # cubic B-spline scaling filter


def b3_smooth(c: np.ndarray, d: int) -> np.ndarray:
    """Separable periodic smoothing of every band with the B3-spline filter
    dilated by d ("a trous": taps at offsets -2d .. 2d):
        out[i, j] = sum_{a, b} h[a] h[b] c[(i + (a-2) d) mod n, (j + (b-2) d) mod n]."""
    rows = sum(B3[a] * np.roll(c, -(a - 2) * d, axis=-2) for a in range(5))
    return sum(B3[b] * np.roll(rows, -(b - 2) * d, axis=-1) for b in range(5))


class StarletDictionary:
    """W_s as the isotropic undecimated wavelet transform with J scales
    (the IUWT of Section 2.1): c_0 = x, c_j = h_(2^(j-1)) * c_(j-1),
    w_j = c_(j-1) - c_j (j = 1..J); W_s x = (w_1, ..., w_J, c_J), so the
    planes add up to x.  Not orthonormal: the adjoint is the transpose of
    the analysis (not the sum of the planes), and ||W_s|| > 1."""

    def __init__(self, J: int = 3):
        self.J = J
        self.P = J + 1   # planes per band

    def forward(self, x: np.ndarray) -> np.ndarray:
        """(L, n, n) -> (L, J + 1, n, n)."""
        c = np.asarray(x, np.float64)
        planes = []
        for j in range(1, self.J + 1):
            cn = b3_smooth(c, 2 ** (j - 1))
            planes.append(c - cn)
            c = cn
        planes.append(c)
        return np.stack(planes, axis=1)

    def adjoint(self, u: np.ndarray) -> np.ndarray:
        """W_s^T: (L, J + 1, n, n) -> (L, n, n).  With H_j the (symmetric)
        smoothing of scale j, W_s^T u = sum_j C_(j-1)^T (I - H_j) u_j
        + C_J^T u_c, C_j = H_j ... H_1, evaluated from the coarsest scale:
        r_J = u_c, r_(j-1) = u_j + H_j (r_j - u_j), W_s^T u = r_0."""
        r = np.asarray(u[:, self.J], np.float64)
        for j in range(self.J, 0, -1):
            uj = u[:, j - 1]
            r = uj + b3_smooth(r - uj, 2 ** (j - 1))
        return r

    def frame_norm2(self, n: int) -> float:
        """||W_s||^2 = largest eigenvalue of W_s^T W_s.  Every scale is a
        periodic convolution, so W_s^T W_s is diagonal in the 2-D DFT: its
        eigenvalues are sum_j |W_j(f)|^2 + |C_J(f)|^2 over the n x n
        frequencies, with the filters' responses taken from the DFT of the
        transform of a unit impulse."""
        e = np.zeros((1, n, n))
        e[0, 0, 0] = 1.0
        resp = np.fft.fft2(self.forward(e)[0])          # (J + 1, n, n)
        return float(np.max(np.sum(np.abs(resp) ** 2, axis=0)))


# --------------------------------------------------------------------------
# W_lambda: orthonormal DCT-II along bands
# --------------------------------------------------------------------------


def dct_matrix(L: int) -> np.ndarray:
    """C[k, l] = c_k cos(pi (2l+1) k / (2L)), c_0 = sqrt(1/L), c_k = sqrt(2/L)."""
    k = np.arange(L)[:, None]
    l = np.arange(L)[None, :]
    C = np.cos(np.pi * (2 * l + 1) * k / (2 * L)) * np.sqrt(2.0 / L)
    C[0, :] = np.sqrt(1.0 / L)
    return C


def Wl(x: np.ndarray) -> np.ndarray:
    """W_lambda x^n for every pixel: the DCT of each spectrum (band axis 0)."""
    C = dct_matrix(x.shape[0])
    return np.tensordot(C, x, axes=(1, 0))


def WlT(v: np.ndarray) -> np.ndarray:
    """W_lambda^T v^n for every pixel (inverse DCT, band axis 0)."""
    C = dct_matrix(v.shape[0])
    return np.tensordot(C.T, v, axes=(1, 0))
