"""Spectral unmixing of a reconstructed cube (oracle, FP64, numpy/scipy).

Section 4.3 (Halo data set) separates the sources of a reconstructed cube by
their spectra: k spectra (the paper takes three, from bright pixels of the
halo and of the two galaxies) are chosen as endmembers, and for every pixel
the contribution of each one is found by a positivity-constrained least
squares problem:
    a^n = argmin_{a >= 0} || x^n - E a ||_2^2,
with x^n the spectrum of pixel n (length L) and E the (L, k) matrix of the
endmember spectra.  The abundance maps are a_j^n arranged as (k, n, n).

The oracle solves each pixel's problem with scipy's non-negative least
squares (Lawson-Hanson active set), pixel by pixel.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import nnls


def unmix(X: np.ndarray, E: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """X: cube (L, n, n); E: endmember spectra (k, L) (row j = spectrum j).
    Returns (A, R): abundances (k, n, n) and the squared residual
    || x^n - E a^n ||^2 per pixel (n, n)."""
    X = np.asarray(X, np.float64)
    E = np.asarray(E, np.float64)
    L, n, _ = X.shape
    k = E.shape[0]
    M = E.T                                   # (L, k)
    A = np.zeros((k, n * n))
    R = np.zeros(n * n)
    S = X.reshape(L, n * n)
    for p in range(n * n):
        a, r = nnls(M, S[:, p])
        A[:, p] = a
        R[p] = r * r
    return A.reshape(k, n, n), R.reshape(n, n)


def unmix_pixels(X: np.ndarray, E: np.ndarray, pixels) -> np.ndarray:
    """The same problem at selected pixels only (flat indices i * n + j):
    abundances (len(pixels), k)."""
    L, n, _ = X.shape
    M = np.asarray(E, np.float64).T
    S = np.asarray(X, np.float64).reshape(L, n * n)
    return np.stack([nnls(M, S[:, p])[0] for p in pixels])


def unmix_columns(S: np.ndarray, E: np.ndarray) -> np.ndarray:
    """The same problem for spectra given as the columns of S (L, m):
    abundances (k, m)."""
    M = np.asarray(E, np.float64).T
    S = np.asarray(S, np.float64)
    return np.stack([nnls(M, S[:, c])[0] for c in range(S.shape[1])], axis=1)
