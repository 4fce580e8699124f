"""Visibility-domain measurement operator (oracle, FP64, numpy).

Section 1 notes that the algorithm reconstructs the cube from dirty images
or from visibilities alike, only the direct operator changes.  In the
visibility domain the measurements of band l are complex samples of the
sky's Fourier transform at the band's (u, v) points (continuous, in cycles
across the image, |u|, |v| < n / 2), phases referred to the image centre
c = n / 2:
    (H_l x)_k = sum_{i, j} x[i, j] exp(-2 pi i (u_k (i - c) + v_k (j - c)) / n).
For a real cube the data term 1/2 |v_l - H_l x_l|^2 has the gradient
Re H_l^* (H_l x_l - v_l), with
    (Re H_l^* r)[i, j] = Re sum_k r_k exp(+2 pi i (u_k (i - c) + v_k (j - c)) / n).
Everything here is the defining sum written out (O(K N) per band).
"""
from __future__ import annotations

import numpy as np


class VisibilityOperator:
    """uv: (L, K, 2) sample positions per band; n: image side."""

    def __init__(self, uv: np.ndarray, n: int):
        self.uv = np.asarray(uv, np.float64)
        self.n = n
        c = n / 2.0
        idx = np.arange(n) - c
        # per band: row and column phase factors (K, n)
        self._ph = [(np.exp(-2j * np.pi * np.outer(b[:, 0], idx) / n),
                     np.exp(-2j * np.pi * np.outer(b[:, 1], idx) / n)) for b in self.uv]

    def forward(self, x: np.ndarray) -> np.ndarray:
        """(L, n, n) real -> (L, K) complex visibilities."""
        out = []
        for l, (er, ec) in enumerate(self._ph):
            # sum_ij x[i,j] er[k,i] ec[k,j]
            out.append(np.einsum("ki,ij,kj->k", er, x[l], ec))
        return np.stack(out)

    def adjoint(self, r: np.ndarray) -> np.ndarray:
        """(L, K) complex -> (L, n, n) real: Re H^* r."""
        out = []
        for l, (er, ec) in enumerate(self._ph):
            out.append(np.real(np.einsum("k,ki,kj->ij", r[l], er.conj(), ec.conj())))
        return np.stack(out)

    def normal(self, x: np.ndarray) -> np.ndarray:
        """Re H^* H x (the gradient's linear part)."""
        return self.adjoint(self.forward(x))

    def psf(self) -> np.ndarray:
        """The real point spread function of every band on the 2n x 2n
        offset grid, offset (0, 0) at index (n, n):
            psf_l[n + a, n + b] = sum_k cos(2 pi (u_k a + v_k b) / n),
        so that Re H^* H x is the windowed linear convolution of x with it."""
        L = self.uv.shape[0]
        n = self.n
        d = np.arange(2 * n) - n
        out = np.zeros((L, 2 * n, 2 * n))
        for l in range(L):
            er = np.exp(2j * np.pi * np.outer(self.uv[l, :, 0], d) / n)
            ec = np.exp(2j * np.pi * np.outer(self.uv[l, :, 1], d) / n)
            out[l] = np.real(er.T @ ec)
        return out
