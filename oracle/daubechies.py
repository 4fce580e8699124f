"""Daubechies orthonormal wavelet filters (oracle).

The spatial dictionary W_s is the union of the first eight Daubechies bases
(Section 4.2, implementation details).  The low-pass filter of db_p (p
vanishing moments, 2p taps) is obtained here from its defining property by
spectral factorisation (Daubechies 1988):

    |m0(w)|^2 = cos^{2p}(w/2) * Pp(sin^2(w/2)),
    Pp(y)     = sum_{k<p} binom(p-1+k, k) y^k.

With z = e^{-iw}, sin^2(w/2) = (2 - z - 1/z)/4.  Each root y_j of Pp gives a
reciprocal pair (r, 1/r) of roots in z of z^2 - (2 - 4 y_j) z + 1; the
extremal-phase ("db") filter keeps, for every pair, the root of modulus > 1,
so the filter polynomial is (1 + z)^p prod_j (z - r_j), normalised to a sum
of sqrt(2).  Roots are found with mpmath at 60 significant digits so that the
float64 filters are exact to rounding.
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np


@functools.lru_cache(maxsize=None)
def daubechies_lowpass(p: int) -> np.ndarray:
    """Low-pass analysis filter h of db_p, length 2p, float64."""
    if p < 1:
        raise ValueError("p >= 1")
    with mpmath.workdps(60):
        one = mpmath.mpf(1)
        # Pp(y) coefficients, highest degree first for polyroots
        coeffs = [mpmath.binomial(p - 1 + k, k) for k in range(p)][::-1]
        ys = mpmath.polyroots(coeffs, maxsteps=400, extraprec=200) if p > 1 else []
        poly = [mpmath.mpc(1)]                      # ascending powers of z
        def mul(a, b):
            out = [mpmath.mpc(0)] * (len(a) + len(b) - 1)
            for i, ai in enumerate(a):
                for j, bj in enumerate(b):
                    out[i + j] += ai * bj
            return out
        for _ in range(p):
            poly = mul(poly, [one, one])           # (1 + z)
        for y in ys:
            b = 2 - 4 * y
            disc = mpmath.sqrt(b * b - 4)
            r1, r2 = (b + disc) / 2, (b - disc) / 2
            r = r1 if abs(r1) > abs(r2) else r2
            poly = mul(poly, [-r, one])            # (z - r)
        s = sum(poly)
        h = [mpmath.re(c * mpmath.sqrt(2) / s) for c in poly]
        return np.array([float(v) for v in h], dtype=np.float64)


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature-mirror high-pass g[m] = (-1)^m h[2p-1-m]."""
    m = np.arange(h.size)
    return ((-1.0) ** m) * h[::-1]


def daubechies_bank(P: int = 8):
    """Filters (h, g) of db1 ... dbP."""
    return [(daubechies_lowpass(p), highpass(daubechies_lowpass(p)))
            for p in range(1, P + 1)]
