"""Pins of the oracle's operators against mathematics, not against itself.

* Daubechies filters: closed forms (tests/golden), sum, double-shift
  orthogonality, vanishing moments, extremal phase.
* H_l: the FFT form equals the defining double sum; adjoint identity; a
  delta PSF gives the identity.
* W_s: every basis orthonormal as a dense matrix (also for lengths shorter
  than the filter); the union is a Parseval frame; Haar and db2 one-level
  transforms equal their hand-written matrices.
* W_lambda: orthonormal; equals scipy's DCT-II / DCT-III (ortho).
"""
import os

import mpmath
import numpy as np
import pytest
import scipy.fft

from oracle import operators as op
from oracle.daubechies import daubechies_lowpass, highpass

GOLD = os.path.join(os.path.dirname(__file__), "golden", "daubechies_closed_forms.txt")


def _closed_forms():
    out = {}
    env = dict(s2=mpmath.sqrt(2), s3=mpmath.sqrt(3), a=mpmath.sqrt(10),
               b=mpmath.sqrt(5 + 2 * mpmath.sqrt(10)))
    with mpmath.workdps(40):
        for line in open(GOLD):
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, expr = line.split(":", 1)
            out[name.strip()] = np.array(
                [float(eval(t, {"__builtins__": {}}, env)) for t in expr.split("|")])
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_daubechies_closed_form(p):
    ref = _closed_forms()[f"db{p}"]
    np.testing.assert_allclose(daubechies_lowpass(p), ref, rtol=0, atol=2e-16)


@pytest.mark.parametrize("p", range(1, 9))
def test_daubechies_invariants(p):
    h = daubechies_lowpass(p)
    g = highpass(h)
    assert h.size == 2 * p
    assert abs(h.sum() - np.sqrt(2)) < 1e-15
    for m in range(p):
        dot = np.dot(h[:h.size - 2 * m], h[2 * m:])
        assert abs(dot - (1.0 if m == 0 else 0.0)) < 1e-15
    k = np.arange(2 * p, dtype=np.float64)
    for j in range(p):                      # p vanishing moments of g
        mom = np.sum(g * k ** j)
        scale = np.sum(np.abs(g) * k ** j)
        assert abs(mom) <= 1e-14 * scale
    assert abs(np.sum(g * k ** p)) > 1e-6 * np.sum(np.abs(g) * k ** p)


@pytest.mark.parametrize("p", range(2, 9))
def test_daubechies_extremal_phase(p):
    # after removing the p zeros at z = -1, all remaining zeros of
    # sum_k h_k z^k lie outside the unit circle (checked with numpy's
    # companion-matrix root finder, not the construction's mpmath roots)
    h = daubechies_lowpass(p)
    rest = np.polydiv(h[::-1], np.poly(-np.ones(p)))[0]
    roots = np.roots(rest)
    assert np.all(np.abs(roots) > 1.0)


def _random_psf(rng, L, n):
    return rng.standard_normal((L, 2 * n, 2 * n))   # not symmetric: complex K


@pytest.mark.parametrize("n", [3, 4, 6])
def test_H_fft_equals_direct_sum(n):
    rng = np.random.default_rng(n)
    L = 2
    psf = _random_psf(rng, L, n)
    K = op.psf_spectrum(psf)
    x = rng.standard_normal((L, n, n))
    r = rng.standard_normal((L, n, n))
    np.testing.assert_allclose(op.H(x, K), op.H_direct(x, psf), rtol=0, atol=1e-12)
    np.testing.assert_allclose(op.HT(r, K), op.HT_direct(r, psf), rtol=0, atol=1e-12)


def test_H_adjoint_identity():
    rng = np.random.default_rng(11)
    L, n = 3, 16
    K = op.psf_spectrum(_random_psf(rng, L, n))
    x = rng.standard_normal((L, n, n))
    y = rng.standard_normal((L, n, n))
    lhs = np.sum(op.H(x, K) * y)
    rhs = np.sum(x * op.HT(y, K))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(x * x) * np.sum(y * y)) * np.abs(K).max()


def test_delta_psf_is_identity():
    n, L = 8, 2
    psf = np.zeros((L, 2 * n, 2 * n))
    psf[:, n, n] = 1.0
    K = op.psf_spectrum(psf)
    x = np.random.default_rng(1).standard_normal((L, n, n))
    np.testing.assert_allclose(op.H(x, K), x, atol=1e-15)
    np.testing.assert_allclose(op.HT(x, K), x, atol=1e-15)


def _basis_matrix(n, J, h, g):
    I = np.eye(n * n).reshape(n * n, n, n)
    return op.dwt2(I, h, g, J).reshape(n * n, n * n).T


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_each_basis_orthonormal(n):
    for J in range(1, int(np.log2(n)) + 1):
        for p in range(1, 9):
            h = daubechies_lowpass(p)
            A = _basis_matrix(n, J, h, highpass(h))
            np.testing.assert_allclose(A.T @ A, np.eye(n * n), atol=2e-15)
            np.testing.assert_allclose(A @ A.T, np.eye(n * n), atol=2e-15)
            # idwt2 is the transpose
            c = np.random.default_rng(p).standard_normal((n, n))
            np.testing.assert_allclose(op.idwt2(c, h, highpass(h), J).ravel(),
                                       A.T @ c.ravel(), atol=1e-14)


@pytest.mark.parametrize("P,J,n", [(8, 3, 16), (8, 1, 8), (3, 2, 8), (1, 3, 8)])
def test_union_is_parseval_and_adjoint(P, J, n):
    W = op.SpatialDictionary(P, J)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, n, n))
    u = rng.standard_normal((2, P, n, n))
    np.testing.assert_allclose(W.adjoint(W.forward(x)), x, atol=1e-14)
    assert abs(np.sum(W.forward(x) ** 2) - np.sum(x ** 2)) < 1e-12 * np.sum(x ** 2)
    assert abs(np.sum(W.forward(x) * u) - np.sum(x * W.adjoint(u))) < 1e-12


def test_haar_one_level_closed_form():
    n = 8
    x = np.random.default_rng(3).standard_normal((n, n))
    h = daubechies_lowpass(1)
    c = op.dwt2(x, h, highpass(h), 1)
    r = 1 / np.sqrt(2)
    lo = r * (x[:, 0::2] + x[:, 1::2])
    hi = r * (x[:, 0::2] - x[:, 1::2])
    rows = np.concatenate([lo, hi], axis=1)
    ref = np.concatenate([r * (rows[0::2] + rows[1::2]), r * (rows[0::2] - rows[1::2])], axis=0)
    np.testing.assert_allclose(c, ref, atol=1e-15)


def test_db2_one_level_matrix():
    # explicit periodised 1-D analysis matrix from the closed-form filter
    M = 8
    s3, s2 = np.sqrt(3), np.sqrt(2)
    h = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * s2)
    g = np.array([h[3], -h[2], h[1], -h[0]])
    A = np.zeros((M, M))
    for k in range(M // 2):
        for m in range(4):
            A[k, (2 * k + m) % M] += h[m]
            A[M // 2 + k, (2 * k + m) % M] += g[m]
    x = np.random.default_rng(4).standard_normal(M)
    c, d = op._analysis_1d(x[None], daubechies_lowpass(2), highpass(daubechies_lowpass(2)), axis=-1)
    np.testing.assert_allclose(np.concatenate([c[0], d[0]]), A @ x, atol=1e-15)


@pytest.mark.parametrize("L", [1, 2, 7, 8, 64])
def test_dct_orthonormal_and_scipy(L):
    C = op.dct_matrix(L)
    np.testing.assert_allclose(C @ C.T, np.eye(L), atol=1e-14)
    x = np.random.default_rng(L).standard_normal((L, 3, 3))
    np.testing.assert_allclose(op.Wl(x), scipy.fft.dct(x, type=2, norm="ortho", axis=0), atol=1e-13)
    np.testing.assert_allclose(op.WlT(x), scipy.fft.idct(x, type=2, norm="ortho", axis=0), atol=1e-13)
