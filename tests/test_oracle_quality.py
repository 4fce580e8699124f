"""Pins of the oracle's quality measures (Section 4.1, SNR and WMSE).

SNR is pinned by an estimate whose error is a known fraction of the true
sky (closed form), WMSE by the identity operator (plain mean squared error)
and by direct, non-FFT convolution."""
import numpy as np

from oracle import muffin as mf
from oracle import operators as op


def _delta_psf(L, n):
    psf = np.zeros((L, 2 * n, 2 * n))
    psf[:, n, n] = 1.0
    return psf


def test_snr_closed_form():
    rng = np.random.default_rng(11)
    L, n = 3, 8
    truth = np.abs(rng.standard_normal((L, n, n)))
    K = op.psf_spectrum(_delta_psf(L, n))
    for s_db in (0.5, 12.0, 24.0, 31.0):
        r = 10.0 ** (-s_db / 20.0)            # |x* - x| = r |x*|
        snr, _ = mf.quality((1.0 - r) * truth, truth, K)
        assert abs(snr - s_db) < 1e-10
    snr0, _ = mf.quality(np.zeros_like(truth), truth, K)
    assert abs(snr0) < 1e-12                  # the zero estimate: 0 dB


def test_wmse_identity_is_mean_squared_error():
    rng = np.random.default_rng(12)
    L, n = 4, 8
    truth = rng.standard_normal((L, n, n))
    x = truth + 0.1 * rng.standard_normal((L, n, n))
    K = op.psf_spectrum(_delta_psf(L, n))
    _, wmse = mf.quality(x, truth, K)
    assert abs(wmse - np.mean((truth - x) ** 2)) < 1e-14
    _, w0 = mf.quality(truth, truth, K)
    assert w0 == 0.0


def test_wmse_matches_direct_convolution():
    rng = np.random.default_rng(13)
    L, n = 2, 8
    truth = np.abs(rng.standard_normal((L, n, n)))
    x = rng.standard_normal((L, n, n))
    psf = rng.standard_normal((L, 2 * n, 2 * n))
    _, wmse = mf.quality(x, truth, op.psf_spectrum(psf))
    hd = op.H_direct(truth - x, psf)
    ref = sum(np.sum(hd[l] ** 2) for l in range(L)) / (L * n * n)
    assert abs(wmse - ref) <= 1e-12 * ref
