"""Pins of the unmixing oracle (Section 4.3): the optimality (KKT)
conditions of the positivity-constrained least squares, exact recovery of
non-negative mixtures, and the closed form for orthonormal endmembers."""
import numpy as np

from oracle import unmix as ou


def _spectra(k, L, seed):
    rng = np.random.default_rng(seed)
    nu = np.linspace(1.0, 2.0, L)
    # power laws with different indices plus a line: positive, independent
    E = np.stack([nu ** rng.uniform(-2.0, 1.0) for _ in range(k)])
    E[-1] += 3.0 * np.exp(-0.5 * ((nu - 1.5) / 0.05) ** 2)
    return E


def test_kkt_conditions_hold():
    rng = np.random.default_rng(1)
    k, L, n = 3, 24, 6
    E = _spectra(k, L, 2)
    X = rng.standard_normal((L, n, n))          # arbitrary signs: active bounds
    A, R = ou.unmix(X, E)
    M = E.T
    for p in range(n * n):
        x = X.reshape(L, -1)[:, p]
        a = A.reshape(k, -1)[:, p]
        g = M.T @ (M @ a - x)                   # gradient of 1/2 |x - M a|^2
        assert np.all(a >= 0)
        assert np.all(g >= -1e-10 * (1 + np.abs(M.T @ x).max()))
        assert np.all(np.abs(g * a) <= 1e-9 * (1 + np.abs(M.T @ x).max()))
        assert abs(R.reshape(-1)[p] - np.sum((x - M @ a) ** 2)) <= 1e-10 * (1 + np.sum(x * x))


def test_exact_recovery_of_nonnegative_mixtures():
    rng = np.random.default_rng(3)
    k, L, n = 3, 32, 5
    E = _spectra(k, L, 4)
    A0 = np.abs(rng.standard_normal((k, n, n)))
    A0[rng.uniform(size=A0.shape) < 0.3] = 0.0  # some endmembers absent
    X = np.einsum("kl,kij->lij", E, A0)
    A, R = ou.unmix(X, E)
    assert np.max(np.abs(A - A0)) <= 1e-10 * np.max(A0)
    assert np.max(R) <= 1e-20 * np.sum(X * X)


def test_orthonormal_endmembers_closed_form():
    rng = np.random.default_rng(5)
    k, L, n = 4, 16, 4
    Q, _ = np.linalg.qr(rng.standard_normal((L, k)))
    E = Q.T                                      # orthonormal rows
    X = rng.standard_normal((L, n, n))
    A, _ = ou.unmix(X, E)
    ref = np.maximum(np.einsum("kl,lij->kij", E, X), 0.0)
    assert np.max(np.abs(A - ref)) <= 1e-12
    sel = ou.unmix_pixels(X, E, [0, 5, 15])
    assert np.allclose(sel, A.reshape(k, -1)[:, [0, 5, 15]].T, atol=0, rtol=0)
    cols = ou.unmix_columns(X.reshape(L, -1)[:, [0, 5, 15]], E)
    assert np.allclose(cols, A.reshape(k, -1)[:, [0, 5, 15]], atol=0, rtol=0)
