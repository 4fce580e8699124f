"""Pins of the oracle's IUWT (starlet) dictionary, the other choice of W_s
named in Section 2.1: planes add up to the image, the adjoint identity, the
impulse response against polynomial products of the dilated B3 filter,
constants, and ||W_s||^2 against the dense matrix."""
import numpy as np
import pytest

from oracle import operators as op


def test_planes_add_up_to_the_image():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 16, 16))
    for J in (1, 2, 3, 4):
        w = op.StarletDictionary(J).forward(x)
        assert w.shape == (3, J + 1, 16, 16)
        assert np.max(np.abs(w.sum(axis=1) - x)) <= 1e-13


@pytest.mark.parametrize("J,n", [(1, 8), (2, 8), (3, 16), (4, 16), (3, 8)])
def test_adjoint_identity(J, n):
    rng = np.random.default_rng(J * 10 + n)
    W = op.StarletDictionary(J)
    x = rng.standard_normal((2, n, n))
    u = rng.standard_normal((2, J + 1, n, n))
    lhs = np.sum(W.forward(x) * u)
    rhs = np.sum(x * W.adjoint(u))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def _dilated(d):
    k = np.zeros(4 * d + 1)
    k[::d] = [1, 4, 6, 4, 1]
    return k / 16.0


def test_impulse_response_is_the_dilated_filter_product():
    n, J = 64, 3
    e = np.zeros((1, n, n))
    e[0, 0, 0] = 1.0
    w = op.StarletDictionary(J).forward(e)[0]
    # c_j of an impulse = outer(k_j, k_j), k_j = h * h_2 * ... * h_(2^(j-1))
    # (polynomial products), centred at the origin with periodic wrap
    k = np.array([1.0])
    prev = np.zeros((n, n))
    prev[0, 0] = 1.0
    for j in range(1, J + 1):
        k = np.convolve(k, _dilated(2 ** (j - 1)))
        half = (len(k) - 1) // 2
        c = np.zeros((n, n))
        for a, ka in enumerate(k):
            for b, kb in enumerate(k):
                c[(a - half) % n, (b - half) % n] += ka * kb
        assert np.max(np.abs(w[j - 1] - (prev - c))) <= 1e-15
        prev = c
    assert np.max(np.abs(w[J] - prev)) <= 1e-15


def test_constant_image():
    x = np.full((2, 8, 8), 3.5)
    w = op.StarletDictionary(3).forward(x)
    assert np.max(np.abs(w[:, :3])) <= 1e-14
    assert np.max(np.abs(w[:, 3] - 3.5)) <= 1e-14


@pytest.mark.parametrize("J,n", [(1, 8), (2, 8), (3, 8)])
def test_frame_norm_against_dense_matrix(J, n):
    W = op.StarletDictionary(J)
    I = np.eye(n * n).reshape(-1, 1, n, n)
    M = np.stack([W.forward(e).ravel() for e in I], axis=1)
    lam = np.linalg.eigvalsh(M.T @ M)
    assert abs(W.frame_norm2(n) - lam[-1]) <= 1e-12 * lam[-1]
    assert lam[-1] > 1.0                     # redundant, not a Parseval frame
    assert op.SpatialDictionary(2, 1).norm2 == 1.0
