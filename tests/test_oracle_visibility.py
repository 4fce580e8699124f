"""Pins of the visibility-domain operator (oracle.visibility): the adjoint
identity, integer sample positions against the library FFT, and the normal
operator against the direct-sum convolution by its point spread function
(the identity the GPU iteration relies on)."""
import numpy as np

from oracle import muffin as mf
from oracle import operators as op
from oracle.visibility import VisibilityOperator


def _uv(L, K, n, seed):
    rng = np.random.default_rng(seed)
    r = 0.45 * n * np.sqrt(rng.uniform(size=(L, K)))
    t = rng.uniform(0, 2 * np.pi, size=(L, K))
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=-1)


def test_adjoint_identity():
    rng = np.random.default_rng(1)
    L, K, n = 2, 37, 8
    H = VisibilityOperator(_uv(L, K, n, 2), n)
    x = rng.standard_normal((L, n, n))
    r = rng.standard_normal((L, K)) + 1j * rng.standard_normal((L, K))
    lhs = np.sum(np.real(np.conj(H.forward(x)) * r))
    rhs = np.sum(x * H.adjoint(r))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_integer_positions_are_fft_samples():
    rng = np.random.default_rng(3)
    n = 16
    uv = rng.integers(-7, 8, size=(1, 20, 2)).astype(float)
    H = VisibilityOperator(uv, n)
    x = rng.standard_normal((1, n, n))
    F = np.fft.fft2(x[0])
    c = n / 2
    want = np.array([F[int(u) % n, int(v) % n] * np.exp(2j * np.pi * (u + v) * c / n)
                     for u, v in uv[0]])
    assert np.max(np.abs(H.forward(x)[0] - want)) <= 1e-11 * np.max(np.abs(want))


def test_normal_operator_is_psf_convolution():
    rng = np.random.default_rng(4)
    L, K, n = 2, 50, 8
    H = VisibilityOperator(_uv(L, K, n, 5), n)
    psf = H.psf()
    assert np.allclose(psf[:, n, n], K)
    assert np.allclose(psf[:, 1:, 1:], psf[:, 1:, 1:][:, ::-1, ::-1])   # symmetric
    x = rng.standard_normal((L, n, n))
    want = op.H_direct(x, psf)
    assert np.max(np.abs(H.normal(x) - want)) <= 1e-11 * np.max(np.abs(want))


def test_visibility_problem_lipschitz_is_top_eigenvalue():
    rng = np.random.default_rng(6)
    L, K, n = 1, 30, 4
    uv = _uv(L, K, n, 7)
    vis = rng.standard_normal((L, K)) + 1j * rng.standard_normal((L, K))
    pb = mf.make_vis_problem(vis, uv, n, P=2, J=1)
    I = np.eye(n * n).reshape(-1, 1, n, n)
    M = np.stack([pb.adj(pb.fwd(e)).ravel() for e in I], axis=1)
    lam = np.linalg.eigvalsh(M)[-1]
    assert abs(mf.lipschitz_op(pb, iters=5000, tol=1e-15) - lam) <= 1e-8 * lam
