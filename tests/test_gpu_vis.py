"""Visibility-domain data (muffin_vis_*, visibilities = 1) against the
oracle's direct sums: back-projection, point spread function and degridding;
the set-up's Lipschitz constant; plain MUFFIN and ADA-PT (theta history,
PSURE, SUGAR) in FP64, where the oracle takes the gradient as
Re H^* (H x - v) by direct sums and the library as the PSF convolution."""
import numpy as np
import pytest

import synth
from oracle import muffin as om
from oracle.visibility import VisibilityOperator

pytestmark = pytest.mark.gpu


def _mm():
    from paper_1905_08468_amd import muffin as mm
    return mm


def host(t):
    return t.double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    s = np.linalg.norm(np.asarray(b).ravel())
    return d / s if s > 0 else d


@pytest.mark.parametrize("n,L,K,mode", [(16, 3, 60, "f64"), (64, 2, 500, "f64"),
                                        (32, 2, 130, "f32")])
def test_prepare_and_degrid_match_oracle(n, L, K, mode):
    mm = _mm()
    import torch
    p = synth.make_vis_problem(n, L, 6, 1, K, seed=n + K)
    H = VisibilityOperator(p.uv, n)
    m = mm.F64 if mode == "f64" else mm.F32
    dirty, psf, dimg, nrm = mm.vis_prepare(p.uv, p.vis, n, m, delta=p.delta)
    tol = 1e-12 if mode == "f64" else 1e-6
    assert rel(host(dirty), H.adjoint(p.vis)) < tol
    assert rel(host(psf), H.psf()) < tol
    assert rel(host(dimg), H.adjoint(p.delta)) < tol
    assert abs(nrm - np.sum(np.abs(p.vis) ** 2)) <= 1e-12 * nrm
    dt = torch.float64 if mode == "f64" else torch.float32
    sky = torch.from_numpy(p.sky).to("cuda", dt)
    got = mm.vis_degrid(p.uv, sky).cpu().numpy()
    ref = H.forward(host(sky))
    assert rel(got, ref) < (1e-11 if mode == "f64" else 1e-6)


def _case(mm, n=16, L=3, K=80, seed=3, sure=False, iters=9, Delta=3):
    p = synth.make_vis_problem(n, L, 6, 1, K, seed=seed)
    alpha, beta = synth.random_weights(L, n, seed)
    pb = om.make_vis_problem(p.vis, p.uv, n, P=8, J=2, alpha=alpha, beta=beta)
    dirty, psf, dimg, nrm = mm.vis_prepare(p.uv, p.vis, n, mm.F64, delta=p.delta)
    bound = np.max(np.abs(host(psf)).sum(axis=(1, 2)))    # >= lambda_max of the PSF convolution
    mu0, ga0 = 0.5, 0.4
    tau = 0.9 / (bound / 2 + 10.0 * ((2 * np.max(beta)) ** 2 + (2 * np.max(alpha)) ** 2))
    cfg = mm.default_config(n, L, mode=mm.F64, levels=2, mu=mu0, gamma=ga0, tau=tau,
                            pi_iters=0, visibilities=1, vis_norm2=nrm, vis_count=2.0 * L * K)
    if sure:
        cfg.sure = 1
        cfg.delta_period = Delta
        cfg.eps_fd = 0.05 * p.sigma_w
        cfg.sigma_w = p.sigma_w
        cfg.eta_mu = cfg.eta_gamma = 2e-4
    h = mm.Muffin(cfg)
    h.set_problem(dirty, psf, alpha, beta, dimg if sure else None)
    return p, pb, h, tau, (mu0, ga0)


def test_plain_iterations_match_oracle():
    mm = _mm()
    p, pb, h, tau, (mu, ga) = _case(mm)
    h.run(9)
    ref = om.run_muffin(pb, mu, ga, tau, 9)
    assert rel(host(h.sky()), ref.X) < 1e-10
    assert rel(host(h.get_state(1, 0)), ref.U) < 1e-10
    h.close()


def test_adapt_matches_oracle():
    mm = _mm()
    p, pb, h, tau, (mu0, ga0) = _case(mm, sure=True, iters=12)
    rep = h.run(12)
    ref = om.run_adapt(pb, mu0, ga0, 12, p.delta, 0.05 * p.sigma_w, p.sigma_w, Delta=3,
                       eta_mu=2e-4, eta_gamma=2e-4, tau=tau)
    assert rep["theta_updates"] == len(ref.history) == 4
    for row, r in zip(h.history(), ref.history):
        assert int(row[0]) == r["k"]
        for j, key in [(4, "sugar_mu"), (5, "sugar_gamma"), (6, "psure")]:
            assert abs(row[j] - r[key]) <= 1e-9 * max(1.0, abs(r[key])), key
        assert abs(row[1] - r["mu"]) <= 1e-12 * max(1.0, abs(r["mu"]))
        assert abs(row[2] - r["gamma"]) <= 1e-12 * max(1.0, abs(r["gamma"]))
    assert rel(host(h.sky()), ref.X) < 1e-10
    h.close()


def test_setup_lipschitz_matches_oracle():
    mm = _mm()
    n, L, K = 16, 2, 70
    p = synth.make_vis_problem(n, L, 5, 1, K, seed=9)
    pb = om.make_vis_problem(p.vis, p.uv, n, P=8, J=2)
    dirty, psf, _, nrm = mm.vis_prepare(p.uv, p.vis, n, mm.F64)
    cfg = mm.default_config(n, L, mode=mm.F64, levels=2, pi_iters=3000, pi_tol=1e-14,
                            visibilities=1, vis_norm2=nrm)
    h = mm.Muffin(cfg)
    h.set_problem(dirty, psf)
    a, b = h.weights()
    assert rel(a, pb.alpha) < 1e-12 and rel(b, pb.beta) < 1e-12
    # the top eigenvalue of the dense normal operator (per band, the max);
    # the power iteration converges at the rate of the eigenvalue gap, so
    # after 3000 steps it is checked to 1e-6 (it approaches from below)
    I = np.eye(n * n).reshape(-1, 1, n, n)
    lam = 0.0
    for l in range(L):
        sub = VisibilityOperator(p.uv[l:l + 1], n)
        M = np.stack([sub.normal(e).ravel() for e in I], axis=1)
        lam = max(lam, np.linalg.eigvalsh(M)[-1])
    got = h.report()["beta_H"]
    assert got <= lam * (1 + 1e-12) and lam - got <= 1e-6 * lam
    h.close()


def test_bad_visibility_configs():
    mm = _mm()
    c = mm.default_config(16, 2, visibilities=1, sure=1, eps_fd=0.1, sigma_w=1.0)
    with pytest.raises(mm.MuffinError) as e:     # no measurement count for PSURE
        mm.Muffin(c)
    assert e.value.code == -1
    with pytest.raises(mm.MuffinError) as e:
        mm.vis_prepare(np.zeros((1, 3, 2)), np.zeros((1, 3)), 4)   # n < 8
    assert e.value.code == -1
