"""The IUWT (starlet) spatial dictionary on the GPU against the oracle:
the transform and its adjoint, the set-up (weights from the transform of
the dirty cube, ||W_s||^2 in the step rule), plain MUFFIN iterations in FP64
and FP32, and ADA-PT (all six state sets and the theta history) in FP64."""
import numpy as np
import pytest

import synth
from oracle import muffin as om
from oracle import operators as op

pytestmark = pytest.mark.gpu


def _mm():
    from paper_1905_08468_amd import muffin as mm
    return mm


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).to("cuda:0")


def host(t):
    return t.double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    s = np.linalg.norm(np.asarray(b).ravel())
    return d / s if s > 0 else d


def _cfg(mm, n, L, J, **kw):
    return mm.default_config(n, L, dictionary=mm.DICT_STARLET, levels=J, **kw)


@pytest.mark.parametrize("n,L,J", [(8, 2, 1), (8, 1, 3), (32, 3, 2), (64, 2, 3), (128, 2, 5)])
@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_transform_and_adjoint(n, L, J, mode):
    mm = _mm()
    import torch
    dt = torch.float64 if mode == "f64" else torch.float32
    rng = np.random.default_rng(n + L + J)
    x = rng.standard_normal((L, n, n))
    u = rng.standard_normal((L, J + 1, n, n))
    m = mm.F64 if mode == "f64" else mm.F32
    h = mm.Muffin(_cfg(mm, n, L, J, mode=m))
    assert h.planes == J + 1
    W = op.StarletDictionary(J)
    xd, ud = dev(x, dt), dev(u, dt)
    got_w = host(h.op("Ws", xd))
    got_t = host(h.op("WsT", ud))
    ref_w = W.forward(x.astype(np.float32).astype(np.float64) if mode == "f32" else x)
    ref_t = W.adjoint(u.astype(np.float32).astype(np.float64) if mode == "f32" else u)
    tol = 1e-13 if mode == "f64" else 2e-6
    assert rel(got_w, ref_w) < tol and rel(got_t, ref_t) < tol
    h.close()


def test_setup_weights_and_step_rule():
    mm = _mm()
    n, L, J = 32, 4, 3
    prob = synth.make_problem(n, L, seed=5, **synth.scaled_counts(64))
    pb = om.make_problem(prob.dirty, prob.psf, J=J, dictionary="starlet")
    h = mm.Muffin(_cfg(mm, n, L, J, mode=mm.F64, mu=0.8, gamma=0.6, pi_iters=2000,
                       pi_tol=1e-14))
    h.set_problem(dev(prob.dirty), dev(prob.psf))
    a, b = h.weights()
    assert rel(a, pb.alpha) < 1e-13 and rel(b, pb.beta) < 1e-13
    rep = h.report()
    nrm = om.ws_norm2_of(pb.Ws, n)
    tau_ref = om.tau_rule(rep["beta_H"], 10.0, pb.mu_l(0.8), pb.gamma_n(0.6).ravel(),
                          ws_norm2=nrm)
    assert abs(rep["tau"] - tau_ref) <= 1e-12 * tau_ref
    h.close()


def _tau(psf, sigma, mu_l, gamma_n, nrm, rho=0.9):
    bound = max(np.abs(psf[l]).sum() for l in range(psf.shape[0])) ** 2
    return rho / (bound / 2 + sigma * (nrm * np.max(mu_l) ** 2 + np.max(gamma_n) ** 2))


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_plain_iterations_match_oracle(mode):
    mm = _mm()
    import torch
    n, L, J, iters = 32, 4, 3, 15
    prob = synth.make_problem(n, L, seed=6, **synth.scaled_counts(64))
    alpha, beta = synth.random_weights(L, n, 6)
    pb = om.make_problem(prob.dirty, prob.psf, J=J, alpha=alpha, beta=beta, dictionary="starlet")
    mu, gamma = 0.7, 0.4
    tau = _tau(prob.psf, 10.0, mu * beta, gamma * alpha, om.ws_norm2_of(pb.Ws, n))
    ref = om.run_muffin(pb, mu, gamma, tau, iters)
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    h = mm.Muffin(_cfg(mm, n, L, J, mode=m, mu=mu, gamma=gamma, tau=tau, pi_iters=0))
    h.set_problem(dev(prob.dirty, dt), dev(prob.psf, dt), alpha, beta)
    h.run(iters)
    tol = 1e-10 if mode == "f64" else 1e-5
    assert rel(host(h.sky()), ref.X) < tol
    assert rel(host(h.get_state(1, 0)), ref.U) < tol
    h.close()


def test_adapt_f64_matches_oracle():
    mm = _mm()
    n, L, J, iters, Delta = 32, 4, 2, 12, 3
    prob = synth.make_problem(n, L, seed=21, **synth.scaled_counts(64))
    alpha, beta = synth.random_weights(L, n, 21)
    mu0, ga0, eps = 0.5, 0.4, 0.05 * prob.sigma_w
    pb = om.make_problem(prob.dirty, prob.psf, J=J, alpha=alpha, beta=beta, dictionary="starlet")
    tau = _tau(prob.psf, 10.0, 2 * beta, 2 * alpha, om.ws_norm2_of(pb.Ws, n))
    ref = om.run_adapt(pb, mu0, ga0, iters, prob.delta, eps, prob.sigma_w, Delta=Delta,
                       eta_mu=2e-4, eta_gamma=2e-4, tau=tau)
    cfg = _cfg(mm, n, L, J, mode=mm.F64, mu=mu0, gamma=ga0, tau=tau, pi_iters=0, sure=1,
               delta_period=Delta, eps_fd=eps, sigma_w=prob.sigma_w, eta_mu=2e-4,
               eta_gamma=2e-4)
    h = mm.Muffin(cfg)
    h.set_problem(dev(prob.dirty), dev(prob.psf), alpha, beta, dev(prob.delta))
    rep = h.run(iters)
    assert rep["theta_updates"] == len(ref.history) == 4
    for row, r in zip(h.history(), ref.history):
        assert int(row[0]) == r["k"]
        for j, key in [(4, "sugar_mu"), (5, "sugar_gamma"), (6, "psure")]:
            assert abs(row[j] - r[key]) <= 1e-9 * max(1.0, abs(r[key])), key
        assert abs(row[1] - r["mu"]) <= 1e-12 * max(1.0, abs(r["mu"]))
        assert abs(row[2] - r["gamma"]) <= 1e-12 * max(1.0, abs(r["gamma"]))
    assert rel(host(h.sky()), ref.X) < 1e-10
    for s, key in [(1, "Sb"), (2, "Dm"), (3, "Dg"), (4, "Dbm"), (5, "Dbg")]:
        got = host(h.get_state(0, s))
        exp = ref.states[key].X
        assert rel(got, exp) < 1e-9 or np.abs(exp).max() == 0, key
    h.close()


def test_bad_starlet_configs():
    mm = _mm()
    with pytest.raises(mm.MuffinError) as e:
        mm.Muffin(_cfg(mm, 32, 2, 6))            # at most 5 scales
    assert e.value.code == -2
    c = mm.default_config(32, 2)
    c.dictionary = 7
    with pytest.raises(mm.MuffinError) as e:
        mm.Muffin(c)
    assert e.value.code == -1
