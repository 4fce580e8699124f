"""GPU path vs the FP64 CPU oracle, through the C ABI.

Inputs come from the seeded generator (synth); the oracle and the GPU get
the same arrays.  Tolerances: relative L2 <= 1e-12 per FP64 operator,
<= 1e-10 for FP64 iterations (accumulated rounding over hundreds of
iterations), <= 1e-5 for the FP32 form.  Step sizes for the parity runs are
fixed by the test from the PSF's l1 norm (a valid Lipschitz bound by Young's
inequality), so neither side's power iteration enters the comparison.
"""
import numpy as np
import pytest

import synth
from oracle import muffin as om
from oracle import operators as op

pytestmark = pytest.mark.gpu


def _mm():
    from paper_1905_08468_amd import muffin as mm
    return mm


def _torch():
    import torch
    return torch


def dev(a, dtype=None):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    return t.double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    s = np.linalg.norm(np.asarray(b).ravel())
    return d / s if s > 0 else d


def safe_tau(psf, sigma, mu_l, gamma_n, rho=0.9):
    """tau from an l1 bound on ||H_l|| (Young), usable by both sides."""
    bound = max(np.abs(psf[l]).sum() for l in range(psf.shape[0])) ** 2
    return rho / (bound / 2 + sigma * (np.max(mu_l) ** 2 + np.max(gamma_n) ** 2))


def _problem(n, L, seed, counts=None):
    kw = counts or synth.scaled_counts(max(n, 64))
    return synth.make_problem(n, L, seed=seed, **kw)


# ------------------------------------------------------------- operators --

@pytest.mark.parametrize("n,L", [(8, 1), (16, 3), (64, 5), (128, 2), (256, 2)])
def test_convolution_ops_f64(n, L):
    mm = _mm()
    rng = np.random.default_rng(n + L)
    psf = rng.standard_normal((L, 2 * n, 2 * n))   # non-symmetric: complex K
    x = rng.standard_normal((L, n, n))
    K = op.psf_spectrum(psf)
    cfg = mm.default_config(n, L, mode=mm.F64, tau=1.0, pi_iters=0)
    h = mm.Muffin(cfg)
    h.set_problem(dev(x), dev(psf), np.ones(n * n), np.ones(L))
    assert rel(host(h.op("H", dev(x))), op.H(x, K)) < 1e-12
    assert rel(host(h.op("HT", dev(x))), op.HT(x, K)) < 1e-12
    assert rel(host(h.op("HTH", dev(x))), op.HT(op.H(x, K), K)) < 1e-12
    # adjoint identity on the GPU results
    y = rng.standard_normal((L, n, n))
    lhs = np.sum(host(h.op("H", dev(x))) * y)
    rhs = np.sum(x * host(h.op("HT", dev(y))))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12
    h.close()


@pytest.mark.parametrize("n,L,P,J", [(8, 2, 8, 3), (16, 3, 8, 3), (64, 2, 8, 3), (64, 1, 3, 2),
                                     (32, 2, 1, 1), (128, 1, 8, 4), (16, 1, 8, 4)])
def test_wavelet_ops_f64(n, L, P, J):
    mm = _mm()
    rng = np.random.default_rng(7 * n + P)
    x = rng.standard_normal((L, n, n))
    u = rng.standard_normal((L, P, n, n))
    W = op.SpatialDictionary(P, J)
    cfg = mm.default_config(n, L, mode=mm.F64, n_bases=P, levels=J)
    h = mm.Muffin(cfg)
    assert rel(host(h.op("Ws", dev(x))), W.forward(x)) < 1e-12
    assert rel(host(h.op("WsT", dev(u))), W.adjoint(u)) < 1e-12
    h.close()


# FP32: the tile staging by 16-byte vectors (every level whose half-plane
# side is a multiple of four) and its scalar fallback (the coarsest levels of
# n = 8 and 16), the 16- and 32-wide tiles (half-plane side >= 64), P < 8
@pytest.mark.parametrize("n,L,P,J", [(8, 2, 8, 3), (16, 3, 8, 4), (64, 2, 8, 3), (64, 1, 3, 2),
                                     (128, 2, 8, 4), (256, 1, 8, 3), (256, 1, 5, 2)])
def test_wavelet_ops_f32(n, L, P, J):
    mm = _mm()
    torch = _torch()
    rng = np.random.default_rng(11 * n + P)
    x = rng.standard_normal((L, n, n)).astype(np.float32)
    u = rng.standard_normal((L, P, n, n)).astype(np.float32)
    W = op.SpatialDictionary(P, J)
    cfg = mm.default_config(n, L, mode=mm.F32, n_bases=P, levels=J)
    h = mm.Muffin(cfg)
    assert rel(host(h.op("Ws", dev(x, torch.float32))), W.forward(x.astype(np.float64))) < 1e-5
    assert rel(host(h.op("WsT", dev(u, torch.float32))), W.adjoint(u.astype(np.float64))) < 1e-5
    h.close()


@pytest.mark.parametrize("L", [1, 5, 16, 33, 64, 256])
def test_dct_ops_f64(L):
    mm = _mm()
    n = 16
    x = np.random.default_rng(L).standard_normal((L, n, n))
    h = mm.Muffin(mm.default_config(n, L, mode=mm.F64))
    assert rel(host(h.op("dct", dev(x))), op.Wl(x)) < 1e-12
    assert rel(host(h.op("idct", dev(x))), op.WlT(x)) < 1e-12
    h.close()


def test_ops_f32():
    mm = _mm()
    torch = _torch()
    n, L, P = 64, 8, 8
    rng = np.random.default_rng(3)
    prob = _problem(n, L, 3)
    x = rng.standard_normal((L, n, n))
    K = op.psf_spectrum(prob.psf)
    h = mm.Muffin(mm.default_config(n, L, mode=mm.F32, tau=1.0, pi_iters=0))
    h.set_problem(dev(prob.dirty, torch.float32), dev(prob.psf, torch.float32),
                  np.ones(n * n), np.ones(L))
    xf = dev(x, torch.float32)
    x32 = host(xf)
    assert rel(host(h.op("HTH", xf)), op.HT(op.H(x32, K), K)) < 2e-6
    assert rel(host(h.op("Ws", xf)), op.SpatialDictionary(P, 3).forward(x32)) < 2e-6
    assert rel(host(h.op("dct", xf)), op.Wl(x32)) < 2e-6
    h.close()


# ------------------------------------------------------------ iterations --

def _config(mm, n, L, **kw):
    return mm.default_config(n, L, **kw)


def test_one_iteration_from_random_state_f64():
    mm = _mm()
    n, L, P, J = 32, 5, 8, 3
    prob = _problem(n, L, 11)
    alpha, beta = synth.random_weights(L, n, 11)
    X, U, V, T = synth.random_state(L, n, P, 11, scale=float(np.abs(prob.dirty).mean()))
    mu, gamma = 0.7, 0.3
    pb = om.make_problem(prob.dirty, prob.psf, P=P, J=J, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, mu * beta, gamma * alpha)
    ref, _ = om.muffin_step(om.State(X, U, V, T), pb.Y, pb, mu, gamma, tau)
    h = mm.Muffin(_config(mm, n, L, mode=mm.F64, mu=mu, gamma=gamma, tau=tau, pi_iters=0))
    h.set_problem(dev(prob.dirty), dev(prob.psf), alpha, beta)
    for which, arr in enumerate([X, U, V, T]):
        h.set_state(which, 0, dev(arr))
    h.run(1)
    for which, arr in enumerate([ref.X, ref.U, ref.V, ref.T]):
        assert rel(host(h.get_state(which, 0)), arr) < 1e-12, which
    h.close()


def test_c0_plain_f64_200_iterations():
    """Plain FP64 MUFFIN, 64 x 64 x 8, mu = gamma = 1, 200 iterations."""
    mm = _mm()
    n, L = 64, 8
    prob = synth.make_config("c0", seed=0)
    alpha, beta = synth.random_weights(L, n, 0)
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, beta, alpha)
    ref = om.run_muffin(pb, 1.0, 1.0, tau, 200)
    h = mm.Muffin(_config(mm, n, L, mode=mm.F64, mu=1.0, gamma=1.0, tau=tau, pi_iters=0))
    h.set_problem(dev(prob.dirty), dev(prob.psf), alpha, beta)
    h.run(200)
    x = host(h.sky())
    assert rel(x, ref.X) < 1e-10
    for which, arr in [(1, ref.U), (2, ref.V), (3, ref.T)]:
        assert rel(host(h.get_state(which, 0)), arr) < 1e-10
    h.close()


@pytest.mark.parametrize("rule", ["opnorm", "sum"])
def test_setup_weights_lipschitz_tau_f64(rule):
    mm = _mm()
    n, L = 32, 4
    prob = _problem(n, L, 5)
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3)          # weight rule
    bh = om.lipschitz(pb.K, n, iters=2000, tol=1e-14)
    tau_ref = om.tau_rule(bh, 10.0, pb.mu_l(0.8), pb.gamma_n(0.6).ravel(), rule, 0.99)
    cfg = _config(mm, n, L, mode=mm.F64, mu=0.8, gamma=0.6, pi_iters=2000, pi_tol=1e-14,
                  tau_rule=mm.TAU_OPNORM if rule == "opnorm" else mm.TAU_PAPER_SUM)
    h = mm.Muffin(cfg)
    h.set_problem(dev(prob.dirty), dev(prob.psf))
    a, b = h.weights()
    assert rel(a, pb.alpha) < 1e-13 and rel(b, pb.beta) < 1e-13
    rep = h.report()
    assert abs(rep["beta_H"] - bh) <= 1e-8 * bh
    assert abs(rep["tau"] - tau_ref) <= 1e-8 * tau_ref
    h.close()


def _adapt_case(mm, mode, n=32, L=6, iters=12, Delta=3, seed=21, reset=True):
    prob = _problem(n, L, seed)
    alpha, beta = synth.random_weights(L, n, seed)
    mu0, ga0 = 0.5, 0.4
    eps = 0.05 * prob.sigma_w
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, 2 * beta, 2 * alpha)
    ref = om.run_adapt(pb, mu0, ga0, iters, prob.delta, eps, prob.sigma_w, Delta=Delta,
                       eta_mu=2e-4, eta_gamma=2e-4, tau=tau, deriv_reset=reset)
    cfg = _config(mm, n, L, mode=mode, mu=mu0, gamma=ga0, tau=tau, pi_iters=0, sure=1,
                  delta_period=Delta, eps_fd=eps, sigma_w=prob.sigma_w, eta_mu=2e-4,
                  eta_gamma=2e-4, deriv_reset=1 if reset else 0)
    torch = _torch()
    dt = torch.float64 if mode == mm.F64 else torch.float32
    h = mm.Muffin(cfg)
    h.set_problem(dev(prob.dirty, dt), dev(prob.psf, dt), alpha, beta, dev(prob.delta, dt))
    rep = h.run(iters)
    return h, rep, ref


@pytest.mark.parametrize("reset", [True, False])
def test_adapt_f64_matches_oracle(reset):
    mm = _mm()
    h, rep, ref = _adapt_case(mm, mm.F64, reset=reset)
    assert rep["theta_updates"] == len(ref.history) == 4
    hist = h.history()
    for row, r in zip(hist, ref.history):
        assert int(row[0]) == r["k"]
        for j, key in [(4, "sugar_mu"), (5, "sugar_gamma"), (6, "psure")]:
            assert abs(row[j] - r[key]) <= 1e-9 * max(1.0, abs(r[key])), key
        assert abs(row[1] - r["mu"]) <= 1e-12 * max(1.0, abs(r["mu"]))
        assert abs(row[2] - r["gamma"]) <= 1e-12 * max(1.0, abs(r["gamma"]))
    assert rel(host(h.sky()), ref.X) < 1e-10
    st = ref.states
    for s, key in [(1, "Sb"), (2, "Dm"), (3, "Dg"), (4, "Dbm"), (5, "Dbg")]:
        got = host(h.get_state(0, s))
        exp = getattr(st[key], "X")
        assert rel(got, exp) < 1e-9 or np.abs(exp).max() == 0, key
    h.close()


def test_c0_plain_f32_form():
    mm = _mm()
    torch = _torch()
    n, L, iters = 64, 8, 50
    prob = synth.make_config("c0", seed=1)
    alpha, beta = synth.random_weights(L, n, 1)
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, beta, alpha)
    ref = om.run_muffin(pb, 1.0, 1.0, tau, iters)
    h = mm.Muffin(_config(mm, n, L, mode=mm.F32, mu=1.0, gamma=1.0, tau=tau, pi_iters=0))
    h.set_problem(dev(prob.dirty, torch.float32), dev(prob.psf, torch.float32), alpha, beta)
    h.run(iters)
    err = rel(host(h.sky()), ref.X)
    assert err < 1e-5, err
    h.close()


# ------------------------------------------------------------ edge cases --

def test_single_band_and_zero_gamma():
    mm = _mm()
    n, L = 16, 1
    prob = _problem(n, L, 4)
    alpha, beta = synth.random_weights(L, n, 4)
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, beta, alpha)
    for mu, gamma in [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0)]:
        ref = om.run_muffin(pb, mu, gamma, tau, 15)
        h = mm.Muffin(_config(mm, n, L, mode=mm.F64, mu=mu, gamma=gamma, tau=tau, pi_iters=0))
        h.set_problem(dev(prob.dirty), dev(prob.psf), alpha, beta)
        h.run(15)
        assert rel(host(h.sky()), ref.X) < 1e-11
        h.close()


def test_error_codes():
    mm = _mm()
    torch = _torch()
    with pytest.raises(mm.MuffinError) as e:
        mm.Muffin(mm.default_config(48, 4))
    assert e.value.code == -2
    with pytest.raises(mm.MuffinError) as e:
        mm.Muffin(mm.default_config(16, 300))
    assert e.value.code == -2
    with pytest.raises(mm.MuffinError) as e:
        mm.Muffin(mm.default_config(16, 4, sure=1))     # eps_fd, sigma_w missing
    assert e.value.code == -1
    h = mm.Muffin(mm.default_config(16, 2, tau=0.1, pi_iters=0))
    with pytest.raises(mm.MuffinError) as e:
        h.run(1)
    assert e.value.code == -6
    bad = torch.zeros((2, 16, 16), dtype=torch.float64, device="cuda:0")
    bad[1, 3, 3] = float("nan")
    psf = torch.zeros((2, 32, 32), dtype=torch.float64, device="cuda:0")
    psf[:, 16, 16] = 1.0
    with pytest.raises(mm.MuffinError) as e:
        h.set_problem(bad, psf, np.ones(256), np.ones(2))
    assert e.value.code == -4
    h.close()


# ---------------------------------------------- full-size launch configs --

@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_full_side_operators(mode):
    """n = 1024 (the benchmark's FFT, wavelet and tile configuration) on two
    bands, element by element against the oracle."""
    mm = _mm()
    torch = _torch()
    n, L = 1024, 2
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    tol = 1e-12 if mode == "f64" else 3e-6
    rng = np.random.default_rng(101)
    prob = synth.make_problem(n, L, n_src=500, n_blob=20, n_base=20000, seed=101)
    x = np.abs(rng.standard_normal((L, n, n)))
    h = mm.Muffin(mm.default_config(n, L, mode=m, tau=1.0, pi_iters=0))
    h.set_problem(dev(prob.dirty, dt), dev(prob.psf, dt), np.ones(n * n), np.ones(L))
    xd = dev(x, dt)
    xr = host(xd)
    psf = host(dev(prob.psf, dt))
    K = op.psf_spectrum(psf)
    assert rel(host(h.op("HTH", xd)), op.HT(op.H(xr, K), K)) < tol
    W = op.SpatialDictionary(8, 3)
    u = h.op("Ws", xd)
    assert rel(host(u), W.forward(xr)) < tol
    assert rel(host(h.op("WsT", u)), W.adjoint(host(u))) < tol
    h.close()


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_max_side_operators(mode):
    """n = 2048, the largest image side (4096-point column transforms, the
    generic FFT path), one band, element by element against the oracle;
    the starlet dictionary at the same side."""
    mm = _mm()
    torch = _torch()
    n, L = 2048, 1
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    tol = 1e-12 if mode == "f64" else 3e-6
    rng = np.random.default_rng(202)
    prob = synth.make_problem(n, L, n_src=300, n_blob=10, n_base=20000, seed=202)
    x = np.abs(rng.standard_normal((L, n, n)))
    h = mm.Muffin(mm.default_config(n, L, mode=m, tau=1.0, pi_iters=0))
    h.set_problem(dev(prob.dirty, dt), dev(prob.psf, dt), np.ones(n * n), np.ones(L))
    xd = dev(x, dt)
    xr = host(xd)
    K = op.psf_spectrum(host(dev(prob.psf, dt)))
    assert rel(host(h.op("HTH", xd)), op.HT(op.H(xr, K), K)) < tol
    W = op.SpatialDictionary(8, 3)
    u = h.op("Ws", xd)
    assert rel(host(u), W.forward(xr)) < tol
    assert rel(host(h.op("WsT", u)), W.adjoint(host(u))) < tol
    h.close()
    hs = mm.Muffin(mm.default_config(n, L, mode=m, tau=1.0, pi_iters=0,
                                     dictionary=mm.DICT_STARLET, levels=3))
    Ws = op.StarletDictionary(3)
    us = hs.op("Ws", xd)
    assert rel(host(us), Ws.forward(xr)) < tol
    assert rel(host(hs.op("WsT", us)), Ws.adjoint(host(us))) < tol
    hs.close()


@pytest.mark.parametrize("n", [256, 512])
@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_pruned_fft_sides(n, mode):
    """The other sides with pruned FFT passes (n = 256: three-stage
    transforms, 16 rows per block; n = 512: 1024-point columns), H^T H on two
    bands, element by element against the oracle."""
    mm = _mm()
    torch = _torch()
    L = 2
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    tol = 1e-12 if mode == "f64" else 3e-6
    rng = np.random.default_rng(n)
    prob = synth.make_problem(n, L, n_src=200, n_blob=10, n_base=4000, seed=n)
    x = np.abs(rng.standard_normal((L, n, n)))
    h = mm.Muffin(mm.default_config(n, L, mode=m, tau=1.0, pi_iters=0))
    h.set_problem(dev(prob.dirty, dt), dev(prob.psf, dt), np.ones(n * n), np.ones(L))
    xd = dev(x, dt)
    K = op.psf_spectrum(host(dev(prob.psf, dt)))
    assert rel(host(h.op("HTH", xd)), op.HT(op.H(host(xd), K), K)) < tol
    h.close()


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_adapt_pruned_side_256(mode):
    """ADA-PT at n = 256 (all six state sets through the pruned chain, the
    residual partials of its middle row pass), three iterations with a theta
    update after each, against the oracle."""
    mm = _mm()
    m = mm.F64 if mode == "f64" else mm.F32
    h, rep, ref = _adapt_case(mm, m, n=256, L=2, iters=3, Delta=1, seed=41)
    assert rep["theta_updates"] == len(ref.history) == 3
    if mode == "f64":
        assert rel(host(h.sky()), ref.X) < 1e-10
        for s, key in [(1, "Sb"), (2, "Dm"), (3, "Dg"), (4, "Dbm"), (5, "Dbg")]:
            exp = getattr(ref.states[key], "X")
            assert rel(host(h.get_state(0, s)), exp) < 1e-9 or np.abs(exp).max() == 0, key
        for row, r in zip(h.history(), ref.history):
            assert abs(row[6] - r["psure"]) <= 1e-9 * max(1.0, abs(r["psure"]))
            assert abs(row[1] - r["mu"]) <= 1e-12 * max(1.0, abs(r["mu"]))
    else:
        assert rel(host(h.sky()), ref.X) < 1e-5
        assert abs(rep["mu"] - ref.mu) <= 1e-3 * abs(ref.mu)
        assert abs(rep["gamma"] - ref.gamma) <= 1e-3 * abs(ref.gamma)
    h.close()


def test_full_cube_dct_sampled_f32():
    """1024^2 pixels x 256 bands (the benchmark's DCT configuration); sampled
    pixel spectra against the oracle's DCT."""
    mm = _mm()
    torch = _torch()
    n, L = 1024, 256
    g = torch.Generator(device="cuda:0").manual_seed(5)
    x = torch.randn((L, n, n), generator=g, device="cuda:0", dtype=torch.float32)
    h = mm.Muffin(mm.default_config(n, L, mode=mm.F32))
    y = h.op("dct", x)
    z = h.op("idct", x)
    idx = np.random.default_rng(6).choice(n * n, size=512, replace=False)
    ii = torch.from_numpy(idx).to("cuda:0")
    xs = x.reshape(L, -1)[:, ii].double().cpu().numpy()
    ys = y.reshape(L, -1)[:, ii].double().cpu().numpy()
    zs = z.reshape(L, -1)[:, ii].double().cpu().numpy()
    assert rel(ys, op.Wl(xs)) < 3e-6
    assert rel(zs, op.WlT(xs)) < 3e-6
    h.close()


@pytest.mark.timeout(600)
def test_full_cube_operators_sampled_f32():
    """1024^2 pixels x 256 bands (the benchmark's FFT and wavelet launch
    configuration): H^T H, W_s and W_s^T over the whole cube, three sampled
    bands against the oracle."""
    mm = _mm()
    torch = _torch()
    n, L = 1024, 256
    prob = synth.make_config("c2", seed=3, device="cuda:0")
    h = mm.Muffin(mm.default_config(n, L, mode=mm.F32, tau=1.0, pi_iters=0))
    h.set_problem(dev(prob.dirty, torch.float32), dev(prob.psf, torch.float32),
                  np.ones(n * n), np.ones(L))
    g = torch.Generator(device="cuda:0").manual_seed(9)
    x = torch.rand((L, n, n), generator=g, device="cuda:0", dtype=torch.float32)
    y = h.op("HTH", x)
    u = h.op("Ws", x)
    w = h.op("WsT", u)
    W = op.SpatialDictionary(8, 3)
    for b in (0, 131, 255):
        xb = x[b:b + 1].double().cpu().numpy()
        psf32 = prob.psf[b:b + 1].astype(np.float32).astype(np.float64)
        K = op.psf_spectrum(psf32)
        assert rel(host(y[b:b + 1]), op.HT(op.H(xb, K), K)) < 3e-6, b
        ub = host(u[b:b + 1])
        assert rel(ub, W.forward(xb)) < 3e-6, b
        assert rel(host(w[b:b + 1]), W.adjoint(ub)) < 3e-6, b
    h.close()


# --------------------------------------------------------- precision forms --

@pytest.mark.parametrize("L", [1, 7, 32, 40, 256])
def test_dct_ops_bf16_split(L):
    """BF16 hi+lo split DCT: ~2^-17 relative per product."""
    mm = _mm()
    torch = _torch()
    n = 16
    x = np.random.default_rng(L + 1).standard_normal((L, n, n))
    h = mm.Muffin(mm.default_config(n, L, mode=mm.F32_BF16DCT))
    xf = dev(x, torch.float32)
    x32 = host(xf)
    assert rel(host(h.op("dct", xf)), op.Wl(x32)) < 3e-5
    assert rel(host(h.op("idct", xf)), op.WlT(x32)) < 3e-5
    h.close()


def test_c0_plain_bf16_form():
    mm = _mm()
    torch = _torch()
    n, L, iters = 64, 8, 50
    prob = synth.make_config("c0", seed=2)
    alpha, beta = synth.random_weights(L, n, 2)
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, beta, alpha)
    ref = om.run_muffin(pb, 1.0, 1.0, tau, iters)
    h = mm.Muffin(_config(mm, n, L, mode=mm.F32_BF16DCT, mu=1.0, gamma=1.0, tau=tau, pi_iters=0))
    h.set_problem(dev(prob.dirty, torch.float32), dev(prob.psf, torch.float32), alpha, beta)
    h.run(iters)
    err = rel(host(h.sky()), ref.X)
    assert err < 1e-3, err
    h.close()


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_adapt_reduced_precision_forms(form):
    mm = _mm()
    mode = mm.F32 if form == "f32" else mm.F32_BF16DCT
    h, rep, ref = _adapt_case(mm, mode)
    tol = 1e-5 if form == "f32" else 1e-3
    assert rel(host(h.sky()), ref.X) < tol
    # theta after the updates; SUGAR's finite-difference term amplifies
    # rounding by 1/eps, so theta is compared at a looser bound
    assert abs(rep["mu"] - ref.mu) <= 1e-3 * abs(ref.mu)
    assert abs(rep["gamma"] - ref.gamma) <= 1e-3 * abs(ref.gamma)
    h.close()


@pytest.fixture(scope="module")
def full_side_adapt():
    """ADA-PT on one 1024^2 band (the benchmark's side: every state set goes
    through the n = 1024 convolution chain), two iterations, a theta update
    after each; the oracle's run is shared by both precisions."""
    n, L, seed = 1024, 1, 31
    prob = _problem(n, L, seed)
    alpha, beta = synth.random_weights(L, n, seed)
    eps = 0.05 * prob.sigma_w
    pb = om.make_problem(prob.dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, 2 * beta, 2 * alpha)
    kw = dict(mu0=0.5, gamma0=0.4, iters=2, Delta=1, eps=eps, tau=tau)
    ref = om.run_adapt(pb, kw["mu0"], kw["gamma0"], kw["iters"], prob.delta, eps,
                       prob.sigma_w, Delta=1, eta_mu=2e-4, eta_gamma=2e-4, tau=tau)
    return prob, alpha, beta, kw, ref


@pytest.mark.timeout(900)  # the oracle's two 1024^2 iterations take about a minute
@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_full_side_adapt_iterations(mode, full_side_adapt):
    mm = _mm()
    torch = _torch()
    prob, alpha, beta, kw, ref = full_side_adapt
    n, L = 1024, 1
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    cfg = _config(mm, n, L, mode=m, mu=kw["mu0"], gamma=kw["gamma0"], tau=kw["tau"],
                  pi_iters=0, sure=1, delta_period=kw["Delta"], eps_fd=kw["eps"],
                  sigma_w=prob.sigma_w, eta_mu=2e-4, eta_gamma=2e-4)
    h = mm.Muffin(cfg)
    h.set_problem(dev(prob.dirty, dt), dev(prob.psf, dt), alpha, beta, dev(prob.delta, dt))
    rep = h.run(kw["iters"])
    assert rep["theta_updates"] == len(ref.history) == 2
    if mode == "f64":
        assert rel(host(h.sky()), ref.X) < 1e-10
        for s, key in [(1, "Sb"), (2, "Dm"), (3, "Dg"), (4, "Dbm"), (5, "Dbg")]:
            exp = getattr(ref.states[key], "X")
            assert rel(host(h.get_state(0, s)), exp) < 1e-9 or np.abs(exp).max() == 0, key
        for row, r in zip(h.history(), ref.history):
            assert abs(row[1] - r["mu"]) <= 1e-12 * max(1.0, abs(r["mu"]))
            assert abs(row[2] - r["gamma"]) <= 1e-12 * max(1.0, abs(r["gamma"]))
    else:
        assert rel(host(h.sky()), ref.X) < 1e-5
        assert abs(rep["mu"] - ref.mu) <= 1e-3 * abs(ref.mu)
        assert abs(rep["gamma"] - ref.gamma) <= 1e-3 * abs(ref.gamma)
    h.close()


# ------------------------------------------- band counts above 128 (DCT) --
# The spectral kernels give each wave the 16-band output tiles kt and kt + 8;
# the second exists only when L > 128 (bands 128 ... 255: the dual update and
# clip of those DCT coefficients, their mask bits, and the T rows of the
# adjoint product).  Per-band gains drawn uniformly in [0.2, 1.8] spread the
# dirty cube's spectrum over every DCT frequency, so coefficients above 128
# clip from the second iteration on and the derivative role reads set bits.

def _band_gain_case(L, seed):
    n = 32
    prob = _problem(n, L, seed)
    gain = np.random.default_rng(seed + 1000).uniform(0.2, 1.8, L)
    dirty = prob.dirty * gain[:, None, None]
    alpha, beta = synth.random_weights(L, n, seed)
    return n, prob, dirty, alpha, beta


_BAND_REF = {}


def _band_adapt_ref(L, seed, iters, Delta, mu0, ga0, eta):
    key = (L, seed, iters, Delta, mu0, ga0, eta)
    if key not in _BAND_REF:
        n, prob, dirty, alpha, beta = _band_gain_case(L, seed)
        pb = om.make_problem(dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
        tau = safe_tau(prob.psf, 10.0, 2 * mu0 * beta, 2 * ga0 * alpha)
        eps = 0.05 * prob.sigma_w
        ref = om.run_adapt(pb, mu0, ga0, iters, prob.delta, eps, prob.sigma_w, Delta=Delta,
                           eta_mu=eta, eta_gamma=eta, tau=tau)
        # the spectral clip is active above band 128 in the reference run
        _, it = om.muffin_step(ref.states["S"], pb.Y, pb, ref.mu, ref.gamma, tau)
        assert np.mean(np.abs(it["vt"][128:]) > 1) > 0.005
        _BAND_REF[key] = (n, prob, dirty, alpha, beta, tau, eps, ref)
    return _BAND_REF[key]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("form", ["f64", "bf16"])
@pytest.mark.parametrize("L", [129, 200, 256])
def test_adapt_band_counts_above_128(L, form):
    """ADA-PT (Algs. 2-5) at n = 32 with L = 129, 200, 256 bands, 8 iterations
    with theta updates at k = 3 and 6, against the oracle: in FP64 X, V, T of
    all six state sets, U of both trajectories and the theta / SUGAR / PSURE
    history; in the bf16 form X and theta."""
    mm = _mm()
    torch = _torch()
    iters, Delta, mu0, ga0, eta = 8, 3, 0.5, 2.0, 1e-4
    n, prob, dirty, alpha, beta, tau, eps, ref = _band_adapt_ref(L, 61 + L, iters, Delta,
                                                                  mu0, ga0, eta)
    mode = mm.F64 if form == "f64" else mm.F32_BF16DCT
    dt = torch.float64 if form == "f64" else torch.float32
    cfg = _config(mm, n, L, mode=mode, mu=mu0, gamma=ga0, tau=tau, pi_iters=0, sure=1,
                  delta_period=Delta, eps_fd=eps, sigma_w=prob.sigma_w, eta_mu=eta,
                  eta_gamma=eta)
    h = mm.Muffin(cfg)
    h.set_problem(dev(dirty, dt), dev(prob.psf, dt), alpha, beta, dev(prob.delta, dt))
    rep = h.run(iters)
    assert rep["theta_updates"] == len(ref.history) == 2
    if form == "f64":
        assert rel(host(h.sky()), ref.X) < 1e-10
        sets = [(0, "S"), (1, "Sb"), (2, "Dm"), (3, "Dg"), (4, "Dbm"), (5, "Dbg")]
        for s, key in sets:
            st = ref.states[key]
            for which, arr in [(0, st.X), (2, st.V), (3, st.T)]:
                got = host(h.get_state(which, s))
                assert rel(got, arr) < 1e-9 or np.abs(arr).max() == 0, (key, which)
            # the bands above 128 on their own
            got_v = host(h.get_state(2, s))[128:]
            assert rel(got_v, st.V[128:]) < 1e-9 or np.abs(st.V[128:]).max() == 0, key
        for s, key in [(0, "S"), (1, "Sb")]:
            assert rel(host(h.get_state(1, s)), ref.states[key].U) < 1e-9, key
        for row, r in zip(h.history(), ref.history):
            assert int(row[0]) == r["k"]
            for j, key in [(4, "sugar_mu"), (5, "sugar_gamma"), (6, "psure")]:
                assert abs(row[j] - r[key]) <= 1e-9 * max(1.0, abs(r[key])), key
            assert abs(row[1] - r["mu"]) <= 1e-12 * max(1.0, abs(r["mu"]))
            assert abs(row[2] - r["gamma"]) <= 1e-12 * max(1.0, abs(r["gamma"]))
    else:
        assert rel(host(h.sky()), ref.X) < 1e-3
        assert abs(rep["mu"] - ref.mu) <= 1e-3 * abs(ref.mu)
        assert abs(rep["gamma"] - ref.gamma) <= 1e-3 * abs(ref.gamma)
    h.close()


@pytest.mark.timeout(600)
def test_plain_f32_256_bands():
    """Plain MUFFIN in FP32 at n = 32, L = 256 (both k-tiles of every wave of
    the FP32 spectral kernel), 20 iterations against the oracle."""
    mm = _mm()
    torch = _torch()
    L, iters, mu, gamma = 256, 20, 0.5, 2.0
    n, prob, dirty, alpha, beta = _band_gain_case(L, 71)
    pb = om.make_problem(dirty, prob.psf, P=8, J=3, alpha=alpha, beta=beta)
    tau = safe_tau(prob.psf, 10.0, mu * beta, gamma * alpha)
    ref = om.run_muffin(pb, mu, gamma, tau, iters)
    _, it = om.muffin_step(ref, pb.Y, pb, mu, gamma, tau)
    assert np.mean(np.abs(it["vt"][128:]) > 1) > 0.005
    h = mm.Muffin(_config(mm, n, L, mode=mm.F32, mu=mu, gamma=gamma, tau=tau, pi_iters=0))
    h.set_problem(dev(dirty, torch.float32), dev(prob.psf, torch.float32), alpha, beta)
    h.run(iters)
    assert rel(host(h.sky()), ref.X) < 1e-5
    assert rel(host(h.get_state(3, 0)), ref.T) < 1e-4
    h.close()
