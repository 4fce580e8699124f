"""Pins of the oracle's iteration, derivative recursions and risk estimates.

Each test checks the oracle against a result fixed by mathematics:
closed forms of special cases, an independent dense solver of the same
objective, finite differences, an exactly-computed divergence, Monte-Carlo
unbiasedness, and the eigenvalues of a dense matrix.
"""
import numpy as np
import pytest

from oracle import muffin as mf
from oracle import operators as op
from oracle.daubechies import daubechies_lowpass, highpass


def _dense(fn, L, n):
    """Dense matrix of a per-cube linear map (L, n, n) -> (L, n, n)."""
    I = np.eye(L * n * n).reshape(L * n * n, L, n, n)
    return np.stack([fn(e).ravel() for e in I], axis=1)


def _blur_psf(L, n, width=0.8, delta_w=1.0):
    """Positive, well-conditioned PSF: a unit spike plus a narrow Gaussian."""
    m = 2 * n
    ii, jj = np.meshgrid(np.arange(m) - n, np.arange(m) - n, indexing="ij")
    psf = np.zeros((L, m, m))
    for l in range(L):
        w = width * (1 + 0.3 * l)
        psf[l] = 0.3 * np.exp(-(ii ** 2 + jj ** 2) / (2 * w * w))
        psf[l, n, n] += delta_w
    return psf


def _delta_psf(L, n):
    psf = np.zeros((L, 2 * n, 2 * n))
    psf[:, n, n] = 1.0
    return psf


# ---------------------------------------------------------------- set-up --

def test_power_iteration_equals_eigvalsh():
    rng = np.random.default_rng(0)
    L, n = 3, 4
    psf = rng.standard_normal((L, 2 * n, 2 * n))
    K = op.psf_spectrum(psf)
    lam = mf.lipschitz(K, n, iters=5000, tol=1e-15)
    ref = 0.0
    for l in range(L):
        Hl = _dense(lambda e: op.H_direct(e, psf[l:l + 1]), 1, n)
        ref = max(ref, np.linalg.eigvalsh(Hl.T @ Hl).max())
    assert abs(lam - ref) <= 1e-10 * ref
    assert lam <= np.max(np.abs(K)) ** 2 * (1 + 1e-12)


def test_power_iteration_delta_psf():
    K = op.psf_spectrum(_delta_psf(2, 8))
    assert abs(mf.lipschitz(K, 8) - 1.0) < 1e-12


def test_weights_are_inverse_norms():
    rng = np.random.default_rng(1)
    L, n = 3, 8
    X0 = rng.standard_normal((L, n, n))
    Ws = op.SpatialDictionary(8, 3)
    a, b = mf.weights(X0, Ws, 1e-6)
    # both dictionaries preserve norms (orthonormal DCT, Parseval union)
    np.testing.assert_allclose(a, 1 / (np.linalg.norm(X0.reshape(L, -1), axis=0) + 1e-6), rtol=1e-13)
    np.testing.assert_allclose(b, 1 / (np.linalg.norm(X0.reshape(L, -1), axis=1) + 1e-6), rtol=1e-13)


def test_tau_rules():
    mu_l = np.array([0.1, 0.3])
    g_n = np.array([0.2, 0.05, 0.4])
    t1 = mf.tau_rule(4.0, 10.0, mu_l, g_n, "opnorm", 0.99)
    t2 = mf.tau_rule(4.0, 10.0, mu_l, g_n, "sum", 0.99)
    assert abs(t1 - 0.99 / (2.0 + 10 * (0.09 + 0.16))) < 1e-15
    assert abs(t2 - 0.99 / (2.0 + 10 * (0.01 + 0.09 + 0.04 + 0.0025 + 0.16))) < 1e-15


# ------------------------------------------------------- special cases --

def test_zero_regularisation_is_projected_landweber():
    rng = np.random.default_rng(2)
    L, n = 2, 6
    psf = rng.standard_normal((L, 2 * n, 2 * n))
    Y = rng.standard_normal((L, n, n))
    pb = mf.make_problem(Y, psf, P=2, J=1, alpha=np.ones(n * n), beta=np.ones(L))
    st = mf.State.zeros(L, n, 2)
    st.X = np.abs(rng.standard_normal((L, n, n)))
    tau = 0.01
    new, _ = mf.muffin_step(st, Y, pb, 0.0, 0.0, tau)
    ref = st.X - tau * op.HT_direct(op.H_direct(st.X, psf) - Y, psf)
    np.testing.assert_allclose(new.X, np.maximum(ref, 0), atol=1e-13)
    assert not new.U.any() and not new.V.any() and not new.T.any()


def test_identity_operator_converges_to_positive_part():
    rng = np.random.default_rng(3)
    L, n = 2, 8
    Y = rng.standard_normal((L, n, n))
    pb = mf.make_problem(Y, _delta_psf(L, n), P=2, J=2,
                         alpha=np.ones(n * n), beta=np.ones(L))
    tau = mf.tau_rule(1.0, pb.sigma, pb.mu_l(0.0), pb.gamma_n(0.0).ravel())
    st = mf.run_muffin(pb, 0.0, 0.0, tau, 3000)
    np.testing.assert_allclose(st.X, np.maximum(Y, 0), atol=1e-12)


def test_gamma_zero_separates_bands():
    rng = np.random.default_rng(4)
    L, n = 3, 8
    psf = rng.standard_normal((L, 2 * n, 2 * n)) * 0.2
    psf[:, n, n] += 1
    Y = rng.standard_normal((L, n, n)) + 1
    beta = np.array([0.7, 1.0, 1.3])
    pb = mf.make_problem(Y, psf, P=4, J=2, alpha=np.ones(n * n), beta=beta)
    tau = 0.05
    full = mf.run_muffin(pb, 0.4, 0.0, tau, 30).X
    for l in range(L):
        pl = mf.make_problem(Y[l:l + 1], psf[l:l + 1], P=4, J=2,
                             alpha=np.ones(n * n), beta=beta[l:l + 1])
        np.testing.assert_allclose(mf.run_muffin(pl, 0.4, 0.0, tau, 30).X[0], full[l], atol=1e-13)


def _soft(z, t):
    return np.sign(z) * np.maximum(np.abs(z) - t, 0)


def test_identity_single_basis_limit_is_wavelet_shrinkage():
    # H = I, P = 1, gamma = 0: the minimiser of 1/2||y-x||^2 + mu b ||Psi x||_1
    # is Psi^T soft_{mu b}(Psi y); with a large offset it is >= 0, so the
    # positivity constraint is inactive.
    rng = np.random.default_rng(5)
    L, n, J = 2, 8, 2
    Y = rng.standard_normal((L, n, n)) + 20.0
    beta = np.array([1.0, 0.6])
    mu = 0.5
    pb = mf.make_problem(Y, _delta_psf(L, n), P=1, J=J, alpha=np.ones(n * n), beta=beta)
    tau = mf.tau_rule(1.0, pb.sigma, pb.mu_l(mu), pb.gamma_n(0.0).ravel())
    X = mf.run_muffin(pb, mu, 0.0, tau, 4000).X
    h = daubechies_lowpass(1)
    g = highpass(h)
    ref = np.stack([op.idwt2(_soft(op.dwt2(Y[l], h, g, J), mu * beta[l]), h, g, J)
                    for l in range(L)])
    assert ref.min() > 0
    np.testing.assert_allclose(X, ref, atol=1e-10)


def test_identity_spectral_limit_is_dct_shrinkage():
    rng = np.random.default_rng(6)
    L, n = 6, 4
    Y = rng.standard_normal((L, n, n)) + 15.0
    alpha = rng.uniform(0.5, 1.5, n * n)
    gamma = 0.7
    pb = mf.make_problem(Y, _delta_psf(L, n), P=2, J=1, alpha=alpha, beta=np.ones(L))
    tau = mf.tau_rule(1.0, pb.sigma, pb.mu_l(0.0), pb.gamma_n(gamma).ravel())
    X = mf.run_muffin(pb, 0.0, gamma, tau, 4000).X
    C = op.dct_matrix(L)
    Yp = Y.reshape(L, -1)
    ref = C.T @ _soft(C @ Yp, gamma * alpha[None, :])
    assert ref.min() > 0
    np.testing.assert_allclose(X.reshape(L, -1), ref, atol=1e-10)


def _admm_dense(Hd, y, A, w, iters=40000, rho=1.0):
    """Independent dense ADMM for min 1/2||y - Hx||^2 + ||w * (A x)_{reg}||_1
    + i(x >= 0).  A stacks [I; regularisation rows]; w = weights (0 on the
    positivity block).  x-update uses an explicit inverse."""
    nx = Hd.shape[1]
    npos = nx
    Minv = np.linalg.inv(Hd.T @ Hd + rho * A.T @ A)
    z = np.zeros(A.shape[0])
    u = np.zeros(A.shape[0])
    Hty = Hd.T @ y
    for _ in range(iters):
        x = Minv @ (Hty + rho * A.T @ (z - u))
        Ax = A @ x
        v = Ax + u
        z = np.empty_like(v)
        z[:npos] = np.maximum(v[:npos], 0)
        z[npos:] = _soft(v[npos:], w[npos:] / rho)
        u = u + Ax - z
    return np.maximum(x, 0)


@pytest.mark.parametrize("dictionary", ["daubechies", "starlet"])
def test_dense_solve_matches_objective(dictionary):
    rng = np.random.default_rng(7)
    L, n, P, J = 2, 4, 2, 1
    psf = _blur_psf(L, n)
    Xs = np.abs(rng.standard_normal((L, n, n))) * 2
    K = op.psf_spectrum(psf)
    Y = op.H(Xs, K) + 0.3 * rng.standard_normal((L, n, n))
    alpha = rng.uniform(0.5, 1.5, n * n)
    beta = rng.uniform(0.5, 1.5, L)
    mu, gamma = 0.3, 0.2
    pb = mf.make_problem(Y, psf, P=P, J=J, alpha=alpha, beta=beta, dictionary=dictionary)
    P = pb.Ws.P
    # dense operators, built from the defining sums (not the FFT form)
    Hd = np.zeros((L * n * n, L * n * n))
    for l in range(L):
        blk = _dense(lambda e: op.H_direct(e, psf[l:l + 1]), 1, n)
        Hd[l * n * n:(l + 1) * n * n, l * n * n:(l + 1) * n * n] = blk
    I = np.eye(L * n * n).reshape(-1, L, n, n)
    Ws_full = np.stack([pb.Ws.forward(e).ravel() for e in I], axis=1)
    Wl_full = np.stack([op.Wl(e).ravel() for e in I], axis=1)
    A = np.vstack([np.eye(L * n * n), Ws_full, Wl_full])
    w_sp = np.repeat(mu * beta, P * n * n)
    w_spec = np.tile(gamma * alpha, L)
    w = np.concatenate([np.zeros(L * n * n), w_sp, w_spec])
    xs = _admm_dense(Hd, Y.ravel(), A, w)
    F_star = mf.objective(xs.reshape(L, n, n), pb, mu, gamma)
    beta_H = mf.lipschitz(pb.K, n)
    tau = mf.tau_rule(beta_H, pb.sigma, pb.mu_l(mu), pb.gamma_n(gamma).ravel(),
                      ws_norm2=mf.ws_norm2_of(pb.Ws, n))
    X = mf.run_muffin(pb, mu, gamma, tau, 6000).X
    F = mf.objective(X, pb, mu, gamma)
    assert abs(F - F_star) <= 1e-8 * abs(F_star)
    assert F >= F_star - 1e-9 * abs(F_star)


# --------------------------------------------- derivative recursions --

def _window(pb, Y, st0, mu, gamma, tau, steps):
    st = st0.copy()
    for _ in range(steps):
        st, _ = mf.muffin_step(st, Y, pb, mu, gamma, tau)
    return st


def _deriv_window(pb, Y, st0, mu, gamma, tau, steps):
    L, n, _ = Y.shape
    P = pb.Ws.P
    st = st0.copy()
    dm, dg = mf.State.zeros(L, n, P), mf.State.zeros(L, n, P)
    for _ in range(steps):
        new, it = mf.muffin_step(st, Y, pb, mu, gamma, tau)
        dm = mf.deriv_step_mu(dm, it, pb, mu, gamma, tau)
        dg = mf.deriv_step_gamma(dg, it, pb, mu, gamma, tau)
        st = new
    return st, dm, dg


def _fd_problem(seed=8, dictionary="daubechies"):
    import synth
    rng = np.random.default_rng(seed)
    L, n, P, J = 4, 8, 3, 2
    prob = synth.make_problem(n, L, n_src=6, n_blob=2, n_base=40, seed=seed)
    alpha, beta = synth.random_weights(L, n, seed)
    pb = mf.make_problem(prob.dirty, prob.psf, P=P, J=J, alpha=alpha, beta=beta,
                         dictionary=dictionary)
    P = pb.Ws.P
    X, U, V, T = synth.random_state(L, n, P, seed, scale=float(np.abs(prob.dirty).mean()))
    return pb, mf.State(X, U, V, T), prob


@pytest.mark.parametrize("dictionary", ["daubechies", "starlet"])
@pytest.mark.parametrize("which", ["mu", "gamma"])
def test_derivative_recursions_match_finite_differences(which, dictionary):
    pb, st0, _ = _fd_problem(dictionary=dictionary)
    mu, gamma = 0.8, 0.6
    beta_H = mf.lipschitz(pb.K, pb.Y.shape[1], iters=300, tol=1e-12)
    tau = mf.tau_rule(beta_H, pb.sigma, pb.mu_l(mu), pb.gamma_n(gamma).ravel(),
                      ws_norm2=mf.ws_norm2_of(pb.Ws, pb.Y.shape[1]))
    steps = 5
    _, dm, dg = _deriv_window(pb, pb.Y, st0, mu, gamma, tau, steps)
    d = dm if which == "mu" else dg
    h = 1e-6
    if which == "mu":
        xp = _window(pb, pb.Y, st0, mu + h, gamma, tau, steps).X
        xm = _window(pb, pb.Y, st0, mu - h, gamma, tau, steps).X
    else:
        xp = _window(pb, pb.Y, st0, mu, gamma + h, tau, steps).X
        xm = _window(pb, pb.Y, st0, mu, gamma - h, tau, steps).X
    fd = (xp - xm) / (2 * h)
    scale = np.abs(d.X).max()
    assert scale > 0
    err = np.abs(fd - d.X)
    # away from the kinks of (.)_+ and sat the two agree to FD accuracy
    frac_bad = np.mean(err > 1e-5 * scale)
    assert frac_bad < 0.01
    assert np.median(err) < 1e-7 * scale


# ------------------------------------------------------ risk estimates --

def test_psure_divergence_term_is_exact_in_linear_regime():
    # mu = gamma = 0 and positivity inactive: k Landweber steps from zero are
    # linear in y, X = J y; the FDMC term (1/eps)<H(Xbar - X), delta> equals
    # delta^T H J delta for every eps.
    rng = np.random.default_rng(9)
    L, n = 2, 4
    psf = _blur_psf(L, n)
    K = op.psf_spectrum(psf)
    Y = 50.0 + rng.standard_normal((L, n, n))
    pb = mf.make_problem(Y, psf, P=2, J=1, alpha=np.ones(n * n), beta=np.ones(L))
    tau = 0.2
    k = 4
    delta = rng.standard_normal((L, n, n))
    eps = 0.37
    X = mf.run_muffin(pb, 0.0, 0.0, tau, k).X
    pbb = mf.make_problem(Y + eps * delta, psf, P=2, J=1, alpha=np.ones(n * n), beta=np.ones(L))
    Xb = mf.run_muffin(pbb, 0.0, 0.0, tau, k).X
    assert X.min() > 0 and Xb.min() > 0
    Hd = np.zeros((L * n * n, L * n * n))
    for l in range(L):
        Hd[l * n * n:(l + 1) * n * n, l * n * n:(l + 1) * n * n] = \
            _dense(lambda e: op.H_direct(e, psf[l:l + 1]), 1, n)
    A = np.eye(L * n * n) - tau * Hd.T @ Hd
    J = np.zeros_like(A)
    for _ in range(k):
        J = A @ J + tau * Hd.T
    lhs = np.sum(op.H(Xb - X, K) * delta) / eps
    rhs = delta.ravel() @ Hd @ J @ delta.ravel()
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


@pytest.mark.slow
def test_psure_unbiased_monte_carlo():
    rng = np.random.default_rng(10)
    L, n = 1, 4
    psf = _blur_psf(L, n)
    K = op.psf_spectrum(psf)
    Xs = 50.0 + np.abs(rng.standard_normal((L, n, n)))
    sw = 0.5
    tau, k = 0.2, 3
    est, risk = [], []
    for s in range(400):
        r = np.random.default_rng(1000 + s)
        Y = op.H(Xs, K) + sw * r.standard_normal((L, n, n))
        delta = r.standard_normal((L, n, n))
        eps = 1e-3
        pb = mf.make_problem(Y, psf, P=1, J=1, alpha=np.ones(n * n), beta=np.ones(L))
        pbb = mf.make_problem(Y + eps * delta, psf, P=1, J=1, alpha=np.ones(n * n), beta=np.ones(L))
        X = mf.run_muffin(pb, 0.0, 0.0, tau, k).X
        Xb = mf.run_muffin(pbb, 0.0, 0.0, tau, k).X
        est.append(mf.psure(Y, X, Xb, K, delta, sw, eps))
        risk.append(np.sum(op.H(Xs - X, K) ** 2))
    est, risk = np.array(est), np.array(risk)
    diff = est - risk
    se = diff.std(ddof=1) / np.sqrt(diff.size)
    assert abs(diff.mean()) < 4 * se


def test_sugar_is_derivative_of_psure():
    pb, _, prob = _fd_problem(12)
    L, n, _ = pb.Y.shape
    mu, gamma = 0.5, 0.4
    beta_H = mf.lipschitz(pb.K, n, iters=300, tol=1e-12)
    tau = mf.tau_rule(beta_H, pb.sigma, pb.mu_l(mu), pb.gamma_n(gamma).ravel())
    eps = 0.05 * prob.sigma_w
    delta = prob.delta
    Ybar = pb.Y + eps * delta
    zero = mf.State.zeros(L, n, pb.Ws.P)
    steps = 6

    def psure_at(m, g):
        X = _window(pb, pb.Y, zero, m, g, tau, steps).X
        Xb = _window(pb, Ybar, zero, m, g, tau, steps).X
        return mf.psure(pb.Y, X, Xb, pb.K, delta, prob.sigma_w, eps)

    st, dm, dg = _deriv_window(pb, pb.Y, zero, mu, gamma, tau, steps)
    _, dbm, dbg = _deriv_window(pb, Ybar, zero, mu, gamma, tau, steps)
    s_mu = mf.sugar(pb.Y, st.X, dm.X, dbm.X, pb.K, delta, prob.sigma_w, eps)
    s_ga = mf.sugar(pb.Y, st.X, dg.X, dbg.X, pb.K, delta, prob.sigma_w, eps)
    h = 1e-6
    fd_mu = (psure_at(mu + h, gamma) - psure_at(mu - h, gamma)) / (2 * h)
    fd_ga = (psure_at(mu, gamma + h) - psure_at(mu, gamma - h)) / (2 * h)
    assert abs(s_mu - fd_mu) <= 1e-4 * max(abs(fd_mu), 1e-3 * abs(psure_at(mu, gamma)))
    assert abs(s_ga - fd_ga) <= 1e-4 * max(abs(fd_ga), 1e-3 * abs(psure_at(mu, gamma)))


def test_adapt_loop_updates_theta_and_is_deterministic():
    pb, _, prob = _fd_problem(13)
    n = pb.Y.shape[1]
    beta_H = mf.lipschitz(pb.K, n, iters=300, tol=1e-12)
    kw = dict(iters=9, delta=prob.delta, eps=0.05 * prob.sigma_w, sigma_w=prob.sigma_w,
              Delta=3, eta_mu=1e-3, eta_gamma=1e-3, beta_H=beta_H)
    r1 = mf.run_adapt(pb, 0.5, 0.4, **kw)
    r2 = mf.run_adapt(pb, 0.5, 0.4, **kw)
    assert len(r1.history) == 3
    assert np.array_equal(r1.X, r2.X)
    h0 = r1.history[0]
    assert h0["mu"] == max(0.5 - 1e-3 * h0["sugar_mu"], 0.0)
    assert h0["gamma"] == max(0.4 - 1e-3 * h0["sugar_gamma"], 0.0)
    assert r1.X.min() >= 0


# ------------------------------------------------ the ADA-PT driver itself --
# Algorithm 5 and eq. `adaptgrad`: the driver's SUGAR values must be the
# derivatives of the PSURE it logs, taken over the iterations its reading of
# the derivative state says they cover, and each theta update (with the step
# size refreshed after it) must feed the next window.  The references below
# use only run_muffin / muffin_step and psure(), never the derivative
# recursions or the driver.

def _driver_problem(seed=14):
    pb, _, prob = _fd_problem(seed)
    n = pb.Y.shape[1]
    beta_H = mf.lipschitz(pb.K, n, iters=300, tol=1e-12)
    eps = 0.05 * prob.sigma_w
    return pb, prob, beta_H, eps


def _psure_after(pb, prob, eps, steps, mu, gamma, tau, start=None):
    """PSURE of both trajectories after `steps` iterations of Alg. 2 at fixed
    (mu, gamma, tau), from zero or from the pair of states `start`."""
    L, n, _ = pb.Y.shape
    Ybar = pb.Y + eps * prob.delta
    zero = mf.State.zeros(L, n, pb.Ws.P)
    s0, sb0 = (zero, zero) if start is None else start
    S = _window(pb, pb.Y, s0, mu, gamma, tau, steps)
    Sb = _window(pb, Ybar, sb0, mu, gamma, tau, steps)
    return mf.psure(pb.Y, S.X, Sb.X, pb.K, prob.delta, prob.sigma_w, eps), S, Sb


def _fd_sugar(pb, prob, eps, steps, mu, gamma, tau, start=None, h=1e-6):
    f = lambda m, g: _psure_after(pb, prob, eps, steps, m, g, tau, start)[0]
    return ((f(mu + h, gamma) - f(mu - h, gamma)) / (2 * h),
            (f(mu, gamma + h) - f(mu, gamma - h)) / (2 * h))


def _close(a, b, scale, tol=1e-4):
    return abs(a - b) <= tol * scale


def test_adapt_driver_one_window_sugar_is_fd_of_psure():
    # eta = 0, a single window of Delta = iters: the logged SUGAR values are
    # the derivatives in mu and gamma of the logged PSURE over the whole run
    pb, prob, beta_H, eps = _driver_problem()
    mu, gamma, Delta = 0.5, 0.4, 6
    tau = mf.tau_rule(beta_H, pb.sigma, pb.mu_l(mu), pb.gamma_n(gamma).ravel())
    res = mf.run_adapt(pb, mu, gamma, Delta, prob.delta, eps, prob.sigma_w, Delta=Delta,
                       eta_mu=0.0, eta_gamma=0.0, tau=tau, deriv_reset=True)
    assert len(res.history) == 1
    h0 = res.history[0]
    ps, S, Sb = _psure_after(pb, prob, eps, Delta, mu, gamma, tau)
    assert abs(h0["psure"] - ps) <= 1e-12 * abs(ps)
    assert np.array_equal(res.X, S.X) and np.array_equal(res.Xbar, Sb.X)
    fd_mu, fd_ga = _fd_sugar(pb, prob, eps, Delta, mu, gamma, tau)
    scale = max(abs(fd_mu), abs(fd_ga), 1e-3 * abs(ps))
    assert _close(h0["sugar_mu"], fd_mu, scale), (h0["sugar_mu"], fd_mu)
    assert _close(h0["sugar_gamma"], fd_ga, scale), (h0["sugar_gamma"], fd_ga)
    # the two derivatives are distinct quantities (a swapped pair would fail)
    assert abs(fd_mu - fd_ga) > 10 * 1e-4 * scale


@pytest.mark.parametrize("reset", [True, False])
def test_adapt_driver_three_windows(reset):
    # eta = 0, three windows.  deriv_reset: the SUGAR at k = 3 Delta is the
    # derivative of PSURE over the last window, the Delta-step map from the
    # states at k = 2 Delta (held fixed); without the reset it is the
    # derivative over the whole 3 Delta-step map from zero.  Every logged
    # PSURE is that of the iterates at its k.
    pb, prob, beta_H, eps = _driver_problem(15)
    mu, gamma, Delta = 0.6, 0.3, 3
    tau = mf.tau_rule(beta_H, pb.sigma, pb.mu_l(mu), pb.gamma_n(gamma).ravel())
    res = mf.run_adapt(pb, mu, gamma, 3 * Delta, prob.delta, eps, prob.sigma_w, Delta=Delta,
                       eta_mu=0.0, eta_gamma=0.0, tau=tau, deriv_reset=reset)
    assert [r["k"] for r in res.history] == [Delta, 2 * Delta, 3 * Delta]
    for q, row in enumerate(res.history, start=1):
        ps, _, _ = _psure_after(pb, prob, eps, q * Delta, mu, gamma, tau)
        assert abs(row["psure"] - ps) <= 1e-12 * abs(ps), q
        assert row["mu"] == mu and row["gamma"] == gamma and row["tau"] == tau
    last = res.history[-1]
    ps3, S3, Sb3 = _psure_after(pb, prob, eps, 3 * Delta, mu, gamma, tau)
    assert np.array_equal(res.X, S3.X) and np.array_equal(res.Xbar, Sb3.X)
    assert abs(last["psure"] - mf.psure(pb.Y, res.X, res.Xbar, pb.K, prob.delta,
                                        prob.sigma_w, eps)) <= 1e-12 * abs(ps3)
    if reset:
        _, S2, Sb2 = _psure_after(pb, prob, eps, 2 * Delta, mu, gamma, tau)
        fd_mu, fd_ga = _fd_sugar(pb, prob, eps, Delta, mu, gamma, tau, start=(S2, Sb2))
    else:
        fd_mu, fd_ga = _fd_sugar(pb, prob, eps, 3 * Delta, mu, gamma, tau)
    scale = max(abs(fd_mu), abs(fd_ga), 1e-3 * abs(ps3))
    assert _close(last["sugar_mu"], fd_mu, scale), (last["sugar_mu"], fd_mu)
    assert _close(last["sugar_gamma"], fd_ga, scale), (last["sugar_gamma"], fd_ga)
    # the two readings give different gradients on this problem, so each
    # test can only pass with its own reading
    if reset:
        other = _fd_sugar(pb, prob, eps, 3 * Delta, mu, gamma, tau)
    else:
        _, S2, Sb2 = _psure_after(pb, prob, eps, 2 * Delta, mu, gamma, tau)
        other = _fd_sugar(pb, prob, eps, Delta, mu, gamma, tau, start=(S2, Sb2))
    assert abs(other[0] - fd_mu) > 10 * 1e-4 * scale or abs(other[1] - fd_ga) > 10 * 1e-4 * scale


def test_adapt_driver_theta_step_and_tau_refresh_feed_the_next_window():
    # eta > 0 with tau from the step rule: theta moves against the gradient
    # of PSURE over the first window (eq. `adaptgrad`, clamped at 0), tau is
    # recomputed from the new theta, and the second window runs both
    # trajectories from the states at k = Delta with the new theta and tau.
    pb, prob, beta_H, eps = _driver_problem(16)
    mu0, ga0, Delta = 0.5, 0.4, 4
    eta_mu, eta_ga = 2e-3, 1e-3
    tau_of = lambda m, g: mf.tau_rule(beta_H, pb.sigma, pb.mu_l(m), pb.gamma_n(g).ravel())
    res = mf.run_adapt(pb, mu0, ga0, 2 * Delta, prob.delta, eps, prob.sigma_w, Delta=Delta,
                       eta_mu=eta_mu, eta_gamma=eta_ga, beta_H=beta_H, tau=None,
                       deriv_reset=True)
    tau0 = tau_of(mu0, ga0)
    g_mu, g_ga = _fd_sugar(pb, prob, eps, Delta, mu0, ga0, tau0)
    mu1 = max(mu0 - eta_mu * g_mu, 0.0)
    ga1 = max(ga0 - eta_ga * g_ga, 0.0)
    h0 = res.history[0]
    # the step is a real move, larger than the finite-difference error
    assert abs(mu1 - mu0) > 1e-3 * mu0 and abs(ga1 - ga0) > 1e-3 * ga0
    assert abs(h0["mu"] - mu1) <= 1e-4 * eta_mu * max(abs(g_mu), 1.0)
    assert abs(h0["gamma"] - ga1) <= 1e-4 * eta_ga * max(abs(g_ga), 1.0)
    assert abs(h0["tau"] - tau_of(mu1, ga1)) <= 1e-6 * tau_of(mu1, ga1)
    # second window from the first window's end states, with the driver's
    # own theta_1 (so only its use is under test here)
    _, S1, Sb1 = _psure_after(pb, prob, eps, Delta, mu0, ga0, tau0)
    tau1 = tau_of(h0["mu"], h0["gamma"])
    ps2, S2, Sb2 = _psure_after(pb, prob, eps, Delta, h0["mu"], h0["gamma"], tau1,
                                start=(S1, Sb1))
    np.testing.assert_allclose(res.X, S2.X, rtol=0, atol=1e-12 * np.abs(S2.X).max())
    np.testing.assert_allclose(res.Xbar, Sb2.X, rtol=0, atol=1e-12 * np.abs(Sb2.X).max())
    h1 = res.history[1]
    assert abs(h1["psure"] - ps2) <= 1e-10 * abs(ps2)
    fd_mu, fd_ga = _fd_sugar(pb, prob, eps, Delta, h0["mu"], h0["gamma"], tau1,
                             start=(S1, Sb1))
    scale = max(abs(fd_mu), abs(fd_ga), 1e-3 * abs(ps2))
    assert _close(h1["sugar_mu"], fd_mu, scale) and _close(h1["sugar_gamma"], fd_ga, scale)
    # a run that kept the first step size would end elsewhere
    _, S2_stale, _ = _psure_after(pb, prob, eps, Delta, h0["mu"], h0["gamma"], tau0,
                                  start=(S1, Sb1))
    assert np.abs(S2_stale.X - res.X).max() > 1e-9 * np.abs(res.X).max()


def test_adapt_driver_clamps_theta_at_zero():
    # a step larger than theta ends at 0 (mu, gamma are non-negative,
    # Section 2.1), and the run continues with that value
    pb, prob, beta_H, eps = _driver_problem(17)
    mu0, ga0, Delta = 0.5, 0.4, 3
    tau = mf.tau_rule(beta_H, pb.sigma, pb.mu_l(1.0), pb.gamma_n(1.0).ravel())
    g_mu, g_ga = _fd_sugar(pb, prob, eps, Delta, mu0, ga0, tau)
    big_mu = 10 * mu0 / abs(g_mu)
    big_ga = 10 * ga0 / abs(g_ga)
    res = mf.run_adapt(pb, mu0, ga0, Delta, prob.delta, eps, prob.sigma_w, Delta=Delta,
                       eta_mu=big_mu, eta_gamma=big_ga, tau=tau)
    h0 = res.history[0]
    exp_mu = max(mu0 - big_mu * g_mu, 0.0)
    exp_ga = max(ga0 - big_ga * g_ga, 0.0)
    assert (exp_mu == 0.0) == (h0["mu"] == 0.0) and (exp_ga == 0.0) == (h0["gamma"] == 0.0)
    assert h0["mu"] >= 0.0 and h0["gamma"] >= 0.0
    assert h0["mu"] == 0.0 or h0["gamma"] == 0.0
