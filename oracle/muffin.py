"""MUFFIN, its derivative recursions and ADA-PT (oracle, FP64, numpy).

Paper passages followed (arXiv 1905.08468):
  weights            Section 2.1, eq. `2regpar` and the alpha/beta rule below it
  step-size rule     Section 2.2, the condition on tau and sigma after eq. `sat`
  prox operators     Section 2.2, eqs. `projpos` and `sat`
  one iteration      Algorithm 2 (eqs. `updatenode2` ... `upt`), which is
                     Algorithm 1 (eqs. `grad1` ... `updatex1`) split by band
                     and by pixel
  d/dmu recursion    Algorithm 3
  d/dgamma recursion Algorithm 4 (the text of Section 3.2 names the two
                     algorithms the other way round; the captions and the
                     equations decide: Alg. 3 is d/dmu, Alg. 4 is d/dgamma)
  weak derivatives   Section 3.2, the definitions of U(.) and Pi(.)
  PSURE-FDMC         Section 3.1, eqs. `PSURE`, `PSURE0`
  SUGAR-FDMC         Section 3.2, eq. `SUGAR`
  ADA-PT             Section 3.3, eq. `adaptgrad` and Algorithm 5
  objective          Section 2.1, eqs. `probopt`, `RegAll`
  W_s choices        Section 2.1: the union of Daubechies bases or the IUWT
                     (operators.StarletDictionary); the step rule carries
                     ||W_s||^2 of the condition of Section 2.2
  SNR, WMSE          Section 4.1, the two point estimates of quality
  visibilities       Section 1 (the same algorithm with the visibility-domain
                     direct operator, oracle.visibility)

Readings where the paper is silent (each also listed in the design notes):
  * X, U, V, T and all derivative states start at zero.
  * tau is either the operator-norm form of the step condition
    (rule "opnorm": tau = rho / (beta_H/2 + sigma (max mu_l^2 + max gamma_n^2)))
    or the printed sum form (rule "sum"); tau is recomputed after every
    theta update and is a constant for the derivative recursions.
  * theta is updated after every Delta completed iterations, from X^(k) and
    the derivatives accumulated since the start of the window; derivative
    states (X', U', V', T') are then reset to zero (or carried over when
    `deriv_reset` is False).  theta is clamped at >= 0.
  * the perturbed run (Y + eps delta) uses the same weights, tau and theta.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .operators import H, HT, SpatialDictionary, StarletDictionary, Wl, WlT, psf_spectrum

# --------------------------------------------------------------------------
# prox operators and weak derivatives (eqs. projpos, sat; Section 3.2)
# --------------------------------------------------------------------------


def pos(u):
    """(u)_+ : u where u > 0, else 0 (eq. `projpos`)."""
    return np.where(u > 0, u, 0.0)


def sat(u):
    """sat(u): -1 below -1, 1 above 1, u otherwise (eq. `sat`)."""
    return np.where(u < -1, -1.0, np.where(u > 1, 1.0, u))


def U_weak(u):
    """Weak derivative of (.)_+: 1 if u > 0 else 0."""
    return (u > 0).astype(np.float64)


def Pi_weak(u):
    """Weak derivative of sat: 1 if -1 <= u <= 1 else 0."""
    return ((u >= -1) & (u <= 1)).astype(np.float64)


# --------------------------------------------------------------------------
# set-up: weights, Lipschitz constant, step sizes
# --------------------------------------------------------------------------


def weights(X0: np.ndarray, Ws: SpatialDictionary, eps_w: float):
    """alpha_n = 1/(||W_lambda x0^n||_2 + eps), beta_l = 1/(||W_s x0_l||_2 + eps)
    (Section 2.1, below eq. `2regpar`).  Returns alpha (N,), beta (L,)."""
    L, n, _ = X0.shape
    wl = Wl(X0).reshape(L, n * n)
    alpha = 1.0 / (np.sqrt(np.sum(wl ** 2, axis=0)) + eps_w)
    ws = Ws.forward(X0).reshape(L, -1)
    beta = 1.0 / (np.sqrt(np.sum(ws ** 2, axis=1)) + eps_w)
    return alpha, beta


def ws_norm2_of(Ws, n: int) -> float:
    """||W_s||^2 of a spatial dictionary on n x n images."""
    return Ws.frame_norm2(n) if hasattr(Ws, "frame_norm2") else Ws.norm2


def lipschitz(K: np.ndarray, n: int, iters: int = 1000, tol: float = 1e-13,
              seed: int = 7) -> float:
    """beta_H = max_l lambda_max(H_l^T H_l), the Lipschitz constant of the
    gradient of the least-squares term (Section 2.2), by power iteration on
    every band with the Rayleigh quotient."""
    L = K.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((L, n, n))
    lam = np.zeros(L)
    for _ in range(iters):
        w = HT(H(v, K), K)
        new = np.sum(v * w, axis=(1, 2)) / np.sum(v * v, axis=(1, 2))
        v = w / np.sqrt(np.sum(w * w, axis=(1, 2)))[:, None, None]
        done = np.max(np.abs(new - lam) / np.abs(new)) <= tol
        lam = new
        if done:
            break
    return float(np.max(lam))


def tau_rule(beta_H, sigma, mu_l, gamma_n, rule="opnorm", rho=0.99, ws_norm2=1.0):
    """Primal step tau satisfying the convergence condition of Section 2.2;
    ||W_lambda|| = 1, ||W_s||^2 = ws_norm2 (1 for the union of orthonormal
    bases)."""
    if rule == "opnorm":
        k = ws_norm2 * np.max(mu_l ** 2) + np.max(gamma_n ** 2)
    elif rule == "sum":
        k = ws_norm2 * np.sum(mu_l ** 2) + np.sum(gamma_n ** 2)
    else:
        raise ValueError(rule)
    return rho / (beta_H / 2.0 + sigma * k)


# --------------------------------------------------------------------------
# one MUFFIN iteration (Algorithm 2)
# --------------------------------------------------------------------------


@dataclass
class State:
    X: np.ndarray
    U: np.ndarray
    V: np.ndarray
    T: np.ndarray

    @staticmethod
    def zeros(L, n, P):
        return State(np.zeros((L, n, n)), np.zeros((L, P, n, n)),
                     np.zeros((L, n, n)), np.zeros((L, n, n)))

    def copy(self):
        return State(self.X.copy(), self.U.copy(), self.V.copy(), self.T.copy())


@dataclass
class Problem:
    """Everything one solve keeps fixed.  With `vis` set (a visibility
    operator), Y holds the complex visibilities (L, K) and H is `vis`;
    otherwise Y is the dirty cube and H the convolution by the PSFs."""
    Y: np.ndarray          # (L, n, n) dirty cube, or (L, K) visibilities
    K: np.ndarray          # (L, 2n, 2n) PSF transfer functions (image domain)
    Ws: SpatialDictionary
    alpha: np.ndarray      # (N,)
    beta: np.ndarray       # (L,)
    sigma: float = 10.0
    vis: object = None
    n: int = 0

    @property
    def shape(self):
        L = self.Y.shape[0]
        n = self.n or self.Y.shape[-1]
        return (L, n, n)

    def fwd(self, x):
        """H x (eq. `model`)."""
        return self.vis.forward(x) if self.vis is not None else H(x, self.K)

    def adj(self, r):
        """(Re) H^T r."""
        return self.vis.adjoint(r) if self.vis is not None else HT(r, self.K)

    def mu_l(self, mu):
        return mu * self.beta                      # eq. `2regpar`

    def gamma_n(self, gamma):
        L, n, _ = self.shape
        return (gamma * self.alpha).reshape(n, n)  # eq. `2regpar`


def muffin_step(st: State, Y: np.ndarray, pb: Problem, mu: float, gamma: float,
                tau: float):
    """One iteration of Algorithm 2.  Returns the new state and the
    intermediates the derivative recursions need (m, p, v~, x, x~, the entering
    u and the new v)."""
    mu_l = pb.mu_l(mu)[:, None, None]
    gam = pb.gamma_n(gamma)[None]
    sig = pb.sigma
    x = st.X                                              # eq. updatenode2
    grad = pb.adj(pb.fwd(x) - Y)                          # eq. grad2
    s = mu_l * pb.Ws.adjoint(st.U)                        # eq. adjointspat2
    m = x - tau * (grad + s + st.T)                       # eq. stpm
    xt = pos(m)                                           # eq. stpx
    p = st.U + sig * mu_l[:, :, None] * pb.Ws.forward(2 * xt - x)  # eq. stpp
    u = sat(p)                                            # eq. stpu
    vt = st.V + sig * gam * Wl(2 * xt - x)                # eq. vt
    v = sat(vt)                                           # eq. v
    t = gam * WlT(v)                                      # eq. upt
    inter = dict(x=x, xt=xt, m=m, p=p, vt=vt, u_in=st.U, v_new=v)
    return State(xt, u, v, t), inter


def deriv_step_mu(d: State, it: dict, pb: Problem, mu: float, gamma: float,
                  tau: float) -> State:
    """One iteration of Algorithm 3 (d/dmu), driven by the intermediates `it`
    of the matching primal iteration."""
    beta = pb.beta[:, None, None]
    gam = pb.gamma_n(gamma)[None]
    alpha = pb.gamma_n(1.0)[None]
    sig = pb.sigma
    x_d = d.X
    grad_d = pb.adj(pb.fwd(x_d))
    s_d = mu * beta * pb.Ws.adjoint(d.U) + beta * pb.Ws.adjoint(it["u_in"])
    m_d = x_d - tau * (grad_d + s_d + d.T)
    xt_d = U_weak(it["m"]) * m_d
    p_d = d.U + sig * beta[:, :, None] * pb.Ws.forward(
        2 * it["xt"] - it["x"] + mu * (2 * xt_d - x_d))
    u_d = Pi_weak(it["p"]) * p_d
    vt_d = d.V + sig * gamma * alpha * Wl(2 * xt_d - x_d)
    v_d = Pi_weak(it["vt"]) * vt_d
    t_d = gam * WlT(v_d)
    return State(xt_d, u_d, v_d, t_d)


def deriv_step_gamma(d: State, it: dict, pb: Problem, mu: float, gamma: float,
                     tau: float) -> State:
    """One iteration of Algorithm 4 (d/dgamma)."""
    beta = pb.beta[:, None, None]
    alpha = pb.gamma_n(1.0)[None]
    sig = pb.sigma
    x_d = d.X
    grad_d = pb.adj(pb.fwd(x_d))
    s_d = mu * beta * pb.Ws.adjoint(d.U)
    m_d = x_d - tau * (grad_d + s_d + d.T)
    xt_d = U_weak(it["m"]) * m_d
    p_d = d.U + sig * mu * beta[:, :, None] * pb.Ws.forward(2 * xt_d - x_d)
    u_d = Pi_weak(it["p"]) * p_d
    vt_d = d.V + sig * alpha * Wl(2 * it["xt"] - it["x"] + gamma * (2 * xt_d - x_d))
    v_d = Pi_weak(it["vt"]) * vt_d
    t_d = gamma * alpha * WlT(v_d) + alpha * WlT(it["v_new"])
    return State(xt_d, u_d, v_d, t_d)


# --------------------------------------------------------------------------
# risk estimate and its gradient (Sections 3.1-3.2)
# --------------------------------------------------------------------------


def _rdot(a, b):
    """Real inner product (of complex data: the sum over real and imaginary
    parts)."""
    return float(np.sum(np.real(np.conj(a) * b)))


def _meas(Y):
    """Number of real measurements (complex data count twice)."""
    return Y.size * (2 if np.iscomplexobj(Y) else 1)


def psure(Y, X, Xbar, K, delta, sigma_w, eps, fwd=None):
    """PSURE-FDMC summed over bands (eqs. `PSURE`, `PSURE0`); fwd: the
    direct operator (default: the convolution by the PSFs of K)."""
    fwd = fwd or (lambda z: H(z, K))
    d = fwd(X)
    dbar = fwd(Xbar)
    return float(_rdot(Y - d, Y - d) - _meas(Y) * sigma_w ** 2
                 + sigma_w ** 2 * (2.0 / eps) * _rdot(dbar - d, delta))


def sugar(Y, X, Xd, Xbar_d, K, delta, sigma_w, eps, fwd=None):
    """SUGAR-FDMC summed over bands for one parameter (eq. `SUGAR`)."""
    fwd = fwd or (lambda z: H(z, K))
    d = fwd(X)
    dd = fwd(Xd)
    dbar_d = fwd(Xbar_d)
    return float(2.0 * _rdot(d - Y, dd)
                 + (2.0 * sigma_w ** 2 / eps) * _rdot(dbar_d - dd, delta))


# --------------------------------------------------------------------------
# drivers
# --------------------------------------------------------------------------


def run_muffin(pb: Problem, mu: float, gamma: float, tau: float, iters: int,
               state: State | None = None) -> State:
    """Plain MUFFIN (fixed theta): `iters` iterations of Algorithm 2."""
    L, n, _ = pb.shape
    st = state.copy() if state is not None else State.zeros(L, n, pb.Ws.P)
    for _ in range(iters):
        st, _ = muffin_step(st, pb.Y, pb, mu, gamma, tau)
    return st


@dataclass
class AdaptResult:
    X: np.ndarray
    Xbar: np.ndarray
    mu: float
    gamma: float
    tau: float
    history: list = field(default_factory=list)   # per theta update
    states: dict = field(default_factory=dict)


def run_adapt(pb: Problem, mu0: float, gamma0: float, iters: int, delta,
              eps: float, sigma_w: float, Delta: int = 10, eta_mu: float = 1e-3,
              eta_gamma: float = 1e-3, beta_H: float | None = None,
              tau: float | None = None, tau_mode: str = "opnorm",
              rho: float = 0.99, deriv_reset: bool = True) -> AdaptResult:
    """ADA-PT'ed MUFFIN (Algorithm 5): per iteration, Algorithm 2 on Y and on
    Ybar = Y + eps delta, Algorithms 3-4 for both; after every Delta completed
    iterations theta <- max(theta - eta * SUGAR, 0) (eq. `adaptgrad`).

    tau: if given, a fixed step used throughout; otherwise recomputed from
    beta_H with `tau_mode` at the start and after every theta update."""
    L, n, _ = pb.shape
    P = pb.Ws.P
    Ybar = pb.Y + eps * delta
    mu, gamma = float(mu0), float(gamma0)

    def cur_tau():
        if tau is not None:
            return float(tau)
        return float(tau_rule(beta_H, pb.sigma, pb.mu_l(mu),
                              pb.gamma_n(gamma).ravel(), tau_mode, rho,
                              ws_norm2_of(pb.Ws, pb.shape[-1])))

    t_now = cur_tau()
    S, Sb = State.zeros(L, n, P), State.zeros(L, n, P)
    Dm, Dg = State.zeros(L, n, P), State.zeros(L, n, P)
    Dbm, Dbg = State.zeros(L, n, P), State.zeros(L, n, P)
    hist = []
    for k in range(1, iters + 1):
        S_new, it = muffin_step(S, pb.Y, pb, mu, gamma, t_now)
        Sb_new, itb = muffin_step(Sb, Ybar, pb, mu, gamma, t_now)
        Dm = deriv_step_mu(Dm, it, pb, mu, gamma, t_now)
        Dg = deriv_step_gamma(Dg, it, pb, mu, gamma, t_now)
        Dbm = deriv_step_mu(Dbm, itb, pb, mu, gamma, t_now)
        Dbg = deriv_step_gamma(Dbg, itb, pb, mu, gamma, t_now)
        S, Sb = S_new, Sb_new
        if k % Delta == 0:
            g_mu = sugar(pb.Y, S.X, Dm.X, Dbm.X, pb.K, delta, sigma_w, eps, pb.fwd)
            g_ga = sugar(pb.Y, S.X, Dg.X, Dbg.X, pb.K, delta, sigma_w, eps, pb.fwd)
            r = psure(pb.Y, S.X, Sb.X, pb.K, delta, sigma_w, eps, pb.fwd)
            mu = max(mu - eta_mu * g_mu, 0.0)
            gamma = max(gamma - eta_gamma * g_ga, 0.0)
            t_now = cur_tau()
            hist.append(dict(k=k, sugar_mu=g_mu, sugar_gamma=g_ga, psure=r,
                             mu=mu, gamma=gamma, tau=t_now))
            if deriv_reset:
                Dm, Dg = State.zeros(L, n, P), State.zeros(L, n, P)
                Dbm, Dbg = State.zeros(L, n, P), State.zeros(L, n, P)
    return AdaptResult(X=S.X, Xbar=Sb.X, mu=mu, gamma=gamma, tau=t_now,
                       history=hist,
                       states=dict(S=S, Sb=Sb, Dm=Dm, Dg=Dg, Dbm=Dbm, Dbg=Dbg))


def objective(X, pb: Problem, mu: float, gamma: float) -> float:
    """F(X) of eq. `probopt` with h(X) of eq. `RegAll` (inf if X has a
    negative entry)."""
    if np.any(X < 0):
        return np.inf
    L, n, _ = X.shape
    r = pb.Y - pb.fwd(X)
    data = 0.5 * _rdot(r, r)
    spat = np.sum(pb.mu_l(mu) * np.sum(np.abs(pb.Ws.forward(X)).reshape(L, -1), axis=1))
    spec = np.sum(pb.gamma_n(gamma).ravel()
                  * np.sum(np.abs(Wl(X)).reshape(L, -1), axis=0))
    return float(data + spat + spec)


def quality(X: np.ndarray, truth: np.ndarray, K: np.ndarray) -> tuple[float, float]:
    """SNR (dB) and WMSE of an estimate X of the sky `truth` (Section 4.1):
    SNR = 10 log10(sum_l |x*_l|^2 / sum_l |x*_l - x_l|^2) and
    WMSE = (1 / (N L)) sum_l |H_l (x*_l - x_l)|^2, N pixels per band."""
    L, n, _ = truth.shape
    err = truth - X
    snr = 10.0 * np.log10(np.sum(truth ** 2) / np.sum(err ** 2))
    wmse = float(np.sum(H(err, K) ** 2)) / (n * n * L)
    return float(snr), wmse


def make_vis_problem(vis, uv, n, P=8, J=3, sigma=10.0, alpha=None, beta=None,
                     eps_w=1e-6, dictionary="daubechies") -> Problem:
    """A Problem whose data are visibilities (L, K) at the sample positions
    uv (L, K, 2) of an n x n cube (the visibility-domain operator of
    oracle.visibility).  Weights default to the rule of Section 2.1 with the
    back-projected (dirty) cube Re H^* v as the initial estimate."""
    from .visibility import VisibilityOperator
    op = VisibilityOperator(uv, n)
    Ws = SpatialDictionary(P, J) if dictionary == "daubechies" else StarletDictionary(J)
    if alpha is None or beta is None:
        a, b = weights(op.adjoint(vis), Ws, eps_w)
        alpha = a if alpha is None else alpha
        beta = b if beta is None else beta
    L = vis.shape[0]
    return Problem(Y=np.asarray(vis, np.complex128), K=np.zeros((L, 1, 1)), Ws=Ws,
                   alpha=np.asarray(alpha, np.float64), beta=np.asarray(beta, np.float64),
                   sigma=sigma, vis=op, n=n)


def lipschitz_op(pb: Problem, iters: int = 1000, tol: float = 1e-13, seed: int = 7) -> float:
    """beta_H for any direct operator: max over bands of lambda_max(H^T H)
    by power iteration with the Rayleigh quotient."""
    L, n, _ = pb.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((L, n, n))
    lam = np.zeros(L)
    for _ in range(iters):
        w = pb.adj(pb.fwd(v))
        new = np.sum(v * w, axis=(1, 2)) / np.sum(v * v, axis=(1, 2))
        v = w / np.sqrt(np.sum(w * w, axis=(1, 2)))[:, None, None]
        done = np.max(np.abs(new - lam) / np.abs(new)) <= tol
        lam = new
        if done:
            break
    return float(np.max(lam))


def make_problem(dirty, psf, P=8, J=3, sigma=10.0, alpha=None, beta=None,
                 eps_w=1e-6, dictionary="daubechies") -> Problem:
    """Assemble a Problem; weights default to the rule of Section 2.1 with
    the dirty cube as the initial estimate.  dictionary: "daubechies" (the
    union of db1..dbP, J levels) or "starlet" (the IUWT with J scales)."""
    K = psf_spectrum(psf)
    Ws = SpatialDictionary(P, J) if dictionary == "daubechies" else StarletDictionary(J)
    if alpha is None or beta is None:
        a, b = weights(dirty, Ws, eps_w)
        alpha = a if alpha is None else alpha
        beta = b if beta is None else beta
    return Problem(Y=np.asarray(dirty, np.float64), K=K, Ws=Ws,
                   alpha=np.asarray(alpha, np.float64),
                   beta=np.asarray(beta, np.float64), sigma=sigma)
