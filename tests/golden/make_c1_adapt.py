"""Writes c1_adapt_30.json: the FP64 oracle's ADA-PT run on the 256 x 256 x 64
workload (PSF 512 x 512; 200 point sources, 10 blobs, 4000 baselines; seed 0),
30 iterations with a theta update every 10 (three windows of Algorithm 5).

The oracle needs about 3.5 minutes per ADA-PT iteration at this size, so the
GPU parity test reads the stored result instead of running the oracle.  The
file holds the theta history (eq. `adaptgrad`, PSURE of eq. `PSURE0`, SUGAR
of eq. `SUGAR`), the L2 norm of every band of X for each of the six state
sets (both trajectories and their four derivatives, Algs. 3-4), and X at a
fixed sample of voxels of every set.

Only the oracle and the seeded generator are called.  Run from the
repository root:  python tests/golden/make_c1_adapt.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import muffin as om  # noqa: E402

# The run's parameters; the GPU test reads them from the file.
PARAMS = dict(config="c1", seed=0, P=8, J=3, mu0=1.0, gamma0=1.0, iters=30, Delta=10,
              eta_mu=5e-3, eta_gamma=2e-4, eps_over_sigma_w=0.05, sigma=10.0,
              deriv_reset=True, samples=512, sample_seed=77)


def safe_tau(psf, sigma, mu_l, gamma_n, rho=0.9):
    """Fixed primal step from the l1 norm of the PSFs (a bound on ||H_l||),
    valid for theta up to twice its start in both parameters."""
    bound = max(np.abs(psf[l]).sum() for l in range(psf.shape[0])) ** 2
    return rho / (bound / 2 + sigma * (np.max(mu_l) ** 2 + np.max(gamma_n) ** 2))


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_adapt_30.json")):
    p = PARAMS
    prob = synth.make_config(p["config"], seed=p["seed"])
    L, n = prob.L, prob.n
    pb = om.make_problem(prob.dirty, prob.psf, P=p["P"], J=p["J"], sigma=p["sigma"])
    tau = safe_tau(prob.psf, p["sigma"], 2 * p["mu0"] * pb.beta, 2 * p["gamma0"] * pb.alpha)
    eps = p["eps_over_sigma_w"] * prob.sigma_w
    t0 = time.time()
    res = om.run_adapt(pb, p["mu0"], p["gamma0"], p["iters"], prob.delta, eps, prob.sigma_w,
                       Delta=p["Delta"], eta_mu=p["eta_mu"], eta_gamma=p["eta_gamma"],
                       tau=tau, deriv_reset=p["deriv_reset"])
    rng = np.random.Generator(np.random.PCG64(p["sample_seed"]))
    idx = np.sort(rng.choice(L * n * n, size=p["samples"], replace=False))
    sets = {}
    for name in ("S", "Sb", "Dm", "Dg", "Dbm", "Dbg"):
        X = res.states[name].X
        sets[name] = dict(band_norms=[float(v) for v in np.sqrt(np.sum(X ** 2, axis=(1, 2)))],
                          samples=[float(v) for v in X.ravel()[idx]])
    doc = dict(
        description="FP64 oracle ADA-PT run (Algorithm 5) on the 256x256x64 workload; "
                    "written by tests/golden/make_c1_adapt.py",
        params=p, tau=float(tau), eps=float(eps), sigma_w=float(prob.sigma_w),
        alpha_sum=float(pb.alpha.sum()), beta=[float(v) for v in pb.beta],
        history=res.history, final=dict(mu=res.mu, gamma=res.gamma),
        sample_index=[int(i) for i in idx], sets=sets,
        oracle_seconds=round(time.time() - t0, 1))
    with open(out, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {out} ({doc['oracle_seconds']} s)")


if __name__ == "__main__":
    main()
