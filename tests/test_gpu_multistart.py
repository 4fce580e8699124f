"""Multi-start ADA-PT (muffin_multistart_*) and the quality measures
(muffin_quality, Section 4.1).  Every start of a multi-start run must equal
a lone run of its configuration bit for bit, the FP64 path must follow the
oracle's ADA-PT from the same start, and SNR/WMSE must match the oracle's
on the same estimate."""
import numpy as np
import pytest

import synth
from oracle import muffin as om

pytestmark = pytest.mark.gpu


def _mm():
    from paper_1905_08468_amd import muffin as mm
    return mm


def _problem(n, L, seed):
    return synth.make_problem(n, L, seed=seed, **synth.scaled_counts(64))


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dt)


def _cfg(mm, p, mode, Delta=4, **over):
    return mm.default_config(p.sky.shape[1], p.sky.shape[0], mode=mode, sure=1,
                             delta_period=Delta, eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w,
                             eta_mu=0.02, eta_gamma=0.02, pi_iters=60, **over)


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_quality_matches_oracle(mode):
    mm = _mm()
    import torch
    p = _problem(32, 4, 31)
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    h = mm.Muffin(mm.default_config(32, 4, mode=m, pi_iters=60))
    h.set_problem(_dev(p.dirty, dt), _dev(p.psf, dt))
    h.run(15)
    x = h.sky().double().cpu().numpy()
    snr, wmse = h.quality(_dev(p.sky, dt))
    # the oracle sees the cubes as the device holds them
    npdt = np.float64 if mode == "f64" else np.float32
    K = om.psf_spectrum(p.psf.astype(npdt).astype(np.float64))
    truth = p.sky.astype(npdt).astype(np.float64)
    r_snr, r_wmse = om.quality(x, truth, K)
    tol = 1e-10 if mode == "f64" else 1e-5
    assert abs(snr - r_snr) <= tol * abs(r_snr)
    assert abs(wmse - r_wmse) <= tol * r_wmse
    # the sky itself: infinite SNR, zero WMSE
    s_inf, w0 = h.quality(h.sky())
    assert s_inf == float("inf") and w0 == 0.0
    h.close()


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_multistart_equals_lone_runs(mode):
    mm = _mm()
    import torch
    p = _problem(32, 4, 32)
    m = mm.F64 if mode == "f64" else mm.F32
    dt = torch.float64 if mode == "f64" else torch.float32
    cfg = _cfg(mm, p, m)
    dirty, psf, delta, truth = (_dev(a, dt) for a in (p.dirty, p.psf, p.delta, p.sky))
    ms = mm.MultiStart(cfg)                       # the four couples of Section 4.2
    ms.set_problem(dirty, psf, delta=delta)
    assert ms.chunk == 4
    ms.run(2)                                     # first call records the graph
    ms.run(3)                                     # then graph launches
    snr, wmse = ms.quality(truth)
    for i, (mu0, ga0) in enumerate(mm.MultiStart.PAPER_STARTS):
        c = _cfg(mm, p, m, mu=mu0, gamma=ga0)
        h = mm.Muffin(c)
        h.set_problem(dirty, psf, None, None, delta)
        rep = h.run(20)
        v = ms.start(i)
        assert np.array_equal(v.sky().cpu().numpy(), h.sky().cpu().numpy()), i
        assert np.array_equal(v.history(), h.history()), i
        rv = v.report()
        for k in ("iters_done", "theta_updates", "mu", "gamma", "tau", "beta_H", "psure"):
            assert rv[k] == rep[k], (i, k)
        s1, w1 = h.quality(truth)
        assert s1 == snr[i] and w1 == wmse[i]
        h.close()
    hist = [ms.start(i).history() for i in range(4)]
    assert all(len(hh) == 5 for hh in hist)
    ms.close()


def test_multistart_start_follows_oracle_adapt():
    mm = _mm()
    import torch
    p = _problem(32, 4, 33)
    starts = [(1.0, 3.0), (0.005, 10.0)]
    cfg = _cfg(mm, p, mm.F64)
    ms = mm.MultiStart(cfg, starts=starts)
    dt = torch.float64
    ms.set_problem(_dev(p.dirty, dt), _dev(p.psf, dt), delta=_dev(p.delta, dt))
    ms.run(3)
    a, b = ms.start(0).weights()
    beta_H = ms.start(0).report()["beta_H"]
    pb = om.make_problem(p.dirty, p.psf, P=8, J=cfg.levels, alpha=a, beta=b)
    for i, (mu0, ga0) in enumerate(starts):
        ref = om.run_adapt(pb, mu0, ga0, 12, p.delta, cfg.eps_fd, cfg.sigma_w, Delta=4,
                           eta_mu=cfg.eta_mu, eta_gamma=cfg.eta_gamma, beta_H=beta_H)
        x = ms.start(i).sky().cpu().numpy()
        assert np.linalg.norm(x - ref.X) <= 1e-10 * np.linalg.norm(ref.X)
        hist = ms.start(i).history()
        for row, r in zip(hist, ref.history):
            assert row[0] == r["k"]
            for col, key in ((1, "mu"), (2, "gamma"), (4, "sugar_mu"), (5, "sugar_gamma")):
                assert abs(row[col] - r[key]) <= 1e-9 * max(1.0, abs(r[key])), (i, key)
    ms.close()


def test_multistart_rejects_bad_setups():
    mm = _mm()
    import torch
    p = _problem(16, 2, 34)
    cfg = _cfg(mm, p, mm.F32)
    with pytest.raises(mm.MuffinError) as e:
        mm.MultiStart(cfg, starts=[])
    assert e.value.code == -1
    with pytest.raises(mm.MuffinError) as e:
        mm.MultiStart(cfg, starts=[(1.0, -1.0)])
    assert e.value.code == -1
    ms = mm.MultiStart(cfg, starts=[(1.0, 1.0), (0.5, 2.0)])
    with pytest.raises(mm.MuffinError) as e:       # no problem set yet
        ms.run(1)
    assert e.value.code == -6
    assert mm._lib.muffin_multistart_handle(ms.h, 2) is None
    dt = torch.float32
    with pytest.raises(mm.MuffinError) as e:       # chunk not a multiple of Delta
        ms.set_problem(_dev(p.dirty, dt), _dev(p.psf, dt), delta=_dev(p.delta, dt), chunk=6)
    assert e.value.code == -1
    ms.set_problem(_dev(p.dirty, dt), _dev(p.psf, dt), delta=_dev(p.delta, dt), chunk=8)
    ms.run(1)
    assert ms.start(1).report()["iters_done"] == 8
    ms.close()
