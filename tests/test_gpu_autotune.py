"""Autotuner of the level-1 wavelet tile shapes (muffin_autotune): both
shapes are timed, the choice is recorded per size class and reused, and a
tuned handle computes exactly what an untuned one does (the tile shape does
not change any output's arithmetic)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _mm():
    from paper_1905_08468_amd import muffin as mm
    return mm


def _run(mm, cfg, p, tune, iters=6):
    import torch
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", torch.float32)
    h = mm.Muffin(cfg)
    res = h.autotune(2) if tune else None
    h.set_problem(d(p.dirty), d(p.psf), None, None, d(p.delta))
    h.run(iters)
    out = h.sky().cpu().numpy(), h.get_state(1, 2).cpu().numpy(), h.history()
    h.close()
    return res, out


@pytest.mark.parametrize("n,L", [(64, 8), (128, 6)])
def test_tuned_equals_untuned_and_is_recorded(n, L):
    mm = _mm()
    p = synth.make_problem(n, L, seed=n + L, **synth.scaled_counts(n))
    cfg = mm.default_config(n, L, mode=mm.F32, sure=1, delta_period=3, pi_iters=20,
                            eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w, eta_mu=1e-4,
                            eta_gamma=1e-4)
    res, tuned = _run(mm, cfg, p, True)
    assert res["tunable"] == 1 and res["cached"] == 0
    assert res["syn_tile1"] in (16, 32) and res["an_tile1"] in (16, 32)
    assert min(res["syn_ms"]) > 0 and min(res["an_ms"]) > 0
    _, plain = _run(mm, cfg, p, False)
    for a, b in zip(tuned, plain):
        assert np.array_equal(a, b)
    res2, again = _run(mm, cfg, p, True)
    assert res2["cached"] == 1
    assert (res2["syn_tile1"], res2["an_tile1"]) == (res["syn_tile1"], res["an_tile1"])
    for a, b in zip(again, plain):
        assert np.array_equal(a, b)


def test_untunable_and_out_of_order():
    mm = _mm()
    import torch
    h = mm.Muffin(mm.default_config(32, 2, mode=mm.F64))
    r = h.autotune(1)
    assert r["tunable"] == 0 and r["syn_tile1"] == 16
    h.close()
    h = mm.Muffin(mm.default_config(32, 2, mode=mm.F32, pi_iters=10))
    z = torch.zeros((2, 32, 32), device="cuda:0")
    zp = torch.zeros((2, 64, 64), device="cuda:0")
    zp[:, 32, 32] = 1
    h.set_problem(z, zp)
    with pytest.raises(mm.MuffinError) as e:
        h.autotune(1)
    assert e.value.code == -6
    h.close()
