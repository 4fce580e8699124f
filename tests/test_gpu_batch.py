"""Batching (muffin_batch_*): cubes of different sizes and forms iterated
together through one captured graph per chunk.  Every replay is checked
against the same handles run eagerly (with eager work and synchronisation
between the replays), bit for bit, including the theta history of the
adaptive ones."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _mm():
    from paper_1905_08468_amd import muffin as mm
    return mm


def _make(mm, spec, stream):
    import torch
    n, L, mode, sure, Delta, seed = spec
    dt = torch.float64 if mode == mm.F64 else torch.float32
    p = synth.make_problem(n, L, seed=seed, **synth.scaled_counts(64))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dt)
    cfg = mm.default_config(n, L, mode=mode, sure=sure, delta_period=Delta, pi_iters=30,
                            eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w,
                            eta_mu=1e-4, eta_gamma=1e-4)
    torch.cuda.synchronize()
    h = mm.Muffin(cfg, stream=stream)
    h.set_problem(d(p.dirty), d(p.psf), None, None, d(p.delta) if sure else None)
    return h


SPECS = [(32, 4, 0, 1, 3, 80), (64, 8, 1, 0, 10, 81), (16, 3, 2, 1, 2, 82),
         (128, 2, 1, 0, 10, 83)]


def test_batch_graph_replays_equal_eager_runs():
    mm = _mm()
    import torch
    specs = [(n, L, [mm.F64, mm.F32, mm.F32_BF16DCT][m], s, D, seed)
             for n, L, m, s, D, seed in SPECS]
    batch_h = [_make(mm, sp, torch.cuda.Stream()) for sp in specs]
    eager_h = [_make(mm, sp, torch.cuda.Stream()) for sp in specs]
    b = mm.Batch(batch_h)                 # chunk = lcm(2, 3, 2) = 6
    chunk = 6
    for rnd in range(4):
        b.run(1)                          # round 0 runs eagerly and records the graph
        b.synchronize()
        for he in eager_h:
            he.run(chunk)
        for hb, he in zip(batch_h, eager_h):
            assert np.array_equal(hb.sky().cpu().numpy(), he.sky().cpu().numpy()), rnd
            rb, re = hb.report(), he.report()
            assert rb["iters_done"] == re["iters_done"] == chunk * (rnd + 1)
            assert rb["theta_updates"] == re["theta_updates"]
            if hb.cfg.sure:
                assert np.array_equal(hb.history(), he.history())
                assert np.array_equal(hb.get_state(1, 3).cpu().numpy(),
                                      he.get_state(1, 3).cpu().numpy())
    b.run(3)                              # several launches in one call
    b.synchronize()
    for he in eager_h:
        he.run(3 * chunk)
    for hb, he in zip(batch_h, eager_h):
        assert np.array_equal(hb.sky().cpu().numpy(), he.sky().cpu().numpy())
    b.close()
    for h in batch_h + eager_h:
        h.close()


def test_batch_rejects_bad_setups():
    mm = _mm()
    import torch
    s = torch.cuda.Stream()
    h1 = _make(mm, (32, 2, mm.F32, 1, 3, 90), s)
    with pytest.raises(mm.MuffinError) as e:     # chunk not a multiple of Delta
        mm.Batch([h1], chunk=4)
    assert e.value.code == -1
    h1.run(2)                                    # not at a multiple of the chunk
    with pytest.raises(mm.MuffinError) as e:
        mm.Batch([h1])
    assert e.value.code == -6
    h1.close()
