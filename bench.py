"""Benchmark: ADA-PT'ed MUFFIN iterations/s at 1024^2 x 256 bands on one GPU.

One step = one iteration of the whole hot path (Algorithm 5): Algorithm 2 on
Y and on Ybar = Y + eps delta, the derivative recursions of Algorithms 3-4
for both, and every Delta = 10 steps the SUGAR reduction and theta update.
Inputs are synthetic (seeded generator, 20000 point sources + 200 blobs,
PSFs from 50000 gridded baselines, 20 dB SNR), resident in HBM before the
timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode f32|bf16|f64]
                  [--workload c2|c1|c0] [--no-fp64] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "primal-dual iters/s at 1024²×256 bands (FP32 vs FP64); served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK, MFMA_F32_PEAK, MFMA_F64_PEAK = 2500.0, 157.3, 78.6   # TFLOP/s, dense

# Algorithmic traffic of the single-launch stages of one ADA-PT iteration,
# per voxel (all state sets of the launch together): (working-precision
# values, mask bytes).  Each input and output array is counted once.
#   synthesis_l1: per set the 6 level-1 detail coefficients of the 8 bases
#     (8 x 3/4) + the 2 coarse values (8 x 1/4) in, S out.  6 sets: 6*9.
#   primal_step: per trajectory x, G, H^T y, S, T in, x~ and z = 2 x~ - x
#     out; each derivative x', G', S', T' in, x~', z' out.  2 trajectories:
#     2*(7+6+6).
#   analysis_l1_primal: per set z in; 6 detail coefficients read and
#     written; 2 low-pass values out; the masks of the 8 bases' outputs as
#     bits, one 32-bit word per thread of a 64 x 64 tile (1 byte per
#     voxel) out.  2 sets: 2*(1+12+2).
#   analysis_l1_deriv: as above with the mask words read; the d/dmu sets
#     read the primal's z too.  4 sets: 2*(2+12+2) + 2*(1+12+2), 4 mask
#     bytes.
#   dct_primal: z, V in; V, T out; the masks as bits, one 32-bit word per
#     thread of a 64-pixel x 256-band block (1/8 byte per voxel).  2 sets.
#   dct_deriv: d/dmu: z', V' in, V', T' out; d/dgamma also z and the new
#     primal V.  4 sets: 2*4 + 2*6, 1/2 mask byte.
# FMAs of the level-1 wavelet launches as the kernels issue them (separable
# filters of the Daubechies union p = 1..8, 2p taps, halo columns included):
#   synthesis (32 x 32 coefficient tiles, 512 threads): per block and basis p
#     312 column items x 8 output pairs x 4p + 512 threads x 4 pairs x 4p;
#   analysis (64 x 64 input tiles, 1024 threads): per block and basis p
#     (62 + 2p) rows x 8 items x 16p (row filter) + 1024 threads x 8p.
def wavelet_fmas(stage, n, L, sets):
    if stage == "synthesis_l1":
        blocks = (n // 64) ** 2 * L * sets
        return blocks * sum((312 * 32 + 512 * 16) * p for p in range(1, 9))
    if stage.startswith("analysis_l1"):
        blocks = (n // 64) ** 2 * L * sets
        return blocks * sum((62 + 2 * p) * 8 * 16 * p + 1024 * 8 * p for p in range(1, 9))
    return None


FP32_VECTOR_PEAK, FP32_VECTOR_UNPACKED = 157.3, 78.6   # TFLOP/s (packed FP32 is not used)


def fft_chain_flops(n, L, sets):
    """Nominal flops of the FFT chain: H^T H is four real 2-D transforms of
    the (2n)^2 grid per band and set, counted as 2.5 M log2 M for M = 4 n^2
    points (the radix-2 count of a real transform of M points; the pruned
    passes compute fewer)."""
    import math
    M = 4 * n * n
    return sets * L * 4 * 2.5 * M * math.log2(M)

STAGE_TRAFFIC = {
    # the five launches of the FFT chain (H^T H of every set): the first
    # row pass reads the image (1 V) and writes the half spectrum (2 V); the
    # column passes read and write it (2 + 2 V) and read the transfer
    # function once for all sets (4 V); the middle row pass reads and writes
    # spectra (2 + 2 V); the last reads the spectrum and writes the image
    # (2 + 1 V).  6 sets: 18, 28, 24, 28, 18 V (116 V per chain).
    "fft_row1": (18, 0),
    "fft_col1": (28, 0),
    "fft_row2": (24, 0),
    "fft_col2": (28, 0),
    "fft_row3": (18, 0),
    "synthesis_l1": (54, 0),
    "analysis_l1_primal": (30, 2),
    "analysis_l1_deriv": (62, 4),
    "dct_primal": (8, 0.25),
    "dct_deriv": (20, 0.5),
    "primal_step": (38, 0),
}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (profiles/*_traffic.md: FETCH_SIZE and WRITE_SIZE passes scaled by a
    plain streaming kernel of known size), or None when there is none or when
    the kernel's sources have changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        rec = {}
        for line in open(path):
            k, sep, v = line.strip().partition(": ")
            if sep and k in ("kernel", "traffic_bytes_per_launch", "sources", "sources_sha256"):
                rec[k] = v.strip()
        if rec.get("kernel") != kernel or len(rec) != 4:
            continue
        srcs, shas = rec["sources"].split(), rec["sources_sha256"].split()
        try:
            now = [hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest()
                   for f in srcs]
        except OSError:
            return None
        if now != shas:
            return None
        return int(rec["traffic_bytes_per_launch"])
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="bf16", choices=["f32", "bf16", "f64"])
    ap.add_argument("--workload", default="c2", choices=["c0", "c1", "c2"])
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB device copy (traffic-counter calibration)")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-cubes", type=int, default=48)
    ap.add_argument("--batch-chunks", type=int, default=3)
    ap.add_argument("--no-multistart", action="store_true")
    ap.add_argument("--ms-iters", type=int, default=200)
    ap.add_argument("--ms-trace", type=int, default=0,
                    help="record the multi-start curves every this many iterations "
                         "(over --ms-iters iterations) instead of timing")
    ap.add_argument("--no-unmix", action="store_true")
    ap.add_argument("--no-starlet", action="store_true")
    ap.add_argument("--no-vis", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-sweep", default="",
                    help="comma-separated further arrival rates (req/s) replayed after "
                         "--serve-rate with the same requests")
    return ap.parse_args()


def _oracle_band_step(args):
    """Worker: `iters` iterations of the FP64 oracle on one band's images
    (ADA-PT when `adapt`, else plain MUFFIN), the band's own time in s."""
    dirty, psf, delta, sigma_w, adapt, iters = args
    import numpy as np
    from oracle import muffin as om
    n = dirty.shape[-1]
    pb = om.make_problem(dirty[None], psf[None], P=8, J=3, alpha=np.ones(n * n),
                         beta=np.ones(1))
    t0 = time.perf_counter()
    if adapt:
        om.run_adapt(pb, 1.0, 1.0, iters, delta[None], 0.01 * sigma_w, sigma_w, Delta=10,
                     tau=1e-4)
    else:
        om.run_muffin(pb, 1.0, 1.0, 1e-4, iters)
    return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_warm(_):
    import numpy  # noqa: F401
    from oracle import muffin  # noqa: F401
    return os.getpid()


def cpu_baseline(prob, synth, workers=None):
    """The FP64 oracle, as it stands (numpy, one thread per process), on
    bounded samples, with one band per worker process on the host's cores:
      - the benchmark workload: one ADA-PT iteration of as many 1024^2 bands
        as there are workers, all at once; the per-band work (FFT
        convolutions, wavelet transforms) dominates the oracle's iteration,
        so the cube's rate is the sample's scaled by L / bands;
      - 256^2 x 64 (ADA-PT): one iteration of `workers` bands, scaled;
      - 64^2 x 8 (plain MUFFIN): 20 iterations of the whole cube in one
        process (the oracle's own band loop).
    Worker processes are started fresh (spawn) with one BLAS thread each."""
    import multiprocessing as mp
    import numpy as np
    from oracle import muffin as om
    ncpu = os.cpu_count() or 1
    workers = workers or max(1, min(16, ncpu, prob.L))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                             "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers) as pool:
            pool.map(_oracle_warm, range(workers))
            jobs = [(prob.dirty[b], prob.psf[b], prob.delta[b], prob.sigma_w, True, 1)
                    for b in range(workers)]
            t0 = time.perf_counter()
            per_band = pool.map(_oracle_band_step, jobs)
            wall = time.perf_counter() - t0
            p1 = synth.make_config("c1", seed=0)
            jobs = [(p1.dirty[b], p1.psf[b], p1.delta[b], p1.sigma_w, True, 1)
                    for b in range(min(workers, p1.L))]
            t0 = time.perf_counter()
            pool.map(_oracle_band_step, jobs)
            wall1 = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    p0 = synth.make_config("c0", seed=0)
    pb0 = om.make_problem(p0.dirty, p0.psf, P=8, J=3)
    t0 = time.perf_counter()
    om.run_muffin(pb0, 1.0, 1.0, 1e-3, 20)
    t_c0 = (time.perf_counter() - t0) / 20
    per_iter = wall * prob.L / workers
    nb1 = min(workers, p1.L)
    return {"value": 1.0 / per_iter, "unit": "iters/s", "cores": workers, "kind": "oracle",
            "sample": f"1 ADA-PT iteration (Alg. 5) of the FP64 numpy oracle on {workers} of "
                      f"{prob.L} bands of {prob.n}x{prob.n} px, one band per process on "
                      f"{workers} cores at once ({wall:.1f} s wall; single band "
                      f"{np.mean(per_band):.1f} s), scaled x{prob.L / workers:g}",
            "cpu": _cpu_model(), "host_threads": ncpu,
            "other_workloads": {
                "adapt_256x256x64": {"value": 1.0 / (wall1 * p1.L / nb1), "unit": "iters/s",
                                     "sample": f"1 ADA-PT iteration on {nb1} of {p1.L} bands "
                                               f"at once ({wall1:.1f} s), scaled "
                                               f"x{p1.L / nb1:g}"},
                "plain_64x64x8": {"value": 1.0 / t_c0, "unit": "iters/s",
                                  "sample": "20 plain MUFFIN iterations of the whole cube, "
                                            "one process"}}}


def _class_inputs(synth, torch, n, L, seed, dtype):
    import numpy as np
    p = synth.make_problem(n, L, seed=seed, device="cuda:0", **synth.scaled_counts(n))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype)
    return p, d(p.dirty), d(p.psf), d(p.delta)


def batch_form(mm, torch, synth, n_cubes, chunks, seed=7):
    """Batching form: independent cubes with sizes drawn (seeded) from
    {128, 256, 512}^2 px x {16, 32, 64, 128} bands, FP32, ADA-PT (Delta = 10),
    iterated together as one captured graph per chunk of 10 iterations; the
    same cubes are then run one after the other for comparison."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = [(int(rng.choice([128, 256, 512])), int(rng.choice([16, 32, 64, 128])))
             for _ in range(n_cubes)]
    inputs = {}
    for n, L in sorted(set(sizes)):
        inputs[(n, L)] = _class_inputs(synth, torch, n, L, 1000 + n + L, torch.float32)
    torch.cuda.synchronize()
    hs = []
    tuned = {}
    t0 = time.perf_counter()
    for n, L in sizes:
        p, d, ps, dl = inputs[(n, L)]
        cfg = mm.default_config(n, L, mode=mm.F32, sure=1, delta_period=10,
                                eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w, eta_mu=1e-6,
                                eta_gamma=1e-6, pi_iters=30, pi_tol=1e-4)
        h = mm.Muffin(cfg, stream=torch.cuda.Stream())
        # tile shapes per size class (timed once per class, then recorded)
        r = h.autotune(3)
        tuned[f"{n}x{L}"] = [r["syn_tile1"], r["an_tile1"]]
        h.set_problem(d, ps, None, None, dl)
        hs.append(h)
    setup_s = time.perf_counter() - t0
    vox = sum(n * n * L for n, L in sizes)
    b = mm.Batch(hs, chunk=10)
    b.run(1)                                   # eager chunk + graph capture
    b.synchronize()
    t0 = time.perf_counter()
    b.run(chunks)
    b.synchronize()
    tb = time.perf_counter() - t0
    iters = 10 * chunks
    t0 = time.perf_counter()
    for h in hs:
        h.run(10, report=False)
        h.stream.synchronize()
    ts = (time.perf_counter() - t0) * chunks   # one chunk each, scaled
    b.close()
    for h in hs:
        h.close()
    del inputs
    torch.cuda.empty_cache()
    return {"form": "ADA-PT, FP32, independent cubes as one captured graph per 10 iterations",
            "cubes": n_cubes, "sizes": "n in {128,256,512}, L in {16,32,64,128} (seeded draw)",
            "voxels": vox, "iterations_timed": iters,
            "cube_iters_per_s": round(n_cubes * iters / tb, 2),
            "voxel_updates_per_s": round(vox * iters / tb, 1),
            "ms_per_chunk": round(1e3 * tb / chunks, 2),
            "one_after_another_cube_iters_per_s": round(n_cubes * iters / ts, 2),
            "speedup_vs_one_after_another": round(ts / tb, 3), "setup_s": round(setup_s, 2),
            "tile_shapes": tuned}


def multistart_form(mm, torch, synth, iters, seed=0, eta_mu=5e-3, eta_gamma=1e-3,
                    trace_every=0):
    """Multi-start ADA-PT: the 256^2 px x 64 band cube (PSF 512^2) from the
    four initial couples (mu, gamma) of Section 4.2, FP32, Delta = 10, as one
    batch (one graph launch per 10 iterations of all four starts); then the
    same four starts one after the other.  theta, SNR and WMSE of each start
    after the timed iterations.  trace_every > 0: instead, run `iters`
    iterations untimed and record theta, SUGAR, SNR and WMSE of every start
    each trace_every iterations (the curves of Section 4.2)."""
    p = synth.make_config("c1", seed=seed, device="cuda:0")
    d = lambda a: torch.from_numpy(a).to("cuda:0", torch.float32)
    dirty, psf, delta, truth = d(p.dirty), d(p.psf), d(p.delta), d(p.sky)
    cfg = mm.default_config(p.n, p.L, mode=mm.F32, sure=1, delta_period=10,
                            eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w, eta_mu=eta_mu,
                            eta_gamma=eta_gamma, pi_iters=100)
    chunks = max(1, iters // 10)
    ms = mm.MultiStart(cfg)
    ms.set_problem(dirty, psf, delta=delta)
    if trace_every > 0:
        rows = [[] for _ in ms.starts]
        t0 = time.perf_counter()
        for k in range(trace_every, iters + 1, trace_every):
            ms.run(trace_every // 10)
            snr, wmse = ms.quality(truth)
            for i in range(len(ms.starts)):
                h = ms.start(i).history()[-1]
                rows[i].append([k, round(h[1], 5), round(h[2], 5), float(f"{h[4]:.4g}"),
                                float(f"{h[5]:.4g}"), round(float(snr[i]), 3),
                                float(f"{wmse[i]:.4g}")])
            log(f"[bench] multi-start trace k={k}: gamma "
                + " ".join(f"{r[-1][2]:.3f}" for r in rows) + " snr "
                + " ".join(f"{r[-1][5]:.2f}" for r in rows))
        el = time.perf_counter() - t0
        ms.close()
        return {"form": "multi-start trace, ADA-PT FP32 256x256 px x 64 bands",
                "eta": [eta_mu, eta_gamma], "iterations": iters, "seconds": round(el, 2),
                "columns": ["k", "mu", "gamma", "sugar_mu", "sugar_gamma", "snr_db", "wmse"],
                "starts": [{"theta0": list(t), "rows": r} for t, r in zip(ms.starts, rows)]}
    ms.run(1)                                  # eager chunk + graph capture
    ms.synchronize()
    t0 = time.perf_counter()
    ms.run(chunks)
    ms.synchronize()
    tb = time.perf_counter() - t0
    snr, wmse = ms.quality(truth)
    starts = []
    for i, (m0, g0) in enumerate(ms.starts):
        r = ms.start(i).report()
        starts.append({"theta0": [m0, g0], "mu": round(r["mu"], 6), "gamma": round(r["gamma"], 6),
                       "sugar_mu": float(f"{r['sugar_mu']:.4g}"),
                       "sugar_gamma": float(f"{r['sugar_gamma']:.4g}"),
                       "snr_db": round(float(snr[i]), 3), "wmse": float(f"{wmse[i]:.4g}")})
    ms.close()
    # the same starts one after the other, eager, for the same iterations
    ts = 0.0
    for m0, g0 in mm.MultiStart.PAPER_STARTS:
        c = mm.default_config(p.n, p.L, mode=mm.F32, sure=1, delta_period=10,
                              eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w, eta_mu=eta_mu,
                              eta_gamma=eta_gamma, pi_iters=100, mu=m0, gamma=g0)
        h = mm.Muffin(c)
        h.set_problem(dirty, psf, None, None, delta)
        h.run(10, report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.run(10 * chunks, report=False)
        torch.cuda.synchronize()
        ts += time.perf_counter() - t0
        h.close()
    del dirty, psf, delta, truth
    torch.cuda.empty_cache()
    k = 10 * (chunks + 1)
    return {"form": "ADA-PT, FP32, 256x256 px x 64 bands from the four (mu, gamma) of "
                    "Section 4.2, one captured graph per 10 iterations of all starts",
            "eta": [eta_mu, eta_gamma], "iterations_timed": 10 * chunks,
            "start_iters_per_s": round(4 * 10 * chunks / tb, 2),
            "ms_per_iteration_all_starts": round(1e3 * tb / (10 * chunks), 3),
            "one_after_another_start_iters_per_s": round(4 * 10 * chunks / ts, 2),
            "speedup_vs_one_after_another": round(ts / tb, 3),
            "after_iterations": k, "starts": starts}


def unmix_form(mm, torch, prob, reps=20):
    """Spectral unmixing (Section 4.3) of the 1024^2 x 256 sky in FP32
    against the spectra of three bright pixels (the brightest ones at least
    16 px apart, i.e. of different sources): one kernel launch
    per cube, timed with HIP events on the launch stream."""
    cube = torch.from_numpy(prob.sky).to("cuda:0", torch.float32)
    L, n, _ = cube.shape
    flux = cube.sum(0).flatten()
    cand = torch.topk(flux, 2000).indices.cpu().numpy()
    pix = []                                    # brightest, at least 16 px apart
    for p in cand:
        i, j = int(p) // n, int(p) % n
        if all(max(abs(i - a), abs(j - b)) >= 16 for a, b in pix):
            pix.append((i, j))
        if len(pix) == 3:
            break
    u = mm.Unmixer(mm.Unmixer.spectra_at(cube, pix))
    s = torch.cuda.current_stream()
    a, r = u.run(cube, residual=True)           # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        u.run(cube, residual=True)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = (L + 3 + 1) * n * n * 4
    frac_support = float((a > 0).any(0).float().mean())
    u.close()
    del cube, a, r
    torch.cuda.empty_cache()
    return {"form": "FP32 cube 1024x1024 px x 256 bands, 3 endmembers (brightest pixels), "
                    "per-pixel non-negative least squares",
            "ms_per_cube": round(ms, 4), "pixels_per_s": round(n * n / (ms * 1e-3), 1),
            "algorithmic_GB": round(nbytes / 1e9, 3),
            "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "pixels_with_nonzero_abundance": round(frac_support, 4)}


def vis_form(mm, torch, synth, steps, seed=0):
    """Visibility data: the 256^2 px x 64 band sky sampled at 4000
    baselines per band (continuous positions), ADA-PT in the FP32 + bf16 DCT
    form.  The set-up back-projects the visibilities and the probe and builds
    the PSF with exact sums (timed with HIP events); the iteration then runs
    on the PSF convolution."""
    n, L, K = 256, 64, 4000
    p = synth.make_vis_problem(n, L, 200, 10, K, seed=seed, device="cuda:0")
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    dirty, psf, dimg, nrm = mm.vis_prepare(p.uv, p.vis, n, mm.F32_BF16DCT, delta=p.delta)
    e1.record(s)
    torch.cuda.synchronize()
    prep_ms = e0.elapsed_time(e1)
    terms = L * K * (2 * n * n + 4 * n * n)            # dirty + probe + PSF outputs
    cfg = mm.default_config(n, L, mode=mm.F32_BF16DCT, sure=1, delta_period=10,
                            eps_fd=0.01 * p.sigma_w, sigma_w=p.sigma_w, eta_mu=1e-6,
                            eta_gamma=1e-6, pi_iters=50, pi_tol=1e-6, visibilities=1,
                            vis_norm2=nrm, vis_count=2.0 * L * K)
    h = mm.Muffin(cfg)
    h.set_problem(dirty, psf, None, None, dimg)
    h.run(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.run(steps, report=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rep = h.report()
    h.close()
    del dirty, psf, dimg
    torch.cuda.empty_cache()
    return {"form": "ADA-PT on visibilities (exact sums at 4000 continuous baselines per band), "
                    "256x256 px x 64 bands, FP32 + bf16 DCT",
            "prepare_ms": round(prep_ms, 2),
            "prepare_terms_per_s": round(terms / (prep_ms * 1e-3), 1),
            "value": round(steps / el, 3), "unit": "iters/s",
            "ms_per_step": round(1e3 * el / steps, 3), "psure": rep["psure"]}


def serve_form(mm, torch, synth, prob_c2, n_req, rates, seed=11, slots=8):
    """Serving form (the paper has none; the workload is the serving
    configuration of the benchmark): Poisson arrivals of plain deconvolution
    solves, sizes uniform over n in {64, ..., 1024} x L in {8, ..., 256}
    (powers of two), FP32 with the bf16 DCT, each to a relative change of
    1e-4 or 2000 iterations, through the continuous-batching server.  The
    same seeded draw of `n_req` requests is replayed at every rate of
    `rates` (req/s); inputs of a size class are generated once (the
    1024-pixel classes take the first L bands of the 1024^2 x 256 cube)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ns, Ls = [64, 128, 256, 512, 1024], [8, 16, 32, 64, 128, 256]
    classes = [(n, L) for n in ns for L in Ls]
    picks = [classes[i] for i in rng.integers(0, len(classes), size=n_req)]
    gaps = rng.exponential(1.0, size=n_req)          # arrivals at rate r: gaps / r
    inputs = {}
    for c in sorted(set(picks)):
        n, L = c
        if n == prob_c2.n:
            d = lambda a: torch.from_numpy(np.ascontiguousarray(a[:L])).to("cuda:0",
                                                                            torch.float32)
            inputs[c] = (d(prob_c2.dirty), d(prob_c2.psf))
        else:
            _, di, ps, _ = _class_inputs(synth, torch, n, L, 2000 + n + L, torch.float32)
            inputs[c] = (di, ps)
    torch.cuda.synchronize()
    cfgs = {c: mm.default_config(c[0], c[1], mode=mm.F32_BF16DCT, stop_rel=1e-4,
                                 check_every=10, pi_iters=30, pi_tol=1e-4) for c in inputs}
    srv = mm.Server(max_active=slots)
    # warm-up: one short solve per size class (handles pooled, kernels loaded)
    for t in [srv.submit(cfgs[c], inputs[c][0], inputs[c][1], 10) for c in inputs]:
        srv.wait(t)
    runs = []
    for rate in rates:
        arrivals = np.cumsum(gaps / rate)
        tickets = []
        t0 = time.perf_counter()
        for c, ta in zip(picks, arrivals):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append((c, srv.submit(cfgs[c], inputs[c][0], inputs[c][1], 2000)))
        lat, its, vox_it, stopped = [], [], 0.0, 0
        for c, t in tickets:
            r = srv.wait(t)
            if r["status"] != mm.REQ_DONE:
                raise RuntimeError(f"request {t} ended with status {r['status']}")
            lat.append(r["latency_ms"])
            k = r["report"]["iters_done"]
            its.append(k)
            stopped += r["report"]["stopped"]
            vox_it += c[0] * c[0] * c[1] * k
            log(f"[bench] serve {rate} req/s: request {len(lat)}/{n_req} done "
                f"({c[0]}^2 x {c[1]}, {k} its, {r['latency_ms'] / 1e3:.1f} s)")
        span = time.perf_counter() - t0
        lat = np.array(lat)
        runs.append({"rate_req_per_s": rate,
                     "p50_ms": round(float(np.percentile(lat, 50)), 2),
                     "p99_ms": round(float(np.percentile(lat, 99)), 2),
                     "mean_ms": round(float(lat.mean()), 2),
                     "throughput_req_per_s": round(n_req / span, 4),
                     "voxel_updates_per_s": round(vox_it / span, 1),
                     "iterations_mean": round(float(np.mean(its)), 1),
                     "met_1e-4": stopped, "span_s": round(span, 2)})
    srv.close()
    del inputs
    torch.cuda.empty_cache()
    out = {"form": "plain MUFFIN, FP32 + bf16 DCT, to relative change 1e-4 or 2000 iterations",
           "requests": n_req, "slots": slots,
           "sizes": "n in {64,128,256,512,1024}, L in {8,16,32,64,128,256}, uniform "
                    "(seeded draw); the 1024-pixel classes use the first L bands of the "
                    "1024^2 x 256 cube",
           "drawn": sorted({f"{n}x{L}" for n, L in picks}),
           "voxels_mean": round(float(np.mean([n * n * L for n, L in picks])), 1)}
    out.update(runs[0])
    if len(runs) > 1:
        out["sweep"] = runs
    return out


def _errors(torch, x, ref):
    d = (x.double() - ref).abs()
    return {"max_abs": float(d.max()), "rel_l2": float(torch.linalg.vector_norm(d) /
                                                     torch.linalg.vector_norm(ref))}


def accuracy_form(mm, torch, synth, prob_c2, plain_iters=(20, 500), adapt_iters=(40, 500),
                  eta=(5e-3, 1e-3)):
    """Errors of the reduced-precision forms against the FP64 GPU path (the
    path the parity tests pin to the FP64 oracle) from the same inputs and a
    fixed step tau, after short and long runs: plain MUFFIN at 1024^2 x 256
    (iterations `plain_iters`), ADA-PT at 256^2 x 64 with theta updated every
    10 iterations by steps `eta` (iterations `adapt_iters`; theta moves well
    away from its start, so its error is that of the whole SUGAR path).
    Each form runs once to the last count; the sky is copied at the others."""
    forms = [("f32", mm.F32), ("bf16", mm.F32_BF16DCT)]

    def run(prob, mode, sure, counts, tau):
        dt = torch.float64 if mode == mm.F64 else torch.float32
        cfg = mm.default_config(prob.n, prob.L, mode=mode, sure=1 if sure else 0,
                                delta_period=10, eps_fd=0.01 * prob.sigma_w,
                                sigma_w=prob.sigma_w, eta_mu=eta[0], eta_gamma=eta[1],
                                tau=tau, pi_iters=50, pi_tol=1e-6)
        h = mm.Muffin(cfg)
        dev = lambda a: torch.from_numpy(a).to("cuda:0", dt)
        h.set_problem(dev(prob.dirty), dev(prob.psf), None, None,
                      dev(prob.delta) if sure else None)
        out, done = {}, 0
        for k in counts:
            rep = h.run(k - done)
            done = k
            out[k] = (h.sky().double(), rep)
        h.close()
        torch.cuda.empty_cache()
        return out

    res = {}
    rep0 = run(prob_c2, mm.F64, False, (0,), 0.0)[0][1]   # tau of the FP64 set-up
    tau = rep0["tau"]
    ref = run(prob_c2, mm.F64, False, plain_iters, tau)
    for name, m in forms:
        got = run(prob_c2, m, False, plain_iters, tau)
        for k in plain_iters:
            res.setdefault(f"plain_1024x256_{k}_iters", {})[name] = _errors(torch, got[k][0],
                                                                             ref[k][0])
        del got
    del ref
    torch.cuda.empty_cache()
    p1 = synth.make_config("c1", seed=0, device="cuda:0")
    r0 = run(p1, mm.F64, True, (0,), 0.0)[0][1]
    ref = run(p1, mm.F64, True, adapt_iters, r0["tau"])
    for name, m in forms:
        got = run(p1, m, True, adapt_iters, r0["tau"])
        for k in adapt_iters:
            e = _errors(torch, got[k][0], ref[k][0])
            r, r64 = got[k][1], ref[k][1]
            e["mu"], e["gamma"] = r["mu"], r["gamma"]
            e["mu_rel"] = abs(r["mu"] - r64["mu"]) / abs(r64["mu"]) if r64["mu"] else abs(r["mu"])
            e["gamma_rel"] = abs(r["gamma"] - r64["gamma"]) / abs(r64["gamma"])
            res.setdefault(f"adapt_256x64_{k}_iters", {})[name] = e
    for k in adapt_iters:
        res[f"adapt_256x64_{k}_iters"]["fp64_theta"] = [ref[k][1]["mu"], ref[k][1]["gamma"]]
    res["reference"] = ("FP64 GPU path, same inputs, same fixed tau; ADA-PT with eta = "
                        f"({eta[0]}, {eta[1]}), eps = 0.01 sigma_w, theta(0) = (1, 1)")
    return res


def run_form(mm, torch, prob, mode, sure, steps, warmup, Delta=10, dictionary=0):
    n, L = prob.n, prob.L
    dt = torch.float64 if mode == mm.F64 else torch.float32
    eps = 0.01 * prob.sigma_w
    cfg = mm.default_config(n, L, mode=mode, mu=1.0, gamma=1.0, sure=1 if sure else 0,
                            delta_period=Delta, eps_fd=eps, sigma_w=prob.sigma_w,
                            eta_mu=1e-6, eta_gamma=1e-6, pi_iters=50, pi_tol=1e-6,
                            dictionary=dictionary)
    h = mm.Muffin(cfg)
    dirty = torch.from_numpy(prob.dirty).to("cuda:0", dt)
    psf = torch.from_numpy(prob.psf).to("cuda:0", dt)
    delta = torch.from_numpy(prob.delta).to("cuda:0", dt) if sure else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.set_problem(dirty, psf, None, None, delta)
    setup_s = time.perf_counter() - t0
    del psf
    torch.cuda.empty_cache()
    h.run(warmup, report=True)
    h.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.run(steps, report=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    timing = h.timing()
    rep = h.report()
    h.set_timing(False)
    # untimed check run without events, to compare the overhead
    torch.cuda.synchronize()
    h.close()
    del dirty, delta
    torch.cuda.empty_cache()
    return dict(elapsed=el, setup_s=setup_s, timing=timing, report=rep)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_1905_08468_amd import muffin as mm

    mode = {"f32": mm.F32, "bf16": mm.F32_BF16DCT, "f64": mm.F64}[args.mode]
    t0 = time.perf_counter()
    prob = synth.make_config(args.workload, seed=args.seed, device="cuda:0")
    log(f"[bench] generated {args.workload} n={prob.n} L={prob.L} in "
        f"{time.perf_counter() - t0:.1f} s")
    n, L = prob.n, prob.L
    LN = n * n * L

    main_form = run_form(mm, torch, prob, mode, True, args.steps, args.warmup)
    el = main_form["elapsed"]
    value = args.steps / el
    log(f"[bench] ADA-PT {args.mode}: {value:.3f} it/s ({1e3 * el / args.steps:.1f} ms/step)")

    # per-stage achieved bandwidth from the live HIP-event timings; the
    # roofline object reports the single-launch stage that takes longest
    es = 8 if mode == mm.F64 else 4
    tm = main_form["timing"]
    stages = {}
    for k, (ms, calls) in tm.items():
        if not calls:
            continue
        entry = {"ms_per_step": round(ms / args.steps, 3), "calls": calls}
        if k in STAGE_TRAFFIC:
            vals, mbytes = STAGE_TRAFFIC[k]
            nbytes = LN * (vals * es + mbytes)
            avg = ms / calls
            entry["algorithmic_GB"] = round(nbytes / 1e9, 2)
            entry["GBps"] = round(nbytes / (avg * 1e-3) / 1e9, 1)
        if k in ("dct_primal", "dct_deriv"):
            # two (L x L)(L x N) products per set; the bf16 form issues three
            # MFMA products (hi hi, lo hi, hi lo) per product
            sets = 2 if k == "dct_primal" else 4
            lp = -(-L // 32) * 32
            mult, peak = (3, MFMA_BF16_PEAK) if mode == mm.F32_BF16DCT else \
                ((1, MFMA_F64_PEAK) if mode == mm.F64 else (1, MFMA_F32_PEAK))
            fl = sets * 2 * 2.0 * lp * lp * n * n * mult
            tf = fl / (ms / calls * 1e-3) / 1e12
            entry["mfma_TFLOPs"] = round(tf, 1)
            entry["mfma_util"] = round(tf / peak, 4)
        if k == "fft_chain":
            # the chain's algorithmic bytes (116 V per voxel for 6 sets) and
            # its nominal flops over its measured time
            sets = 6
            nbytes = LN * es * sum(STAGE_TRAFFIC[f"fft_{p}"][0] for p in
                                   ("row1", "col1", "row2", "col2", "row3"))
            avg = ms / calls
            entry["algorithmic_GB"] = round(nbytes / 1e9, 2)
            entry["GBps"] = round(nbytes / (avg * 1e-3) / 1e9, 1)
            entry["frac_hbm"] = round(nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            tfl = fft_chain_flops(n, L, sets) / (avg * 1e-3) / 1e12
            entry["nominal_TFLOPs"] = round(tfl, 1)
            vec_peak = FP32_VECTOR_UNPACKED if mode != mm.F64 else MFMA_F64_PEAK
            entry["frac_vector_peak"] = round(tfl / vec_peak, 4)
        if k in STAGE_TRAFFIC:
            entry["frac_hbm"] = round(entry["GBps"] / HBM_PEAK_GBS, 4)
        stages[k] = entry
    dom = max((k for k in stages if k in STAGE_TRAFFIC), key=lambda k: tm[k][0])
    vals, mbytes = STAGE_TRAFFIC[dom]
    bytes_launch = LN * (vals * es + mbytes)
    avg_ms = tm[dom][0] / tm[dom][1]
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    kernel_of = {"synthesis_l1": "dwt_sy level 1", "analysis_l1_primal": "dwt_an level 1",
                 "analysis_l1_deriv": "dwt_an level 1", "dct_primal": "dct kernel",
                 "dct_deriv": "dct kernel", "primal_step": "primal_kernel",
                 "fft_row1": "row_pass_pruned", "fft_col1": "col_pass_rt",
                 "fft_row2": "row_pass_pruned", "fft_col2": "col_pass_rt",
                 "fft_row3": "row_pass_pruned"}
    kname = f"{kernel_of[dom]} ({dom})"
    traffic = measured_traffic(kname) if args.workload == "c2" and mode == mm.F32_BF16DCT else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes": bytes_launch}
    # the wavelet launches are close to their FP32 arithmetic too: the FMA
    # rate of the same launch against the vector peak (packed, and the
    # unpacked rate this build's code can reach)
    sets_of = {"synthesis_l1": 6, "analysis_l1_primal": 2, "analysis_l1_deriv": 4}
    if dom in sets_of and mode != mm.F64 and args.workload == "c2":
        fma = wavelet_fmas(dom, n, L, sets_of[dom])
        tfl = 2.0 * fma / (avg_ms * 1e-3) / 1e12
        roofline["alu"] = {"flop_per_launch": 2 * fma, "achieved": round(tfl, 1),
                           "unit": "TFLOP/s", "peak": FP32_VECTOR_PEAK,
                           "frac": round(tfl / FP32_VECTOR_PEAK, 4),
                           "frac_unpacked": round(tfl / FP32_VECTOR_UNPACKED, 4)}

    fp64 = None
    if not args.no_fp64:
        try:
            f = run_form(mm, torch, prob, mm.F64, False, max(2, args.steps // 4), 1)
            k64 = max(2, args.steps // 4)
            fp64 = {"form": "plain FP64 MUFFIN (Alg. 2, fixed theta)",
                    "value": round(k64 / f["elapsed"], 4), "unit": "iters/s",
                    "ms_per_step": round(1e3 * f["elapsed"] / k64, 2)}
            log(f"[bench] plain FP64: {fp64['value']} it/s")
            # the same plain method in the default precision form, for the
            # speedup of that form over the FP64 GPU method
            fm = run_form(mm, torch, prob, mode, False, k64, 1)
            mixed = k64 / fm["elapsed"]
            fp64["same_method_in_this_form"] = {"value": round(mixed, 4), "unit": "iters/s",
                                                "speedup_vs_fp64": round(mixed / fp64["value"], 3)}
            log(f"[bench] plain {args.mode}: {mixed:.3f} it/s, x{mixed / fp64['value']:.2f} vs FP64")
        except Exception as e:  # report, do not hide
            fp64 = {"error": str(e)}
    if args.calib:
        # a plain streaming kernel of known size, for scaling the HBM traffic
        # counters: 2^28 floats (1 GiB) read, converted to half (512 MiB)
        # written, three times; no other step launches this kernel
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        for _ in range(3):
            dst = src.to(torch.float16)
            del dst
        torch.cuda.synchronize()
        del src
        log("[bench] calibration: 3 x (1 GiB f32 read -> 512 MiB f16 written)")
    torch.cuda.empty_cache()
    accuracy = None
    if not args.no_accuracy and args.workload == "c2":
        try:
            accuracy = accuracy_form(mm, torch, synth, prob)
            log(f"[bench] accuracy: {json.dumps(accuracy)}")
        except Exception as e:  # report, do not hide
            accuracy = {"error": str(e)}
    batch = None
    if not args.no_batch:
        try:
            batch = batch_form(mm, torch, synth, args.batch_cubes, args.batch_chunks)
            log(f"[bench] batch: {batch['cube_iters_per_s']} cube-it/s, "
                f"x{batch['speedup_vs_one_after_another']} vs one after another")
        except Exception as e:  # report, do not hide
            batch = {"error": str(e)}
    starlet = None
    if not args.no_starlet:
        try:
            k_st = max(3, args.steps // 4)
            f = run_form(mm, torch, prob, mode, True, k_st, 1, dictionary=mm.DICT_STARLET)
            st_stages = {k: round(ms / k_st, 3) for k, (ms, calls) in f["timing"].items() if calls}
            starlet = {"form": f"ADA-PT with the IUWT (starlet, J=3) spatial dictionary, same "
                               f"cube and precision form", "value": round(k_st / f["elapsed"], 4),
                       "unit": "iters/s", "ms_per_step": round(1e3 * f["elapsed"] / k_st, 2),
                       "stages_ms_per_step": st_stages}
            log(f"[bench] starlet ADA-PT: {starlet['value']} it/s")
        except Exception as e:  # report, do not hide
            starlet = {"error": str(e)}
    visf = None
    if not args.no_vis:
        try:
            visf = vis_form(mm, torch, synth, 20)
            log(f"[bench] visibilities: prepare {visf['prepare_ms']} ms, {visf['value']} it/s")
        except Exception as e:  # report, do not hide
            visf = {"error": str(e)}
    unmix = None
    if not args.no_unmix and args.workload == "c2":
        try:
            unmix = unmix_form(mm, torch, prob)
            log(f"[bench] unmix: {unmix['ms_per_cube']} ms per cube, {unmix['GBps']} GB/s")
        except Exception as e:  # report, do not hide
            unmix = {"error": str(e)}
    multistart = None
    if not args.no_multistart:
        try:
            multistart = multistart_form(mm, torch, synth, args.ms_iters,
                                         trace_every=args.ms_trace)
            if not args.ms_trace:
                log(f"[bench] multi-start: {multistart['start_iters_per_s']} start-it/s, "
                    f"x{multistart['speedup_vs_one_after_another']} vs one after another")
        except Exception as e:  # report, do not hide
            multistart = {"error": str(e)}
    serve = None
    if not args.no_serve:
        try:
            rates = [args.serve_rate] + [float(r) for r in args.serve_sweep.split(",") if r]
            serve = serve_form(mm, torch, synth, prob, args.serve_requests, rates)
            log(f"[bench] serve: p50 {serve['p50_ms']} ms, p99 {serve['p99_ms']} ms, "
                f"{serve['throughput_req_per_s']} req/s")
        except Exception as e:  # report, do not hide
            serve = {"error": str(e)}
    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(prob, synth)
            log(f"[bench] cpu oracle: {cpu['value']:.3e} it/s on {cpu['cores']} cores")
        except Exception as e:  # report, do not hide
            cpu = {"error": str(e)}

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "f32+bf16", "f64": "f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": f"ADA-PT'ed MUFFIN iteration, {n}x{n} px x {L} bands, "
                               f"PSF {2 * n}x{2 * n}, P=8 Daubechies bases, J=3, DCT, "
                               "Delta=10", "n": n, "bands": L,
                   "form": {"f32": "FP32", "bf16": "FP32, DCT on bf16 MFMA hi+lo split",
                            "f64": "FP64"}[args.mode]},
        "voxel_updates_per_s": round(value * LN, 1),
        "setup_s": round(main_form["setup_s"], 3),
        "theta": {"mu": main_form["report"]["mu"], "gamma": main_form["report"]["gamma"],
                  "updates": main_form["report"]["theta_updates"]},
        "roofline": roofline,
        "stages_ms_per_step": stages,
        "fp64_plain": fp64,
        "accuracy": accuracy,
        "batch": batch,
        "multistart": multistart,
        "unmix": unmix,
        "starlet": starlet,
        "visibilities": visf,
        "serve": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
