"""ctypes binding of libmuffin (include/muffin.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Tensors are torch device tensors of the handle's working dtype;
their data pointers and the current torch stream are passed to the C ABI.
If the library has not been built this module raises on import -- there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MUFFIN_LIB", os.path.join(_HERE, "libmuffin.so"))

F64, F32, F32_BF16DCT = 0, 1, 2
TAU_OPNORM, TAU_PAPER_SUM = 0, 1
DICT_DAUBECHIES, DICT_STARLET = 0, 1

ERRORS = {0: "ok", -1: "E_INVAL", -2: "E_SHAPE", -3: "E_NOMEM", -4: "E_NONFINITE",
          -5: "E_HIP", -6: "E_STATE", -7: "E_BUSY", -8: "E_SCRATCH"}
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED = 0, 1, 2, 3


class MuffinError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({_lib.muffin_strerror(code).decode()})")


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("L", C.c_int32), ("n_bases", C.c_int32), ("levels", C.c_int32),
        ("mode", C.c_int32),
        ("mu", C.c_double), ("gamma", C.c_double), ("sigma", C.c_double), ("tau", C.c_double),
        ("tau_rule", C.c_int32), ("rho", C.c_double), ("eps_w", C.c_double),
        ("sure", C.c_int32), ("delta_period", C.c_int32),
        ("eta_mu", C.c_double), ("eta_gamma", C.c_double),
        ("eps_fd", C.c_double), ("sigma_w", C.c_double),
        ("deriv_reset", C.c_int32), ("pi_iters", C.c_int32), ("pi_tol", C.c_double),
        ("stop_rel", C.c_double), ("check_every", C.c_int32),
        ("dictionary", C.c_int32),
        ("visibilities", C.c_int32), ("vis_norm2", C.c_double), ("vis_count", C.c_double),
    ]


class Report(C.Structure):
    _fields_ = [
        ("iters_done", C.c_int32), ("theta_updates", C.c_int32),
        ("mu", C.c_double), ("gamma", C.c_double), ("tau", C.c_double),
        ("beta_H", C.c_double), ("psure", C.c_double), ("sugar_mu", C.c_double),
        ("sugar_gamma", C.c_double), ("res2", C.c_double),
        ("last_rel_change", C.c_double), ("stopped", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(C.Structure):
    _fields_ = [("tunable", C.c_int32), ("cached", C.c_int32), ("syn_tile1", C.c_int32),
                ("an_tile1", C.c_int32), ("syn_ms", C.c_double * 2), ("an_ms", C.c_double * 2)]

    def as_dict(self):
        return {"tunable": self.tunable, "cached": self.cached, "syn_tile1": self.syn_tile1,
                "an_tile1": self.an_tile1, "syn_ms": list(self.syn_ms),
                "an_ms": list(self.an_ms)}


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int32),
                ("max_queue", C.c_int32), ("chunk", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("queued", C.c_int32), ("active", C.c_int32), ("completed", C.c_int32),
                ("failed", C.c_int32), ("cancelled", C.c_int32), ("pooled_handles", C.c_int32),
                ("bytes_in_use", C.c_size_t), ("bytes_budget", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "muffin_default_config", "muffin_workspace_bytes", "muffin_create", "muffin_set_problem",
    "muffin_run", "muffin_get_sky", "muffin_get_state", "muffin_set_state",
    "muffin_get_history", "muffin_get_weights", "muffin_get_report", "muffin_destroy",
    "muffin_strerror", "muffin_op_H", "muffin_op_HT", "muffin_op_HTH", "muffin_op_Ws",
    "muffin_op_WsT", "muffin_op_dct", "muffin_op_idct",
    "muffin_set_timing", "muffin_get_timing", "muffin_stage_name",
    "muffin_set_initial", "muffin_state_bytes", "muffin_state_save", "muffin_state_load",
    "muffin_solve", "muffin_solve_noalloc",
    "muffin_server_default_config", "muffin_server_create", "muffin_server_submit",
    "muffin_server_poll", "muffin_server_wait", "muffin_server_cancel",
    "muffin_server_get_stats", "muffin_server_destroy",
    "muffin_batch_create", "muffin_batch_run", "muffin_batch_destroy",
    "muffin_quality", "muffin_multistart_create", "muffin_multistart_set_problem",
    "muffin_multistart_run", "muffin_multistart_quality", "muffin_multistart_handle",
    "muffin_multistart_destroy",
    "muffin_unmix_plan_create", "muffin_unmix_run", "muffin_unmix_plan_destroy",
    "muffin_autotune", "muffin_vis_prepare", "muffin_vis_degrid",
]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(python paper_1905_08468_amd/build.py)")
    lib = C.CDLL(path)
    vp, i32, dp = C.c_void_p, C.c_int32, C.POINTER(C.c_double)
    cfgp = C.POINTER(Config)
    sig = {
        "muffin_default_config": ([cfgp, i32, i32], C.c_int),
        "muffin_workspace_bytes": ([cfgp], C.c_size_t),
        "muffin_create": ([C.POINTER(vp), cfgp, vp], C.c_int),
        "muffin_set_problem": ([vp, vp, vp, dp, dp, vp], C.c_int),
        "muffin_run": ([vp, i32, C.POINTER(Report)], C.c_int),
        "muffin_get_sky": ([vp, vp], C.c_int),
        "muffin_get_state": ([vp, i32, i32, vp], C.c_int),
        "muffin_set_state": ([vp, i32, i32, vp], C.c_int),
        "muffin_get_history": ([vp, dp, i32], C.c_int),
        "muffin_get_weights": ([vp, dp, dp], C.c_int),
        "muffin_get_report": ([vp, C.POINTER(Report)], C.c_int),
        "muffin_destroy": ([vp], C.c_int),
        "muffin_strerror": ([C.c_int], C.c_char_p),
        "muffin_set_timing": ([vp, i32], C.c_int),
        "muffin_get_timing": ([vp, dp, C.POINTER(C.c_int64), i32], C.c_int),
        "muffin_stage_name": ([i32], C.c_char_p),
        "muffin_set_initial": ([vp, vp], C.c_int),
        "muffin_state_bytes": ([vp], C.c_size_t),
        "muffin_state_save": ([vp, vp, C.c_size_t], C.c_int),
        "muffin_state_load": ([vp, vp, C.c_size_t], C.c_int),
        "muffin_solve": ([cfgp, vp, vp, dp, dp, vp, vp, i32, vp, C.POINTER(Report), vp], C.c_int),
        "muffin_solve_noalloc": ([cfgp, vp, vp, dp, dp, vp, vp, i32, vp, C.POINTER(Report), vp],
                                 C.c_int),
        "muffin_server_default_config": ([C.POINTER(ServerConfig)], C.c_int),
        "muffin_server_create": ([C.POINTER(vp), C.POINTER(ServerConfig)], C.c_int),
        "muffin_server_submit": ([vp, cfgp, vp, vp, dp, dp, vp, i32, vp,
                                  C.POINTER(C.c_int64)], C.c_int),
        "muffin_server_poll": ([vp, C.c_int64, C.POINTER(i32), C.POINTER(Report), dp], C.c_int),
        "muffin_server_wait": ([vp, C.c_int64, C.c_double, C.POINTER(i32), C.POINTER(Report),
                                dp], C.c_int),
        "muffin_server_cancel": ([vp, C.c_int64], C.c_int),
        "muffin_server_get_stats": ([vp, C.POINTER(ServerStats)], C.c_int),
        "muffin_server_destroy": ([vp], C.c_int),
        "muffin_batch_create": ([C.POINTER(vp), C.POINTER(vp), i32, i32, vp], C.c_int),
        "muffin_batch_run": ([vp, i32], C.c_int),
        "muffin_batch_destroy": ([vp], C.c_int),
        "muffin_quality": ([vp, vp, dp, dp], C.c_int),
        "muffin_multistart_create": ([C.POINTER(vp), cfgp, i32, dp, dp, vp], C.c_int),
        "muffin_multistart_set_problem": ([vp, vp, vp, dp, dp, vp, i32], C.c_int),
        "muffin_multistart_run": ([vp, i32], C.c_int),
        "muffin_multistart_quality": ([vp, vp, dp, dp], C.c_int),
        "muffin_multistart_handle": ([vp, i32], vp),
        "muffin_multistart_destroy": ([vp], C.c_int),
        "muffin_unmix_plan_create": ([C.POINTER(vp), dp, i32, i32], C.c_int),
        "muffin_unmix_run": ([vp, vp, i32, i32, vp, vp, vp], C.c_int),
        "muffin_unmix_plan_destroy": ([vp], C.c_int),
        "muffin_autotune": ([vp, i32, C.POINTER(TuneResult)], C.c_int),
        "muffin_vis_prepare": ([vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, dp, vp], C.c_int),
        "muffin_vis_degrid": ([vp, i32, i32, i32, i32, vp, vp, vp], C.c_int),
    }
    for name in ["muffin_op_H", "muffin_op_HT", "muffin_op_HTH", "muffin_op_Ws",
                 "muffin_op_WsT", "muffin_op_dct", "muffin_op_idct"]:
        sig[name] = ([vp, vp, vp], C.c_int)
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = load_library()


def default_config(n: int, L: int, **over) -> Config:
    c = Config()
    rc = _lib.muffin_default_config(C.byref(c), n, L)
    if rc:
        raise MuffinError(rc, "muffin_default_config")
    for k, v in over.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def workspace_bytes(cfg: Config) -> int:
    return int(_lib.muffin_workspace_bytes(C.byref(cfg)))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dptr(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _working_dtype(cfg: Config):
    import torch
    return torch.float64 if cfg.mode == F64 else torch.float32


def check_cube(t, shape, dtype, name, device=None):
    """Raises ValueError unless t is a contiguous device tensor of the given
    shape and dtype (on `device` if given): the library reads and writes
    exactly that many elements through the raw pointer."""
    if t is None:
        raise ValueError(f"{name}: a tensor is required")
    ok = (tuple(t.shape) == tuple(shape) and t.dtype == dtype and t.is_cuda
          and t.is_contiguous() and (device is None or t.device == device))
    if not ok:
        raise ValueError(f"{name}: expected a contiguous {dtype} cuda tensor of shape "
                         f"{tuple(shape)}{'' if device is None else ' on ' + str(device)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}"
                         f"{'' if t.is_contiguous() else ' (not contiguous)'}")


def check_weights(alpha, beta, n, L):
    """Host weight arrays: alpha has n*n entries, beta L (or None).  Returns
    the marshalled pairs of _dptr."""
    a = _dptr(alpha)
    b = _dptr(beta)
    if a is not None and a[0].size != n * n:
        raise ValueError(f"alpha must have n*n = {n * n} entries, got {a[0].size}")
    if b is not None and b[0].size != L:
        raise ValueError(f"beta must have L = {L} entries, got {b[0].size}")
    return a, b


def check_problem(cfg: Config, dirty, psf, alpha, beta, delta, x0=None):
    """The checks every entry point that takes a problem applies: cube shapes,
    the working dtype, one device for all cubes, weight lengths, and the
    probe delta when the configuration runs ADA-PT."""
    n, L = cfg.n, cfg.L
    dt = _working_dtype(cfg)
    check_cube(dirty, (L, n, n), dt, "dirty")
    dv = dirty.device
    check_cube(psf, (L, 2 * n, 2 * n), dt, "psf", dv)
    if delta is not None:
        check_cube(delta, (L, n, n), dt, "delta", dv)
    elif cfg.sure:
        raise ValueError("delta: the probe cube is required when cfg.sure is set")
    if x0 is not None:
        check_cube(x0, (L, n, n), dt, "x0", dv)
    return check_weights(alpha, beta, n, L)


class Muffin:
    """One solve on the current CUDA/HIP device and torch stream."""

    def __init__(self, cfg: Config, stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.dtype = torch.float64 if cfg.mode == F64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = C.c_void_p()
        rc = _lib.muffin_create(C.byref(h), C.byref(cfg), C.c_void_p(s.cuda_stream))
        if rc:
            raise MuffinError(rc, "muffin_create")
        self.h = h

    def _check(self, t, shape, name):
        check_cube(t, shape, self.dtype, name, self.device)

    @property
    def cube(self):
        return (self.cfg.L, self.cfg.n, self.cfg.n)

    def autotune(self, reps: int = 3):
        """Level-1 wavelet tile shapes for this size class (muffin_autotune);
        call before set_problem."""
        r = TuneResult()
        rc = _lib.muffin_autotune(self.h, int(reps), C.byref(r))
        if rc:
            raise MuffinError(rc, "muffin_autotune")
        return r.as_dict()

    def set_problem(self, dirty, psf, alpha=None, beta=None, delta=None):
        a, b = check_problem(self.cfg, dirty, psf, alpha, beta, delta)
        if dirty.device != self.device:
            raise ValueError(f"dirty: on {dirty.device}, the handle is on {self.device}")
        self._keep = (dirty, psf, delta)
        rc = _lib.muffin_set_problem(self.h, _ptr(dirty), _ptr(psf),
                                     a[1] if a else None, b[1] if b else None, _ptr(delta))
        if rc:
            raise MuffinError(rc, "muffin_set_problem")

    def run(self, iters: int, report: bool = True):
        rep = Report()
        rc = _lib.muffin_run(self.h, int(iters), C.byref(rep) if report else None)
        if rc:
            raise MuffinError(rc, "muffin_run")
        return rep.as_dict() if report else None

    def set_initial(self, x0):
        self._check(x0, self.cube, "x0")
        rc = _lib.muffin_set_initial(self.h, _ptr(x0))
        if rc:
            raise MuffinError(rc, "muffin_set_initial")

    def state_save(self) -> np.ndarray:
        nb = int(_lib.muffin_state_bytes(self.h))
        buf = np.empty(nb, dtype=np.uint8)
        rc = _lib.muffin_state_save(self.h, buf.ctypes.data_as(C.c_void_p), nb)
        if rc:
            raise MuffinError(rc, "muffin_state_save")
        return buf

    def state_load(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        rc = _lib.muffin_state_load(self.h, buf.ctypes.data_as(C.c_void_p), buf.size)
        if rc:
            raise MuffinError(rc, "muffin_state_load")

    def report(self):
        rep = Report()
        rc = _lib.muffin_get_report(self.h, C.byref(rep))
        if rc:
            raise MuffinError(rc, "muffin_get_report")
        return rep.as_dict()

    def _settle(self):
        # results were written on the handle's stream: when that is not the
        # caller's current stream, wait for it before torch touches them
        if self.stream != self.torch.cuda.current_stream():
            self.stream.synchronize()

    def sky(self):
        out = self.torch.empty(self.cube, dtype=self.dtype, device=self.device)
        rc = _lib.muffin_get_sky(self.h, _ptr(out))
        if rc:
            raise MuffinError(rc, "muffin_get_sky")
        self._settle()
        return out

    @property
    def planes(self):
        """U planes per band: the bases of the Daubechies union, or the J
        scales and the coarse plane of the starlet."""
        c = self.cfg
        return c.levels + 1 if c.dictionary == DICT_STARLET else c.n_bases

    def _state_shape(self, which):
        n, L, P = self.cfg.n, self.cfg.L, self.planes
        return (L, P, n, n) if which == 1 else (L, n, n)

    def get_state(self, which: int, set_: int = 0):
        out = self.torch.empty(self._state_shape(which), dtype=self.dtype, device=self.device)
        rc = _lib.muffin_get_state(self.h, which, set_, _ptr(out))
        if rc:
            raise MuffinError(rc, "muffin_get_state")
        self._settle()
        return out

    def set_state(self, which: int, set_: int, t):
        self._check(t, self._state_shape(which), "state")
        rc = _lib.muffin_set_state(self.h, which, set_, _ptr(t))
        if rc:
            raise MuffinError(rc, "muffin_set_state")
        self.torch.cuda.current_stream().synchronize()

    def history(self):
        cnt = _lib.muffin_get_history(self.h, None, 0)
        if cnt < 0:
            raise MuffinError(cnt, "muffin_get_history")
        buf = np.zeros((max(cnt, 1), 8))
        _lib.muffin_get_history(self.h, buf.ctypes.data_as(C.POINTER(C.c_double)), cnt)
        return buf[:cnt]

    def quality(self, truth):
        """(SNR in dB, WMSE) of the current sky against the true sky
        (Section 4.1), through muffin_quality."""
        self._check(truth, self.cube, "truth")
        snr, wmse = C.c_double(), C.c_double()
        rc = _lib.muffin_quality(self.h, _ptr(truth), C.byref(snr), C.byref(wmse))
        if rc:
            raise MuffinError(rc, "muffin_quality")
        return snr.value, wmse.value

    def weights(self):
        a = np.zeros(self.cfg.n * self.cfg.n)
        b = np.zeros(self.cfg.L)
        rc = _lib.muffin_get_weights(self.h, a.ctypes.data_as(C.POINTER(C.c_double)),
                                     b.ctypes.data_as(C.POINTER(C.c_double)))
        if rc:
            raise MuffinError(rc, "muffin_get_weights")
        return a, b

    def op(self, name: str, x):
        n, L, P = self.cfg.n, self.cfg.L, self.planes
        fn = getattr(_lib, f"muffin_op_{name}")
        if name == "WsT":
            self._check(x, (L, P, n, n), "in")
            out = self.torch.empty((L, n, n), dtype=self.dtype, device=self.device)
        else:
            self._check(x, (L, n, n), "in")
            shape = (L, P, n, n) if name == "Ws" else (L, n, n)
            out = self.torch.empty(shape, dtype=self.dtype, device=self.device)
        rc = fn(self.h, _ptr(x), _ptr(out))
        if rc:
            raise MuffinError(rc, f"muffin_op_{name}")
        self._settle()
        return out

    def set_timing(self, on: bool = True):
        rc = _lib.muffin_set_timing(self.h, 1 if on else 0)
        if rc:
            raise MuffinError(rc, "muffin_set_timing")

    def timing(self):
        """{stage: (total_ms, calls)} of the device-timed stages."""
        ms = (C.c_double * 32)()
        calls = (C.c_int64 * 32)()
        cnt = _lib.muffin_get_timing(self.h, ms, calls, 32)
        if cnt < 0:
            raise MuffinError(cnt, "muffin_get_timing")
        return {_lib.muffin_stage_name(i).decode(): (ms[i], calls[i]) for i in range(cnt)}

    def close(self):
        if getattr(self, "h", None):
            _lib.muffin_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(cfg: Config, dirty, psf, iters: int, alpha=None, beta=None, delta=None, x0=None,
          stream=None):
    """One-call solve (muffin_solve): returns (sky tensor, report dict)."""
    import torch
    a, b = check_problem(cfg, dirty, psf, alpha, beta, delta, x0)
    dt = _working_dtype(cfg)
    out = torch.empty((cfg.L, cfg.n, cfg.n), dtype=dt, device=dirty.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    rep = Report()
    rc = _lib.muffin_solve(C.byref(cfg), _ptr(dirty), _ptr(psf), a[1] if a else None,
                           b[1] if b else None, _ptr(delta), _ptr(x0), int(iters), _ptr(out),
                           C.byref(rep), C.c_void_p(s.cuda_stream))
    if rc:
        raise MuffinError(rc, "muffin_solve")
    return out, rep.as_dict()


def solve_noalloc(cfg: Config, dirty, psf, iters: int, alpha=None, beta=None, delta=None,
                  x0=None, out=None, stream=None):
    """One-call solve that allocates no device memory in the library
    (muffin_solve_noalloc): its buffers live in a static array of
    NOALLOC_BYTES per GPU.  `out` (the sky) may be passed so that the call
    allocates nothing in torch either.  Returns (sky tensor, report dict)."""
    import torch
    a, b = check_problem(cfg, dirty, psf, alpha, beta, delta, x0)
    dt = _working_dtype(cfg)
    if out is None:
        out = torch.empty((cfg.L, cfg.n, cfg.n), dtype=dt, device=dirty.device)
    check_cube(out, (cfg.L, cfg.n, cfg.n), dt, "out", dirty.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    rep = Report()
    rc = _lib.muffin_solve_noalloc(C.byref(cfg), _ptr(dirty), _ptr(psf), a[1] if a else None,
                                   b[1] if b else None, _ptr(delta), _ptr(x0), int(iters),
                                   _ptr(out), C.byref(rep), C.c_void_p(s.cuda_stream))
    if rc:
        raise MuffinError(rc, "muffin_solve_noalloc")
    return out, rep.as_dict()


NOALLOC_BYTES = 128 << 20


class Server:
    """Continuous-batching request loop (muffin_server_*) on the current device.

    submit() keeps references to the request's tensors until it has ended,
    so the caller may drop its own."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 8, max_queue: int = 4096,
                 chunk: int = 10):
        sc = ServerConfig()
        _lib.muffin_server_default_config(C.byref(sc))
        sc.hbm_budget, sc.max_active, sc.max_queue, sc.chunk = hbm_budget, max_active, \
            max_queue, chunk
        h = C.c_void_p()
        rc = _lib.muffin_server_create(C.byref(h), C.byref(sc))
        if rc:
            raise MuffinError(rc, "muffin_server_create")
        self.h = h
        self._keep = {}

    def submit(self, cfg: Config, dirty, psf, max_iters: int, alpha=None, beta=None,
               delta=None, out=None):
        import torch
        a, b = check_problem(cfg, dirty, psf, alpha, beta, delta)
        dt = _working_dtype(cfg)
        if out is None:
            out = torch.empty((cfg.L, cfg.n, cfg.n), dtype=dt, device=dirty.device)
        check_cube(out, (cfg.L, cfg.n, cfg.n), dt, "out", dirty.device)
        tk = C.c_int64()
        # the C side reads the inputs when it admits the request
        torch.cuda.current_stream().synchronize()
        rc = _lib.muffin_server_submit(self.h, C.byref(cfg), _ptr(dirty), _ptr(psf),
                                       a[1] if a else None, b[1] if b else None, _ptr(delta),
                                       int(max_iters), _ptr(out), C.byref(tk))
        if rc:
            raise MuffinError(rc, "muffin_server_submit")
        self._keep[tk.value] = (dirty, psf, delta, out)
        return tk.value

    def _result(self, ticket, st, rep, lat):
        out = self._keep[ticket][3]
        if st.value not in (REQ_QUEUED, REQ_RUNNING):
            self._keep[ticket] = (None, None, None, out)
        return {"status": st.value, "report": rep.as_dict(), "latency_ms": lat.value, "sky": out}

    def poll(self, ticket: int):
        st, rep, lat = C.c_int32(), Report(), C.c_double()
        rc = _lib.muffin_server_poll(self.h, ticket, C.byref(st), C.byref(rep), C.byref(lat))
        if rc:
            raise MuffinError(rc, "muffin_server_poll")
        return self._result(ticket, st, rep, lat)

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        st, rep, lat = C.c_int32(), Report(), C.c_double()
        rc = _lib.muffin_server_wait(self.h, ticket, float(timeout_ms), C.byref(st),
                                     C.byref(rep), C.byref(lat))
        if rc:
            raise MuffinError(rc, "muffin_server_wait")
        return self._result(ticket, st, rep, lat)

    def cancel(self, ticket: int):
        rc = _lib.muffin_server_cancel(self.h, ticket)
        if rc:
            raise MuffinError(rc, "muffin_server_cancel")

    def stats(self):
        s = ServerStats()
        rc = _lib.muffin_server_get_stats(self.h, C.byref(s))
        if rc:
            raise MuffinError(rc, "muffin_server_get_stats")
        return s.as_dict()

    def close(self):
        if getattr(self, "h", None):
            _lib.muffin_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Handles iterated together as one captured graph per chunk
    (muffin_batch_*).  Each handle needs a stream of its own; `stream` is the
    root the graph is launched on."""

    def __init__(self, handles, chunk: int = 0, stream=None):
        import torch
        self.handles = list(handles)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        arr = (C.c_void_p * len(self.handles))(*[h.h for h in self.handles])
        b = C.c_void_p()
        rc = _lib.muffin_batch_create(C.byref(b), arr, len(self.handles), int(chunk),
                                      C.c_void_p(self.stream.cuda_stream))
        if rc:
            raise MuffinError(rc, "muffin_batch_create")
        self.h = b

    def run(self, chunks: int):
        rc = _lib.muffin_batch_run(self.h, int(chunks))
        if rc:
            raise MuffinError(rc, "muffin_batch_run")

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "h", None):
            _lib.muffin_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _StartView(Muffin):
    """A start's handle inside a MultiStart (owned and destroyed by it)."""

    def __init__(self, h, cfg: Config, owner):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.dtype = torch.float64 if cfg.mode == F64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = None
        self.h = h
        self._owner = owner

    def _settle(self):
        # the start's stream belongs to the library: wait for the device
        self.torch.cuda.synchronize()

    def close(self):
        self.h = None


class MultiStart:
    """One cube from several initial couples theta = (mu, gamma), iterated as
    one batch (muffin_multistart_*).  The default starts are the four couples
    of Section 4.2."""

    PAPER_STARTS = ((1.0, 10.0), (1.0, 3.0), (0.005, 3.0), (0.005, 10.0))

    def __init__(self, cfg: Config, starts=PAPER_STARTS, stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.starts = [(float(m), float(g)) for m, g in starts]
        self.stream = stream if stream is not None else torch.cuda.Stream()
        mu0 = np.array([m for m, _ in self.starts])
        ga0 = np.array([g for _, g in self.starts])
        m = C.c_void_p()
        rc = _lib.muffin_multistart_create(
            C.byref(m), C.byref(cfg), len(self.starts),
            mu0.ctypes.data_as(C.POINTER(C.c_double)), ga0.ctypes.data_as(C.POINTER(C.c_double)),
            C.c_void_p(self.stream.cuda_stream))
        if rc:
            raise MuffinError(rc, "muffin_multistart_create")
        self.h = m
        self.views = [_StartView(_lib.muffin_multistart_handle(m, i), cfg, self)
                      for i in range(len(self.starts))]
        self.chunk = 0

    def set_problem(self, dirty, psf, alpha=None, beta=None, delta=None, chunk: int = 0):
        a, b = check_problem(self.cfg, dirty, psf, alpha, beta, delta)
        self._keep = (dirty, psf, delta)
        # set-up runs on the starts' own streams: inputs must be complete
        self.torch.cuda.current_stream().synchronize()
        rc = _lib.muffin_multistart_set_problem(self.h, _ptr(dirty), _ptr(psf),
                                                a[1] if a else None, b[1] if b else None,
                                                _ptr(delta), int(chunk))
        if rc:
            raise MuffinError(rc, "muffin_multistart_set_problem")
        need = 2
        if self.cfg.sure:
            need = np.lcm(2, int(self.cfg.delta_period))
        self.chunk = int(chunk) if chunk else int(need)

    def run(self, chunks: int):
        """Enqueues chunks x self.chunk iterations of every start."""
        rc = _lib.muffin_multistart_run(self.h, int(chunks))
        if rc:
            raise MuffinError(rc, "muffin_multistart_run")

    def synchronize(self):
        self.torch.cuda.synchronize()

    def quality(self, truth):
        """Per start (SNR dB, WMSE) of Section 4.1 against the true sky."""
        self.views[0]._check(truth, self.views[0].cube, "truth")
        k = len(self.starts)
        snr, wmse = np.zeros(k), np.zeros(k)
        rc = _lib.muffin_multistart_quality(self.h, _ptr(truth),
                                            snr.ctypes.data_as(C.POINTER(C.c_double)),
                                            wmse.ctypes.data_as(C.POINTER(C.c_double)))
        if rc:
            raise MuffinError(rc, "muffin_multistart_quality")
        return snr, wmse

    def start(self, i: int) -> Muffin:
        return self.views[i]

    def close(self):
        if getattr(self, "h", None):
            for v in self.views:
                v.close()
            _lib.muffin_multistart_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Unmixer:
    """Spectral unmixing against k endmember spectra (muffin_unmix_*): per
    pixel, the non-negative least-squares abundances of Section 4.3."""

    def __init__(self, spectra):
        import torch
        self.torch = torch
        e = np.ascontiguousarray(spectra, dtype=np.float64)
        if e.ndim != 2:
            raise ValueError("spectra: (k, L) array")
        self.k, self.L = e.shape
        p = C.c_void_p()
        rc = _lib.muffin_unmix_plan_create(C.byref(p), e.ctypes.data_as(C.POINTER(C.c_double)),
                                           self.k, self.L)
        if rc:
            raise MuffinError(rc, "muffin_unmix_plan_create")
        self.h = p

    @staticmethod
    def spectra_at(cube, pixels):
        """Spectra of the cube at pixels [(i, j), ...] as a host (k, L)
        array (the paper picks them at bright pixels)."""
        return np.stack([cube[:, i, j].double().cpu().numpy() for i, j in pixels])

    def run(self, cube, residual: bool = False, stream=None):
        """cube: device (L, n, n) float32/float64 tensor.  Returns the
        abundances (k, n, n) (and the squared residual (n, n))."""
        torch = self.torch
        L, n, n2 = cube.shape
        if L != self.L or n != n2 or not cube.is_cuda or not cube.is_contiguous() \
                or cube.dtype not in (torch.float32, torch.float64):
            raise ValueError("cube: contiguous float32/float64 cuda tensor (L, n, n)")
        mode = F64 if cube.dtype == torch.float64 else F32
        a = torch.empty((self.k, n, n), dtype=cube.dtype, device=cube.device)
        r = torch.empty((n, n), dtype=cube.dtype, device=cube.device) if residual else None
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = _lib.muffin_unmix_run(self.h, _ptr(cube), n, mode, _ptr(a), _ptr(r),
                                   C.c_void_p(s.cuda_stream))
        if rc:
            raise MuffinError(rc, "muffin_unmix_run")
        return (a, r) if residual else a

    def close(self):
        if getattr(self, "h", None):
            _lib.muffin_unmix_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _vis_dev(a, torch):
    """Complex (L, K) or real (L, K, 2) host/device data -> contiguous device
    float64 (L, K, 2)."""
    if isinstance(a, np.ndarray):
        if np.iscomplexobj(a):
            a = np.stack([a.real, a.imag], axis=-1)
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")
    if a.is_complex():
        a = torch.view_as_real(a)
    return a.to(torch.float64).contiguous()


def vis_prepare(uv, vis, n: int, mode: int = F32, delta=None, stream=None):
    """Inputs of a visibility solve (muffin_vis_prepare): returns
    (dirty = Re H^* v, psf, delta_img = Re H^* delta or None, |v|^2).  uv:
    (L, K, 2) sample positions; vis, delta: complex (L, K)."""
    import torch
    u = _vis_dev(uv, torch)
    v = _vis_dev(vis, torch)
    d = _vis_dev(delta, torch) if delta is not None else None
    L, K = u.shape[0], u.shape[1]
    dt = torch.float64 if mode == F64 else torch.float32
    dirty = torch.empty((L, n, n), dtype=dt, device=u.device)
    psf = torch.empty((L, 2 * n, 2 * n), dtype=dt, device=u.device)
    dimg = torch.empty((L, n, n), dtype=dt, device=u.device) if d is not None else None
    nrm = C.c_double()
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _lib.muffin_vis_prepare(_ptr(u), _ptr(v), _ptr(d), L, K, n, int(mode), _ptr(dirty),
                                 _ptr(psf), _ptr(dimg), C.byref(nrm), C.c_void_p(s.cuda_stream))
    if rc:
        raise MuffinError(rc, "muffin_vis_prepare")
    return dirty, psf, dimg, nrm.value


def vis_degrid(uv, x, stream=None):
    """H x at the sample positions (muffin_vis_degrid): complex (L, K) tensor."""
    import torch
    u = _vis_dev(uv, torch)
    L, K = u.shape[0], u.shape[1]
    n = x.shape[-1]
    if x.dtype not in (torch.float32, torch.float64):
        raise ValueError("x: float32 or float64 cube")
    check_cube(x, (L, n, n), x.dtype, "x")
    mode = F64 if x.dtype == torch.float64 else F32
    out = torch.empty((L, K, 2), dtype=torch.float64, device=u.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _lib.muffin_vis_degrid(_ptr(u), L, K, n, int(mode), _ptr(x), _ptr(out),
                                C.c_void_p(s.cuda_stream))
    if rc:
        raise MuffinError(rc, "muffin_vis_degrid")
    return torch.view_as_complex(out)
