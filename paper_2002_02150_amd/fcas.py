"""Python binding of libfcas.so (the C ABI declared in include/fcas.h).

Argument marshalling only: every step of the fitness, gradient and swarm
update runs in the library's HIP kernels.  Device buffers are torch tensors on
the context's GPU; calls are enqueued on torch's current stream of that device.
If the library has not been built, every entry point raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcas.so")

MIXED = 0
FP64 = 1
SCHEDULE_FUSED = 0
SCHEDULE_TWO_PASS = 1
MAX_DET = 8

ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOSEG", -3: "EUNSUPPORTED_N", -4: "EHIP", -5: "ENOMEM", -6: "ECAPACITY"}

EXPORTED = ("fcas_create", "fcas_destroy", "fcas_workspace_bytes", "fcas_supported_n", "fcas_plan_count",
            "fcas_plan_info", "fcas_select_plan", "fcas_set_segment", "fcas_set_segment_range",
            "fitness_eval_batch", "fitness_eval_batch_static", "fitness_grad_batch", "fitness_polish", "pso_init",
            "pso_step", "pso_run", "pso_best", "pso_best_segments",
            "fcas_inject", "fcas_evaluated", "fcas_device_error", "fcas_set_timing", "fcas_read_timing", "fcas_last_error")


class FcasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Network(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32),
                ("pos_m", ctypes.c_double * 3 * MAX_DET),
                ("tensor", ctypes.c_double * 3 * 3 * MAX_DET)]


class _Config(ctypes.Structure):
    _fields_ = [("fs_hz", ctypes.c_double), ("f_low_hz", ctypes.c_double), ("f_high_hz", ctypes.c_double),
                ("precision", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("max_segments", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("max_samples", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("box_lo", ctypes.c_double * 4), ("box_hi", ctypes.c_double * 4)]


class _PsoParams(ctypes.Structure):
    _fields_ = [("n_runs", ctypes.c_int32), ("n_particles", ctypes.c_int32), ("n_iter", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("w0", ctypes.c_double), ("w1", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("vmax", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class _PsoState(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x", "v", "pbest_x", "pbest_f", "pbest_j", "best_x", "best_f", "best_j",
                                               "iteration")]


_lib = None


def library():
    """The loaded libfcas.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2002_02150_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "fcas_create": ([ctypes.POINTER(_Network), ctypes.POINTER(_Config), ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "fcas_destroy": ([vp], ctypes.c_int),
        "fcas_workspace_bytes": ([vp], ctypes.c_size_t),
        "fcas_supported_n": ([i64], ctypes.c_int),
        "fcas_plan_count": ([], ctypes.c_int),
        "fcas_plan_info": ([i32] + [ctypes.POINTER(i64)] + [ctypes.POINTER(i32)] * 6, ctypes.c_int),
        "fcas_select_plan": ([vp, i32, i32, i32], ctypes.c_int),
        "fcas_set_segment": ([vp, i32, i64, vp, vp, vp], ctypes.c_int),
        "fcas_set_segment_range": ([vp, i32, i64, i64], ctypes.c_int),
        "fitness_eval_batch": ([vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "fitness_eval_batch_static": ([vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "fitness_grad_batch": ([vp, i32, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "fitness_polish": ([vp, i32, vp, vp, i32, ctypes.c_double, i32, vp, vp, vp], ctypes.c_int),
        "pso_init": ([vp, ctypes.POINTER(_PsoParams), ctypes.POINTER(_PsoState), vp, vp], ctypes.c_int),
        "pso_step": ([vp, ctypes.POINTER(_PsoParams), ctypes.POINTER(_PsoState), vp, vp, vp, vp], ctypes.c_int),
        "pso_run": ([vp, ctypes.POINTER(_PsoParams), ctypes.POINTER(_PsoState), i32, vp, vp, vp, vp, vp],
                    ctypes.c_int),
        "pso_best": ([vp, ctypes.POINTER(_PsoParams), ctypes.POINTER(_PsoState), vp, vp, vp, vp, vp], ctypes.c_int),
        "pso_best_segments": ([vp, ctypes.POINTER(_PsoParams), ctypes.POINTER(_PsoState), i32, i32, vp, vp, vp, vp,
                               vp], ctypes.c_int),
        "fcas_inject": ([vp, i64, ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp, vp, vp], ctypes.c_int),
        "fcas_evaluated": ([vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "fcas_device_error": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "fcas_set_timing": ([vp, ctypes.c_int], ctypes.c_int),
        "fcas_read_timing": ([vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)], ctypes.c_int),
        "fcas_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise FcasError(rc, library().fcas_last_error().decode())


def supported_n(n: int) -> bool:
    return bool(library().fcas_supported_n(int(n)))


def plans():
    """[(plan, dict(n, n1, n2, e1, e2, cols, rows))] of every FFT plan."""
    lib = library()
    out = []
    for p in range(lib.fcas_plan_count()):
        n = ctypes.c_int64()
        v = [ctypes.c_int32() for _ in range(6)]
        _check(lib.fcas_plan_info(p, ctypes.byref(n), *[ctypes.byref(x) for x in v]))
        out.append((p, dict(n=n.value, n1=v[0].value, n2=v[1].value, e1=v[2].value, e2=v[3].value,
                            cols=v[4].value, rows=v[5].value)))
    return out


TUNING_PATH = os.path.join(_HERE, "tuning.json")


def load_tuning(path=TUNING_PATH):
    """The autotuner's choices {n_samples: {"plan", "grid1", "grid2"}} (empty if none)."""
    import json
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    return {int(k): v for k, v in data.get("choices", {}).items()}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _want(t, dtype, shape, device, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or tuple(t.shape) != tuple(shape) \
            or not t.is_contiguous() or t.device != device:
        raise ValueError(f"{name}: need a contiguous {dtype} tensor of shape {tuple(shape)} on {device}")


class Context:
    """A library context: network, band, search rectangle, precision, workspace."""

    def __init__(self, pos_m, tensor, fs, f_low, f_high, box_lo, box_hi, precision=MIXED, max_batch=320,
                 max_segments=1, max_samples=131072, workspace_bytes=0, device=0, schedule=SCHEDULE_TWO_PASS,
                 tuning="default"):
        lib = library()
        net = _Network()
        pos_m = [[float(v) for v in row] for row in pos_m]
        D = len(pos_m)
        net.n_det = D
        for i in range(min(D, MAX_DET)):
            for a in range(3):
                net.pos_m[i][a] = pos_m[i][a]
                for b in range(3):
                    net.tensor[i][a][b] = float(tensor[i][a][b])
        cfg = _Config(fs_hz=fs, f_low_hz=f_low, f_high_hz=f_high, precision=precision, max_batch=max_batch,
                      max_segments=max_segments, schedule=schedule, max_samples=max_samples,
                      workspace_bytes=workspace_bytes)
        for d in range(4):
            cfg.box_lo[d] = float(box_lo[d])
            cfg.box_hi[d] = float(box_hi[d])
        h = ctypes.c_void_p()
        _check(lib.fcas_create(ctypes.byref(net), ctypes.byref(cfg), int(device), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", int(device))
        self.n_det = D
        self.fs = fs
        self.precision = precision
        self.max_batch = max_batch
        self.box_lo = [float(v) for v in box_lo]
        self.box_hi = [float(v) for v in box_hi]
        self.seg_samples = {}
        if tuning is not None:
            for n, c in (load_tuning() if tuning == "default" else tuning).items():
                if n <= max_samples and precision == MIXED:
                    self.select_plan(c["plan"], c.get("grid1", 0), c.get("grid2", 0))

    def select_plan(self, plan, grid1=0, grid2=0):
        """Plan (and persistent grid sizes) for segments of its length registered from now on."""
        _check(library().fcas_select_plan(self._h, int(plan), int(grid1), int(grid2)))

    @classmethod
    def from_network(cls, net, **kw):
        return cls(net.pos_m, net.tensor, **kw)

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            library().fcas_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self):
        return library().fcas_workspace_bytes(self._h)

    def set_segment(self, seg_id, xf, psd):
        """xf: complex128 [D, N/2+1], psd: float64 [D, N/2+1] (device tensors)."""
        D, half = xf.shape
        n = 2 * (half - 1)
        _want(xf, torch.complex128, (self.n_det, half), self.device, "xf")
        _want(psd, torch.float64, (self.n_det, half), self.device, "psd")
        _check(library().fcas_set_segment(self._h, int(seg_id), n, _ptr(xf), _ptr(psd), _stream(self.device)))
        self.seg_samples[int(seg_id)] = n

    def set_segment_range(self, seg_id, j_lo, j_hi):
        """Search coalescence samples j_lo <= j < j_hi of segment seg_id only."""
        _check(library().fcas_set_segment_range(self._h, int(seg_id), int(j_lo), int(j_hi)))

    def _batch_args(self, theta, seg):
        n = theta.shape[0]
        _want(theta, torch.float64, (n, 4), self.device, "theta")
        _want(seg, torch.int32, (n,), self.device, "seg")
        return n

    def eval(self, theta, seg, fitness=None, argmax=None):
        n = self._batch_args(theta, seg)
        if fitness is None:
            fitness = torch.empty(n, dtype=torch.float64, device=self.device)
        if argmax is None:
            argmax = torch.empty(n, dtype=torch.int32, device=self.device)
        _want(fitness, torch.float64, (n,), self.device, "fitness")
        _want(argmax, torch.int32, (n,), self.device, "argmax")
        _check(library().fitness_eval_batch(self._h, n, _ptr(theta), _ptr(seg), _ptr(fitness), _ptr(argmax),
                                            _stream(self.device)))
        return fitness, argmax

    def eval_static(self, theta, seg, fitness, argmax):
        """fitness_eval_batch_static: as eval, into caller-provided outputs, with
        the call's scratch memory in the library's static per-GPU array (the
        call allocates nothing; calls on one GPU must not overlap)."""
        n = self._batch_args(theta, seg)
        _want(fitness, torch.float64, (n,), self.device, "fitness")
        _want(argmax, torch.int32, (n,), self.device, "argmax")
        _check(library().fitness_eval_batch_static(self._h, n, _ptr(theta), _ptr(seg), _ptr(fitness), _ptr(argmax),
                                                   _stream(self.device)))
        return fitness, argmax

    def grad(self, theta, seg, fitness=None, argmax=None, grad=None):
        n = self._batch_args(theta, seg)
        fitness = torch.empty(n, dtype=torch.float64, device=self.device) if fitness is None else fitness
        argmax = torch.empty(n, dtype=torch.int32, device=self.device) if argmax is None else argmax
        grad = torch.empty(n, 4, dtype=torch.float64, device=self.device) if grad is None else grad
        _want(grad, torch.float64, (n, 4), self.device, "grad")
        _check(library().fitness_grad_batch(self._h, n, _ptr(theta), _ptr(seg), _ptr(fitness), _ptr(argmax),
                                            _ptr(grad), _stream(self.device)))
        return fitness, argmax, grad

    def inject(self, xf, psd, alpha, delta, tau0, tau15, psi, phi_c, cos_iota, t_c, snr):
        """Adds an SPA signal (scaled to network SNR `snr`) to raw data xf in place."""
        D, half = xf.shape
        _want(xf, torch.complex128, (self.n_det, half), self.device, "xf")
        _want(psd, torch.float64, (self.n_det, half), self.device, "psd")
        prm = (ctypes.c_double * 8)(alpha, delta, tau0, tau15, psi, phi_c, cos_iota, t_c)
        _check(library().fcas_inject(self._h, 2 * (half - 1), prm, float(snr), _ptr(psd), _ptr(xf),
                                     _stream(self.device)))
        return xf

    def device_error(self):
        v = ctypes.c_int32(0)
        _check(library().fcas_device_error(self._h, ctypes.byref(v)))
        return v.value

    def evaluated(self):
        """Points evaluated by this context so far (synchronises)."""
        v = ctypes.c_uint64(0)
        _check(library().fcas_evaluated(self._h, ctypes.byref(v)))
        return v.value

    def set_timing(self, on: bool):
        _check(library().fcas_set_timing(self._h, 1 if on else 0))

    def read_timing(self, which):
        """(total ms, launches) of the FFT kernel `which` ("pass1", "passm",
        "pass2" or "fused") since timing was enabled; resets the record."""
        ms = ctypes.c_double(0)
        cnt = ctypes.c_int64(0)
        _check(library().fcas_read_timing(self._h, which.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


@dataclass
class PsoConfig:
    n_runs: int
    n_particles: int = 40
    n_iter: int = 2000
    w0: float = 0.9
    w1: float = 0.4
    c1: float = 2.0
    c2: float = 2.0
    vmax: float = 0.5
    seed: int = 1

    def _c(self):
        return _PsoParams(self.n_runs, self.n_particles, self.n_iter, 0, self.w0, self.w1, self.c1, self.c2,
                          self.vmax, self.seed)


class Swarm:
    """Device-resident lbest swarm state (Sec. III) driven by pso_init / pso_step / pso_best."""

    def __init__(self, ctx: Context, cfg: PsoConfig):
        self.ctx, self.cfg = ctx, cfg
        R, P, dev = cfg.n_runs, cfg.n_particles, ctx.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.x = torch.zeros(R, P, 4, **f64)
        self.v = torch.zeros(R, P, 4, **f64)
        self.pbest_x = torch.zeros(R, P, 4, **f64)
        self.pbest_f = torch.zeros(R, P, **f64)
        self.pbest_j = torch.zeros(R, P, dtype=torch.int32, device=dev)
        self.best_x = torch.zeros(R, 4, **f64)
        self.best_f = torch.zeros(R, **f64)
        self.best_j = torch.zeros(R, dtype=torch.int32, device=dev)
        self._iter = torch.zeros(2, dtype=torch.int32, device=dev)   # count, and pso_step's tally
        self.iteration = self._iter[:1]
        self.theta = torch.zeros(R * P, 4, **f64)
        self.out_f = torch.zeros(1, **f64)
        self.out_theta = torch.zeros(4, **f64)
        self.out_j = torch.zeros(1, dtype=torch.int32, device=dev)
        self.out_run = torch.zeros(1, dtype=torch.int32, device=dev)
        self._p = cfg._c()
        self._s = _PsoState(*[t.data_ptr() for t in (self.x, self.v, self.pbest_x, self.pbest_f, self.pbest_j,
                                                      self.best_x, self.best_f, self.best_j, self._iter)])

    @property
    def n(self):
        return self.cfg.n_runs * self.cfg.n_particles

    def init(self):
        _check(library().pso_init(self.ctx._h, ctypes.byref(self._p), ctypes.byref(self._s), _ptr(self.theta),
                                  _stream(self.ctx.device)))
        return self.theta

    def step(self, fitness, argmax):
        """One iteration; the iteration count is kept on the device."""
        _want(fitness, torch.float64, (self.n,), self.ctx.device, "fitness")
        _want(argmax, torch.int32, (self.n,), self.ctx.device, "argmax")
        _check(library().pso_step(self.ctx._h, ctypes.byref(self._p), ctypes.byref(self._s), _ptr(fitness),
                                  _ptr(argmax), _ptr(self.theta), _stream(self.ctx.device)))
        return self.theta

    def run(self, n_iter, seg, fitness, argmax):
        """pso_run: n_iter iterations (fitness of the current points, then the
        swarm update) on self.theta; fitness / argmax receive the last
        iteration's values."""
        _want(seg, torch.int32, (self.n,), self.ctx.device, "seg")
        _want(fitness, torch.float64, (self.n,), self.ctx.device, "fitness")
        _want(argmax, torch.int32, (self.n,), self.ctx.device, "argmax")
        _check(library().pso_run(self.ctx._h, ctypes.byref(self._p), ctypes.byref(self._s), int(n_iter),
                                 _ptr(self.theta), _ptr(seg), _ptr(fitness), _ptr(argmax), _stream(self.ctx.device)))
        return self.theta

    def best_segments(self, runs_per_segment, runs_used=None):
        """pso_best_segments: per segment g (runs g*m .. g*m + m - 1, m =
        runs_per_segment) the best of its first runs_used runs (default all):
        fitness, theta, coalescence sample and run index, as device tensors
        [n_seg], [n_seg, 4], [n_seg], [n_seg]."""
        m = int(runs_per_segment)
        u = m if runs_used is None else int(runs_used)
        g, dev = max(self.cfg.n_runs // max(m, 1), 1), self.ctx.device
        f = torch.empty(g, dtype=torch.float64, device=dev)
        th = torch.empty(g, 4, dtype=torch.float64, device=dev)
        j = torch.empty(g, dtype=torch.int32, device=dev)
        run = torch.empty(g, dtype=torch.int32, device=dev)
        _check(library().pso_best_segments(self.ctx._h, ctypes.byref(self._p), ctypes.byref(self._s), m, u,
                                           _ptr(f), _ptr(th), _ptr(j), _ptr(run), _stream(dev)))
        return f, th, j, run

    def best(self):
        _check(library().pso_best(self.ctx._h, ctypes.byref(self._p), ctypes.byref(self._s), _ptr(self.out_f),
                                  _ptr(self.out_theta), _ptr(self.out_j), _ptr(self.out_run),
                                  _stream(self.ctx.device)))
        return self.out_f, self.out_theta, self.out_j, self.out_run


class FitnessFn(torch.autograd.Function):
    """Gamma^2(theta) with its fixed-sample gradient: backward returns
    grad_output[:, None] * dGamma^2/dtheta, the maximising sample held fixed."""

    @staticmethod
    def forward(ctx_, theta, seg, fctx: Context):
        f, j, g = fctx.grad(theta.detach().contiguous(), seg)
        ctx_.save_for_backward(g)
        ctx_.mark_non_differentiable(j)
        return f, j

    @staticmethod
    def backward(ctx_, grad_f, grad_j):
        (g,) = ctx_.saved_tensors
        return grad_f[:, None] * g, None, None


def polish(fctx: Context, theta, seg, steps=20, step_frac=1e-3, trials=8, fitness=None, argmax=None):
    """Gradient ascent of Gamma^2 from the given points (fitness_polish): theta
    is updated in place; returns (theta, fitness, argmax) at the final points."""
    n = fctx._batch_args(theta, seg)
    fitness = torch.empty(n, dtype=torch.float64, device=fctx.device) if fitness is None else fitness
    argmax = torch.empty(n, dtype=torch.int32, device=fctx.device) if argmax is None else argmax
    _check(library().fitness_polish(fctx._h, n, _ptr(theta), _ptr(seg), int(steps), float(step_frac), int(trials),
                                    _ptr(fitness), _ptr(argmax), _stream(fctx.device)))
    return theta, fitness, argmax
