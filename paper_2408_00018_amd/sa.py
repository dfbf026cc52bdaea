"""ctypes binding of the gfx950 annealing library (``include/sa.h``).

Argument marshalling only: every step of the annealing runs in the library's
HIP kernels.  PyTorch supplies the device workspace (a uint8 tensor) and the
HIP stream (the current torch stream).  If the built library is missing, or
no gfx950 device is present, the calls raise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsa_hip.so")

SCHWEFEL, RASTRIGIN, ACKLEY = 0, 1, 2
GRIEWANK, LEVY_MONTALVO, ROSENBROCK = 3, 4, 5  # non-separable: full re-evaluation per move
SHEKEL5, SHEKEL7, SHEKEL10, FOXHOLES, LANGERMAN = 6, 7, 8, 9, 10  # centre families (non-separable)
FP32, FP64 = 0, 1
MOVE_RADIUS, MOVE_RESAMPLE = 0, 1
FLAG_TRACE_X, FLAG_GRAPH, FLAG_LEARNED, FLAG_OVERLAY = 0x1, 0x2, 0x4, 0x8
FLAG_SOS, FLAG_BEST_SEEN, FLAG_ELITIST = 0x10, 0x20, 0x40  # exchange variants
FLAG_FULL_EVAL = 0x80  # separable families: f evaluated in full at every move
NET_RELU_CAUCHY, NET_GELU_GAUSS = 0, 1  # proposal network kinds
EXCHANGE_NEVER = 0xFFFFFFFF

SA_OK = 0
STATUS_NAMES = {0: "SA_OK", -1: "SA_ERR_INVALID", -2: "SA_ERR_NOMEM", -3: "SA_ERR_DEVICE", -4: "SA_ERR_STATE",
                -5: "SA_ERR_UNSUPPORTED"}

EXPORTED = ["sa_workspace_bytes", "sa_create", "sa_run", "sa_reset", "sa_levels_done", "sa_best", "sa_trace",
            "sa_move_log", "sa_set_start", "sa_set_proposal", "sa_set_network_kind", "sa_capture", "sa_capture_count",
            "sa_layout",
            "sa_destroy", "sa_last_error", "sa_run_static", "sa_nm_workspace_bytes", "sa_nm_polish",
            "sa_candidates"]


class SAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("func", ctypes.c_uint32), ("n", ctypes.c_uint32), ("lower", ctypes.c_void_p),
                ("upper", ctypes.c_void_p), ("shift", ctypes.c_void_p)]


class Config(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("chains", ctypes.c_uint32), ("levels", ctypes.c_uint32),
                ("steps", ctypes.c_uint32), ("precision", ctypes.c_uint32), ("move", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("T0", ctypes.c_double), ("alpha", ctypes.c_double),
                ("radius_frac", ctypes.c_double), ("log_chains", ctypes.c_uint32), ("log_level", ctypes.c_uint32),
                ("log_levels", ctypes.c_uint32), ("exchange", ctypes.c_uint32)]


LEVEL_DTYPE = np.dtype([("win_chain", np.uint32), ("reserved", np.uint32), ("f_win", np.float64),
                        ("f_best", np.float64), ("f_rec", np.float64), ("accepts", np.uint64),
                        ("t_ns", np.uint64)])
MOVE_DTYPE = np.dtype([("d", np.uint32), ("accept", np.uint32), ("x_old", np.float64), ("x_new", np.float64),
                       ("df", np.float64)])

_lib = None


class NMConfig(ctypes.Structure):
    _fields_ = [("maxiter", ctypes.c_uint32), ("log_steps", ctypes.c_uint32), ("ftol", ctypes.c_double),
                ("xtol", ctypes.c_double)]


def load_library():
    """Load libsa_hip.so (built by ``python -m paper_2408_00018_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2408_00018_amd.build first")
    # torch ships the HIP runtime this process uses; load it first so the
    # library binds to the same libamdhip64.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, st = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.sa_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]
    L.sa_workspace_bytes.restype = st
    L.sa_create.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Config), vp, vp, ctypes.c_size_t,
                            ctypes.POINTER(vp)]
    L.sa_create.restype = st
    L.sa_run.argtypes = [vp, u32]
    L.sa_run.restype = st
    L.sa_reset.argtypes = [vp, u64]
    L.sa_reset.restype = st
    L.sa_levels_done.argtypes = [vp, ctypes.POINTER(u32)]
    L.sa_levels_done.restype = st
    L.sa_best.argtypes = [vp, vp, vp, vp]
    L.sa_best.restype = st
    L.sa_trace.argtypes = [vp, u32, u32, vp, vp]
    L.sa_trace.restype = st
    L.sa_move_log.argtypes = [vp, vp, vp]
    L.sa_move_log.restype = st
    L.sa_set_start.argtypes = [vp, u32, vp]
    L.sa_set_start.restype = st
    L.sa_set_proposal.argtypes = [vp, vp, ctypes.c_float]
    L.sa_set_proposal.restype = st
    L.sa_set_network_kind.argtypes = [vp, ctypes.c_int]
    L.sa_set_network_kind.restype = st
    L.sa_capture.argtypes = [vp, vp, u64]
    L.sa_capture.restype = st
    L.sa_capture_count.argtypes = [vp, ctypes.POINTER(u64)]
    L.sa_capture_count.restype = st
    L.sa_layout.argtypes = [vp, vp, vp, vp]
    L.sa_layout.restype = st
    L.sa_destroy.argtypes = [vp]
    L.sa_destroy.restype = None
    L.sa_run_static.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Config), vp, vp, vp, vp]
    L.sa_run_static.restype = st
    L.sa_nm_workspace_bytes.argtypes = [ctypes.POINTER(Problem), u32, ctypes.POINTER(NMConfig),
                                        ctypes.POINTER(ctypes.c_size_t)]
    L.sa_nm_workspace_bytes.restype = st
    L.sa_nm_polish.argtypes = [ctypes.POINTER(Problem), vp, u32, ctypes.POINTER(NMConfig), vp, vp, ctypes.c_size_t,
                               vp, vp, vp, vp, vp]
    L.sa_nm_polish.restype = st
    L.sa_candidates.argtypes = [vp, u32, vp, vp, vp, ctypes.POINTER(u32)]
    L.sa_candidates.restype = st
    L.sa_last_error.argtypes = []
    L.sa_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != SA_OK:
        raise SAError(status, load_library().sa_last_error().decode())


@dataclass
class Schedule:
    """Annealing schedule and options (mirrors ``sa_config``)."""
    chains: int
    levels: int
    steps: int
    T0: float
    alpha: float
    seed: int = 0
    precision: int = FP32
    move: int = MOVE_RADIUS
    radius_frac: float = 0.1
    trace_x: bool = False
    graph: bool = False
    learned: bool = False  # reserve room for a learned proposal (sa_set_proposal)
    overlay: bool = False  # force the base-plus-overlay state layout
    log_chains: int = 0
    log_level: int = 0
    log_levels: int = 0
    # levels between broadcasts of the winner: 1 every level (synchronous),
    # k every k-th level (periodic exchange), 0 never (asynchronous)
    exchange: int = 1
    sos: bool = False        # stochastic exchange (SA_FLAG_SOS)
    best_seen: bool = False  # best-seen reduction (SA_FLAG_BEST_SEEN)
    elitist: bool = False    # broadcast the record instead of the winner (SA_FLAG_ELITIST)
    full_eval: bool = False  # full evaluation of f per move instead of the increment (SA_FLAG_FULL_EVAL)

    def to_c(self) -> Config:
        flags = ((FLAG_TRACE_X if self.trace_x else 0) | (FLAG_GRAPH if self.graph else 0) |
                 (FLAG_LEARNED if self.learned else 0) | (FLAG_OVERLAY if self.overlay else 0) |
                 (FLAG_SOS if self.sos else 0) | (FLAG_BEST_SEEN if self.best_seen else 0) |
                 (FLAG_ELITIST if self.elitist else 0) | (FLAG_FULL_EVAL if self.full_eval else 0))
        return Config(self.seed, self.chains, self.levels, self.steps, self.precision, self.move, flags, self.T0,
                      self.alpha, self.radius_frac, self.log_chains, self.log_level, self.log_levels,
                      EXCHANGE_NEVER if self.exchange == 0 else self.exchange)


def _problem_struct(func, lower, upper, shift):
    lo = np.ascontiguousarray(lower, dtype=np.float64)
    hi = np.ascontiguousarray(upper, dtype=np.float64)
    sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.float64)
    p = Problem(func, lo.size, lo.ctypes.data, hi.ctypes.data, None if sh is None else sh.ctypes.data)
    return p, (lo, hi, sh)


def workspace_bytes(func, lower, upper, shift, sched: Schedule) -> int:
    L = load_library()
    p, keep = _problem_struct(func, lower, upper, shift)
    cfg = sched.to_c()
    nbytes = ctypes.c_size_t()
    _check(L.sa_workspace_bytes(ctypes.byref(p), ctypes.byref(cfg), ctypes.byref(nbytes)))
    del keep
    return nbytes.value


def nm_polish(func, lower, upper, shift=None, *, x0, maxiter: int = 10000, ftol: float = 1e-12,
              xtol: float = 1e-10, log_steps: bool = False, stream=None):
    """Nelder-Mead polish of the start points x0 ([k, n] or [n]) on the
    device, one wave per start (``sa_nm_polish``).  Returns dict(x [k, n],
    f [k], iters [k], evals [k], steps [k, maxiter] or None)."""
    import torch
    L = load_library()
    p, keep = _problem_struct(func, lower, upper, shift)
    starts = np.ascontiguousarray(np.atleast_2d(np.asarray(x0, dtype=np.float64)))
    k, n = starts.shape
    assert n == p.n
    cfg = NMConfig(maxiter, 1 if log_steps else 0, ftol, xtol)
    s = stream if stream is not None else torch.cuda.current_stream()
    x = np.zeros((k, n))
    f = np.zeros(k)
    it = np.zeros(k, dtype=np.uint32)
    ev = np.zeros(k, dtype=np.uint32)
    steps = np.zeros((k, maxiter), dtype=np.uint8) if log_steps else None
    _check(L.sa_nm_polish(ctypes.byref(p), starts.ctypes.data, k, ctypes.byref(cfg), ctypes.c_void_p(s.cuda_stream),
                          None, 0, x.ctypes.data, f.ctypes.data, it.ctypes.data, ev.ctypes.data,
                          None if steps is None else steps.ctypes.data))
    del keep
    return dict(x=x, f=f, iters=it, evals=ev, steps=steps)


def run_static(func, lower, upper, shift=None, *, schedule: Schedule, stream=None):
    """One whole run through ``sa_run_static`` (no device allocation: the
    workspace is the library's static per-GPU scratch).  Returns the record
    (x_rec, f_rec, level) as ``Annealer.best`` does."""
    import torch
    L = load_library()
    p, keep = _problem_struct(func, lower, upper, shift)
    cfg = schedule.to_c()
    s = stream if stream is not None else torch.cuda.current_stream()
    x = np.zeros(p.n)
    f = ctypes.c_double()
    lvl = ctypes.c_uint32()
    _check(L.sa_run_static(ctypes.byref(p), ctypes.byref(cfg), ctypes.c_void_p(s.cuda_stream), x.ctypes.data,
                           ctypes.byref(f), ctypes.byref(lvl)))
    del keep
    return x, f.value, lvl.value


class Annealer:
    """One annealing problem on the current torch CUDA (HIP) device."""

    def __init__(self, func: int, lower, upper, shift=None, *, schedule: Schedule, stream=None,
                 torch_workspace: bool = True):
        import torch
        L = load_library()
        self.schedule = schedule
        self.n = int(np.asarray(lower).size)
        self.func = func
        self.lower = np.array(lower, dtype=np.float64)
        self.upper = np.array(upper, dtype=np.float64)
        self.shift = None if shift is None else np.array(shift, dtype=np.float64)
        p, keep = _problem_struct(func, lower, upper, shift)
        cfg = schedule.to_c()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if torch_workspace:
            nbytes = ctypes.c_size_t()
            _check(L.sa_workspace_bytes(ctypes.byref(p), ctypes.byref(cfg), ctypes.byref(nbytes)))
            self._ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
            ws_ptr, ws_bytes = self._ws.data_ptr(), nbytes.value
        ctx = ctypes.c_void_p()
        _check(L.sa_create(ctypes.byref(p), ctypes.byref(cfg), ctypes.c_void_p(self._stream.cuda_stream), ws_ptr,
                           ws_bytes, ctypes.byref(ctx)))
        del keep
        self._ctx = ctx

    @property
    def stream(self):
        return self._stream

    def run(self, levels: int = 0):
        _check(load_library().sa_run(self._ctx, levels))

    def reset(self, seed: int):
        _check(load_library().sa_reset(self._ctx, seed))

    def levels_done(self) -> int:
        v = ctypes.c_uint32()
        _check(load_library().sa_levels_done(self._ctx, ctypes.byref(v)))
        return v.value

    def best(self):
        x = np.zeros(self.n)
        f = ctypes.c_double()
        lvl = ctypes.c_uint32()
        _check(load_library().sa_best(self._ctx, x.ctypes.data, ctypes.byref(f), ctypes.byref(lvl)))
        return x, f.value, lvl.value

    def trace(self, first: int = 0, count: Optional[int] = None, with_x: bool = False):
        if count is None:
            count = self.levels_done() - first
        rec = np.zeros(count, dtype=LEVEL_DTYPE)
        xb = np.zeros((count, self.n)) if with_x else None
        _check(load_library().sa_trace(self._ctx, first, count, rec.ctypes.data,
                                       None if xb is None else xb.ctypes.data))
        return (rec, xb) if with_x else rec

    def set_start(self, level: int, x):
        """Start the run at ``level`` with every chain at ``x`` (before the first run)."""
        xx = np.ascontiguousarray(x, dtype=np.float64)
        assert xx.size == self.n
        _check(load_library().sa_set_start(self._ctx, level, xx.ctypes.data))

    def set_proposal(self, params, eps: float = 0.1):
        """Use the learned proposal with network ``params`` (None: plain moves)."""
        if params is None:
            _check(load_library().sa_set_proposal(self._ctx, None, 0.0))
            return
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_PARAMS
        _check(load_library().sa_set_proposal(self._ctx, p.ctypes.data, eps))

    def set_network_kind(self, kind: int):
        """Kind of network (NET_RELU_CAUCHY or NET_GELU_GAUSS) the learned
        levels evaluate and captures record features for."""
        _check(load_library().sa_set_network_kind(self._ctx, int(kind)))

    def capture(self, records):
        """Record accepted moves of later plain levels into ``records`` (a
        float32 CUDA tensor of shape [capacity, 7]); None stops capturing."""
        if records is None:
            _check(load_library().sa_capture(self._ctx, None, 0))
            self._cap = None
            return
        assert records.is_cuda and records.dtype.is_floating_point and records.element_size() == 4
        assert records.dim() == 2 and records.shape[1] == 7 and records.is_contiguous()
        self._cap = records
        _check(load_library().sa_capture(self._ctx, ctypes.c_void_p(records.data_ptr()), records.shape[0]))

    def candidates(self, k: int = 0):
        """The k lowest-cost candidates of the last level run (one per
        workgroup; k = 0: all of them), lowest first: (x [k, n], f [k]
        re-evaluated in FP64, chains [k])."""
        L = load_library()
        avail = ctypes.c_uint32()
        _check(L.sa_candidates(self._ctx, 0, None, None, None, ctypes.byref(avail)))
        k = avail.value if k == 0 else k
        x = np.zeros((k, self.n))
        f = np.zeros(k)
        ch = np.zeros(k, dtype=np.uint32)
        _check(L.sa_candidates(self._ctx, k, x.ctypes.data, f.ctypes.data, ch.ctypes.data, None))
        return x, f, ch

    def polish(self, k: int = 8, *, maxiter: int = 10000, ftol: float = 1e-12, xtol: float = 1e-10):
        """The hybrid strategy: Nelder-Mead from the record and the k - 1
        lowest-cost candidates of the last level, on the device; returns
        (x, f, start index) of the best polished point."""
        x_rec, _, _ = self.best()
        starts = [x_rec]
        if k > 1:
            cx, _, _ = self.candidates(0)
            starts.extend(cx[:k - 1])
        r = nm_polish(self.func, self.lower, self.upper, self.shift, x0=np.array(starts), maxiter=maxiter, ftol=ftol,
                      xtol=xtol, stream=self._stream)
        j = int(np.argmin(r["f"]))
        return r["x"][j], float(r["f"][j]), j

    def layout(self):
        """(lanes per workgroup, overlay slots per chain or 0, tiles)."""
        v = [ctypes.c_uint32() for _ in range(3)]
        _check(load_library().sa_layout(self._ctx, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def capture_count(self) -> int:
        v = ctypes.c_uint64()
        _check(load_library().sa_capture_count(self._ctx, ctypes.byref(v)))
        return v.value

    def move_log(self):
        s = self.schedule
        moves = np.zeros((s.log_levels, s.log_chains, s.steps), dtype=MOVE_DTYPE)
        final_f = np.zeros((s.log_levels, s.chains))
        _check(load_library().sa_move_log(self._ctx, moves.ctypes.data, final_f.ctypes.data))
        return moves, final_f

    def close(self):
        if getattr(self, "_ctx", None):
            load_library().sa_destroy(self._ctx)
            self._ctx = None
        self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Batched runs (sa_batch_* in include/sa.h)
# ---------------------------------------------------------------------------
EXPORTED_BATCH = ["sa_batch_workspace_bytes", "sa_batch_create", "sa_batch_run", "sa_batch_reset", "sa_batch_best",
                  "sa_batch_trace", "sa_batch_move_log", "sa_batch_layout", "sa_batch_destroy", "sa_batch_autotune",
                  "sa_batch_clock"]
EXPORTED = EXPORTED + EXPORTED_BATCH


class BatchConfig(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("levels", ctypes.c_uint32), ("steps", ctypes.c_uint32),
                ("precision", ctypes.c_uint32), ("move", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("waves_per_group", ctypes.c_uint32), ("T0", ctypes.c_double), ("alpha", ctypes.c_double),
                ("radius_frac", ctypes.c_double), ("log_problem", ctypes.c_uint32), ("log_chains", ctypes.c_uint32),
                ("log_level", ctypes.c_uint32), ("log_levels", ctypes.c_uint32)]


@dataclass
class BatchSchedule:
    """Schedule shared by every problem of a batch (mirrors ``sa_batch_config``)."""
    levels: int
    steps: int
    T0: float
    alpha: float
    seed: int = 0
    precision: int = FP32
    move: int = MOVE_RADIUS
    radius_frac: float = 0.1
    graph: bool = False
    trace_x: bool = False
    waves_per_group: int = 0
    log_problem: int = 0
    log_chains: int = 0
    log_level: int = 0
    log_levels: int = 0

    def to_c(self) -> BatchConfig:
        flags = (FLAG_GRAPH if self.graph else 0) | (FLAG_TRACE_X if self.trace_x else 0)
        return BatchConfig(self.seed, self.levels, self.steps, self.precision, self.move, flags,
                           self.waves_per_group, self.T0, self.alpha,
                           self.radius_frac, self.log_problem, self.log_chains, self.log_level, self.log_levels)


def _bind_batch(L):
    vp, u32, st = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
    P, C = ctypes.POINTER(Problem), ctypes.POINTER(BatchConfig)
    L.sa_batch_workspace_bytes.argtypes = [P, u32, vp, C, ctypes.POINTER(ctypes.c_size_t)]
    L.sa_batch_workspace_bytes.restype = st
    L.sa_batch_create.argtypes = [P, u32, vp, C, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.sa_batch_create.restype = st
    L.sa_batch_run.argtypes = [vp, u32]
    L.sa_batch_run.restype = st
    L.sa_batch_reset.argtypes = [vp, ctypes.c_uint64]
    L.sa_batch_reset.restype = st
    L.sa_batch_best.argtypes = [vp, u32, vp, vp, vp]
    L.sa_batch_best.restype = st
    L.sa_batch_trace.argtypes = [vp, u32, u32, u32, vp, vp]
    L.sa_batch_trace.restype = st
    L.sa_batch_move_log.argtypes = [vp, vp, vp]
    L.sa_batch_move_log.restype = st
    L.sa_batch_layout.argtypes = [vp, vp, vp, vp, vp]
    L.sa_batch_layout.restype = st
    L.sa_batch_destroy.argtypes = [vp]
    L.sa_batch_destroy.restype = None
    L.sa_batch_autotune.argtypes = [P, u32, C, vp, u32, vp, vp, vp]
    L.sa_batch_autotune.restype = st
    L.sa_batch_clock.argtypes = [vp, vp, u32, u32, vp]
    L.sa_batch_clock.restype = st


def _batch_lib():
    L = load_library()
    if not getattr(L, "_batch_bound", False):
        _bind_batch(L)
        L._batch_bound = True
    return L


def _problem_array(problems):
    """problems: sequence of (func, lower, upper, shift-or-None)."""
    arr = (Problem * len(problems))()
    keep = []
    for i, (func, lo, hi, sh) in enumerate(problems):
        p, k = _problem_struct(func, lo, hi, sh)
        arr[i] = p
        keep.append(k)
    return arr, keep


def batch_workspace_bytes(problems, chains, sched: BatchSchedule) -> int:
    L = _batch_lib()
    arr, keep = _problem_array(problems)
    ch = np.ascontiguousarray(chains, dtype=np.uint32)
    cfg = sched.to_c()
    nbytes = ctypes.c_size_t()
    _check(L.sa_batch_workspace_bytes(arr, len(problems), ch.ctypes.data, ctypes.byref(cfg), ctypes.byref(nbytes)))
    del keep
    return nbytes.value


def batch_autotune(problems, sched: BatchSchedule, trial_levels: int = 4, stream=None):
    """Measure candidate layouts on the device; returns (chains, waves_per_group, moves_per_s)."""
    import torch
    L = _batch_lib()
    arr, keep = _problem_array(problems)
    cfg = sched.to_c()
    chains = np.zeros(len(problems), dtype=np.uint32)
    wpg = ctypes.c_uint32()
    rate = ctypes.c_double()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(L.sa_batch_autotune(arr, len(problems), ctypes.byref(cfg), ctypes.c_void_p(st.cuda_stream), trial_levels,
                               chains.ctypes.data, ctypes.byref(wpg), ctypes.byref(rate)))
    del keep
    return chains, wpg.value, rate.value


class BatchAnnealer:
    """Many independent problems advancing together on the current device."""

    def __init__(self, problems, chains, *, schedule: BatchSchedule, stream=None, torch_workspace: bool = True):
        import torch
        L = _batch_lib()
        self.schedule = schedule
        self.ns = [int(np.asarray(p[1]).size) for p in problems]
        self.chains = np.ascontiguousarray(chains, dtype=np.uint32)
        arr, keep = _problem_array(problems)
        cfg = schedule.to_c()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if torch_workspace:
            nbytes = ctypes.c_size_t()
            _check(L.sa_batch_workspace_bytes(arr, len(problems), self.chains.ctypes.data, ctypes.byref(cfg),
                                              ctypes.byref(nbytes)))
            self._ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
            ws_ptr, ws_bytes = self._ws.data_ptr(), nbytes.value
        h = ctypes.c_void_p()
        _check(L.sa_batch_create(arr, len(problems), self.chains.ctypes.data, ctypes.byref(cfg),
                                 ctypes.c_void_p(self._stream.cuda_stream), ws_ptr, ws_bytes, ctypes.byref(h)))
        del keep
        self._h = h

    @property
    def stream(self):
        return self._stream

    def run(self, levels: int = 0):
        _check(_batch_lib().sa_batch_run(self._h, levels))

    def reset(self, seed: int):
        _check(_batch_lib().sa_batch_reset(self._h, seed))

    def best(self, prob: int):
        x = np.zeros(self.ns[prob])
        f = ctypes.c_double()
        lvl = ctypes.c_uint32()
        _check(_batch_lib().sa_batch_best(self._h, prob, x.ctypes.data, ctypes.byref(f), ctypes.byref(lvl)))
        return x, f.value, lvl.value

    def trace(self, prob: int, first: int = 0, count: Optional[int] = None, with_x: bool = False):
        if count is None:
            count = self.schedule.levels - first
        rec = np.zeros(count, dtype=LEVEL_DTYPE)
        xb = np.zeros((count, self.ns[prob])) if with_x else None
        _check(_batch_lib().sa_batch_trace(self._h, prob, first, count, rec.ctypes.data,
                                           None if xb is None else xb.ctypes.data))
        return (rec, xb) if with_x else rec

    def move_log(self):
        s = self.schedule
        moves = np.zeros((s.log_levels, s.log_chains, s.steps), dtype=MOVE_DTYPE)
        final_f = np.zeros((s.log_levels, int(self.chains[s.log_problem])))
        _check(_batch_lib().sa_batch_move_log(self._h, moves.ctypes.data, final_f.ctypes.data))
        return moves, final_f

    def layout(self):
        v = [ctypes.c_uint32() for _ in range(4)]
        _check(_batch_lib().sa_batch_layout(self._h, *[ctypes.byref(x) for x in v]))
        return dict(tiles=v[0].value, groups=v[1].value, waves_per_group=v[2].value, lds_bytes=v[3].value)

    def clock(self, ticks, first_level: int = 0, levels: int = 0) -> int:
        """Record each tile's start and end wall-clock ticks of levels
        [first_level, first_level + levels) of later runs into ``ticks`` (an
        int64 CUDA tensor [levels, tiles, 2]); None stops.  Returns the clock's
        ticks per second."""
        rate = ctypes.c_uint64()
        ptr = None
        if ticks is not None:
            assert ticks.is_cuda and ticks.element_size() == 8 and ticks.numel() >= levels * self.layout()["tiles"] * 2
            ptr = ctypes.c_void_p(ticks.data_ptr())
        _check(_batch_lib().sa_batch_clock(self._h, ptr, first_level, levels, ctypes.byref(rate)))
        return rate.value

    def close(self):
        if getattr(self, "_h", None):
            _batch_lib().sa_batch_destroy(self._h)
            self._h = None
        self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Learned proposal network trainer (sa_mlp_* in include/sa.h)
# ---------------------------------------------------------------------------
MLP_PARAMS = 17666
EXPORTED_MLP = ["sa_mlp_create", "sa_mlp_set_params", "sa_mlp_get_params", "sa_mlp_grad", "sa_mlp_train",
                "sa_mlp_infer", "sa_mlp_set_kind", "sa_mlp_destroy"]
EXPORTED = EXPORTED + EXPORTED_MLP


def _mlp_lib():
    L = load_library()
    if not getattr(L, "_mlp_bound", False):
        vp, u32, u64, st = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.sa_mlp_create.argtypes = [u32, vp, ctypes.POINTER(vp)]
        L.sa_mlp_create.restype = st
        L.sa_mlp_set_params.argtypes = [vp, vp]
        L.sa_mlp_set_params.restype = st
        L.sa_mlp_get_params.argtypes = [vp, vp]
        L.sa_mlp_get_params.restype = st
        L.sa_mlp_grad.argtypes = [vp, vp, u64, vp, u32, vp, vp]
        L.sa_mlp_grad.restype = st
        L.sa_mlp_train.argtypes = [vp, vp, u64, u32, u32, ctypes.c_float, u64, vp]
        L.sa_mlp_train.restype = st
        L.sa_mlp_infer.argtypes = [vp, vp, u32, vp]
        L.sa_mlp_infer.restype = st
        L.sa_mlp_set_kind.argtypes = [vp, ctypes.c_int]
        L.sa_mlp_set_kind.restype = st
        L.sa_mlp_destroy.argtypes = [vp]
        L.sa_mlp_destroy.restype = None
        L._mlp_bound = True
    return L


class MLPTrainer:
    """Trains the proposal network on captured records (a torch float32 tensor
    of shape [N, 7] on the device: 6 features, accepted scaled displacement)."""

    def __init__(self, max_batch: int = 4096, stream=None):
        import torch
        L = _mlp_lib()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.sa_mlp_create(max_batch, ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_PARAMS
        _check(_mlp_lib().sa_mlp_set_params(self._h, p.ctypes.data))

    def set_kind(self, kind: int):
        """Network kind (NET_RELU_CAUCHY or NET_GELU_GAUSS) of the forward
        pass, the loss and inference."""
        _check(_mlp_lib().sa_mlp_set_kind(self._h, int(kind)))

    def params(self):
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_mlp_lib().sa_mlp_get_params(self._h, p.ctypes.data))
        return p

    def grad(self, records, idx):
        """Gradient of the mean loss over records[idx] (idx host indices)."""
        assert records.is_cuda and records.dtype.is_floating_point and records.shape[1] == 7
        ix = np.ascontiguousarray(idx, dtype=np.uint32)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_mlp_lib().sa_mlp_grad(self._h, ctypes.c_void_p(records.data_ptr()), records.shape[0], ix.ctypes.data,
                                      ix.size, g.ctypes.data, ctypes.byref(loss)))
        return g, loss.value

    def train(self, records, batch: int, steps: int, lr: float = 1e-3, seed: int = 0):
        assert records.is_cuda and records.shape[1] == 7
        trace = np.zeros(steps, dtype=np.float32)
        _check(_mlp_lib().sa_mlp_train(self._h, ctypes.c_void_p(records.data_ptr()), records.shape[0], batch, steps,
                                       lr, seed, trace.ctypes.data))
        return trace

    def infer(self, Z):
        """(mu, s) at the current parameters for the rows of Z (a float32 CUDA
        tensor [rows, 6]); returns a float32 CUDA tensor [rows, 2]."""
        import torch
        assert Z.is_cuda and Z.dtype == torch.float32 and Z.dim() == 2 and Z.shape[1] == 6
        Zc = Z.contiguous()
        out = torch.empty((Zc.shape[0], 2), dtype=torch.float32, device=Zc.device)
        self._stream.wait_stream(torch.cuda.current_stream())
        _check(_mlp_lib().sa_mlp_infer(self._h, ctypes.c_void_p(Zc.data_ptr()), Zc.shape[0],
                                       ctypes.c_void_p(out.data_ptr())))
        self._stream.synchronize()
        return out

    def close(self):
        if getattr(self, "_h", None):
            _mlp_lib().sa_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)
