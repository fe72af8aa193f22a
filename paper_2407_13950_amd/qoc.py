"""Python binding of the C ABI in include/qoc.h (argument marshalling only).

Every computation runs in the HIP library libqoc.so; this module converts
numpy arrays / torch tensors into pointers, sizes and memory-kind flags.  It
raises ImportError when the library has not been built -- there is no other
code path.

Array conventions (same as the C ABI and the inputs module):
  alpha          float64 [d]
  window states  complex128 [M-1, E, N]  (W[m-1, c, :] is column c of W^m)
  grad_W         complex128 [M-1, E, N]  (real part dP/dRe W, imaginary part dP/dIm W)
  terms          float64 [4+M]: J, penalty, |U^M|^2, Re gamma, Im gamma, |C^m|^2 ...
Host (numpy / CPU tensor) inputs give host outputs and synchronous calls;
CUDA-tensor inputs give CUDA-tensor outputs written on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqoc.so")

QOC_OK, QOC_EINVAL, QOC_ENOMEM, QOC_EDEVICE, QOC_ENOTCONV, QOC_EUNSUPPORTED, QOC_ESTATE = 0, -1, -2, -3, -4, -5, -6
QOC_HOST, QOC_DEVICE = 0, 1
QOC_FP64, QOC_FP32 = 0, 1
QOC_BWD_AUTO, QOC_BWD_ONE_WAVE, QOC_BWD_TWO_WAVES, QOC_BWD_THREE_WAVES = 0, 1, 2, 3
SCHEDULES = {"auto": QOC_BWD_AUTO, "one_wave": QOC_BWD_ONE_WAVE, "two_waves": QOC_BWD_TWO_WAVES,
             "three_waves": QOC_BWD_THREE_WAVES}

EXPORTED = ["qoc_create", "qoc_destroy", "qoc_get_info", "qoc_set_stream", "qoc_set_controls",
            "qoc_set_window_states", "qoc_objective", "qoc_gradient", "qoc_rollout", "qoc_synchronize",
            "qoc_last_error", "qoc_strerror", "qoc_enable_timing", "qoc_get_timings", "qoc_backward",
            "qoc_batch_create", "qoc_batch_destroy", "qoc_batch_run", "qoc_read_results",
            "qoc_opt_create", "qoc_opt_destroy", "qoc_opt_run", "qoc_opt_get", "qoc_set_schedule",
            "qoc_get_schedule", "qoc_batch_status", "qoc_batch_gradient", "qoc_batch_run_noalloc"]

PHASES = ["controls", "forward", "boundary", "backward", "project", "grad_W", "total"]


class QocError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qoc error {code}: {msg}")
        self.code = code


class SystemDesc(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int32), ("n_levels", ctypes.c_int32),
        ("detuning", ctypes.c_void_p), ("anharmonicity", ctypes.c_void_p), ("cross_kerr", ctypes.c_void_p),
        ("n_carriers", ctypes.c_int32), ("carrier_freq", ctypes.c_void_p),
        ("n_splines", ctypes.c_int32), ("T", ctypes.c_double), ("n_steps", ctypes.c_int64),
        ("n_windows", ctypes.c_int32), ("mu", ctypes.c_double), ("target", ctypes.c_void_p),
        ("precision", ctypes.c_int32), ("fixed_point_iters", ctypes.c_int32), ("solve_tol", ctypes.c_double),
        ("checkpoint_every", ctypes.c_int32), ("device", ctypes.c_int32),
        ("dipole", ctypes.c_void_p),
    ]


class Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("E", ctypes.c_int32), ("d", ctypes.c_int32), ("n_windows", ctypes.c_int32),
                ("n_window_doubles", ctypes.c_int64), ("n_terms", ctypes.c_int32), ("lane_digits", ctypes.c_int32),
                ("columns_per_wave", ctypes.c_int32), ("device_bytes", ctypes.c_int64)]


class Timings(ctypes.Structure):
    _fields_ = [("n_calls", ctypes.c_int32), ("n_grad_calls", ctypes.c_int32), ("mean_ms", ctypes.c_double * 8),
                ("fixed_point_iters", ctypes.c_int32)]


class OptDesc(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("gamma_tik", ctypes.c_double), ("gamma_energy", ctypes.c_double),
                ("amp_bound", ctypes.c_double), ("memory", ctypes.c_int32), ("tol_estimate", ctypes.c_double),
                ("tol_grad", ctypes.c_double)]


class OptStatus(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("evaluations", ctypes.c_int32), ("backward_sweeps", ctypes.c_int32),
                ("stop", ctypes.c_int32), ("F", ctypes.c_double), ("P", ctypes.c_double), ("J", ctypes.c_double),
                ("penalty", ctypes.c_double), ("energy", ctypes.c_double), ("tikhonov", ctypes.c_double),
                ("estimate", ctypes.c_double), ("grad_inf", ctypes.c_double), ("last_step", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqoc.so (raises ImportError if it is missing).  QOC_LIBRARY_OVERRIDE names another
    build of the same library (e.g. one with sanitizers on its host code)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("QOC_LIBRARY_OVERRIDE") or path
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sigs = {
        "qoc_create": ([ctypes.POINTER(SystemDesc), ctypes.POINTER(vp)], ctypes.c_int),
        "qoc_destroy": ([vp], ctypes.c_int),
        "qoc_get_info": ([vp, ctypes.POINTER(Info)], ctypes.c_int),
        "qoc_set_stream": ([vp, vp], ctypes.c_int),
        "qoc_set_controls": ([vp, vp, i64, i32], ctypes.c_int),
        "qoc_set_window_states": ([vp, vp, i64, i32], ctypes.c_int),
        "qoc_objective": ([vp, vp, vp, i32], ctypes.c_int),
        "qoc_gradient": ([vp, vp, vp, vp, vp, i32], ctypes.c_int),
        "qoc_rollout": ([vp, vp, vp, i32], ctypes.c_int),
        "qoc_backward": ([vp, vp, vp, i32], ctypes.c_int),
        "qoc_batch_create": ([i32, i32, i64, ctypes.POINTER(vp)], ctypes.c_int),
        "qoc_batch_destroy": ([vp], ctypes.c_int),
        "qoc_batch_run": ([vp, ctypes.POINTER(vp), i32, vp, vp], ctypes.c_int),
        "qoc_read_results": ([vp, vp, vp, vp, vp, i32], ctypes.c_int),
        "qoc_synchronize": ([vp], ctypes.c_int),
        "qoc_last_error": ([], ctypes.c_char_p),
        "qoc_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "qoc_enable_timing": ([vp, i32], ctypes.c_int),
        "qoc_get_timings": ([vp, ctypes.POINTER(Timings)], ctypes.c_int),
        "qoc_opt_create": ([vp, ctypes.POINTER(OptDesc), vp, vp, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "qoc_opt_destroy": ([vp], ctypes.c_int),
        "qoc_opt_run": ([vp, i32, ctypes.POINTER(OptStatus)], ctypes.c_int),
        "qoc_opt_get": ([vp, vp, vp, i32], ctypes.c_int),
        "qoc_set_schedule": ([vp, i32], ctypes.c_int),
        "qoc_get_schedule": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "qoc_batch_status": ([vp, vp, i32], ctypes.c_int),
        "qoc_batch_gradient": ([ctypes.POINTER(vp), i32, vp], ctypes.c_int),
        "qoc_batch_run_noalloc": ([ctypes.POINTER(vp), i32, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != QOC_OK:
        raise QocError(rc, _lib.qoc_last_error().decode())


def _is_cuda(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


def _ptr_and_kind(x, dtype):
    """(pointer, kind, keepalive) for a numpy array or torch tensor of `dtype` ('f8' or 'c16')."""
    if hasattr(x, "data_ptr"):
        import torch
        want = torch.float64 if dtype == "f8" else torch.complex128
        if x.dtype != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), (QOC_DEVICE if x.is_cuda else QOC_HOST), x
    a = np.ascontiguousarray(x, dtype=np.float64 if dtype == "f8" else np.complex128)
    return a.ctypes.data, QOC_HOST, a


class System:
    """One system/context: qoc_create .. qoc_destroy."""

    def __init__(self, w, precision: str = "fp32", fixed_point_iters: int = 0, solve_tol: float = 0.0,
                 checkpoint_every: Optional[int] = None, device: int = 0, backward_schedule: str = "auto"):
        lib = load_library()
        self.w = w
        self._keep = [np.ascontiguousarray(w.detuning, dtype=np.float64),
                      np.ascontiguousarray(w.anharmonicity, dtype=np.float64),
                      np.ascontiguousarray(w.cross_kerr if w.q > 1 else np.zeros(1), dtype=np.float64),
                      np.ascontiguousarray(np.asarray(w.carriers).reshape(-1), dtype=np.float64),
                      np.ascontiguousarray(w.target, dtype=np.complex128),
                      np.ascontiguousarray(w.dipole_or_zero if w.q > 1 else np.zeros(1), dtype=np.float64)]
        k = self._keep
        ck = w.checkpoint_every if checkpoint_every is None else checkpoint_every
        dip = getattr(w, "dipole", None)
        self.desc = SystemDesc(w.q, w.L, k[0].ctypes.data, k[1].ctypes.data, k[2].ctypes.data, w.n_carriers,
                               k[3].ctypes.data, w.n_splines, w.T, w.n_steps, w.n_windows, w.mu, k[4].ctypes.data,
                               QOC_FP64 if precision == "fp64" else QOC_FP32, fixed_point_iters, solve_tol, ck, device,
                               k[5].ctypes.data if dip is not None else None)
        h = ctypes.c_void_p()
        _check(lib.qoc_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self.h = h
        self.precision = precision
        inf = Info()
        _check(lib.qoc_get_info(self.h, ctypes.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in Info._fields_}
        self.N, self.E, self.d, self.M = inf.N, inf.E, inf.d, inf.n_windows
        # Bumped by every call that changes the inputs or re-runs the forward sweep; the
        # autograd.Function compares it to detect that its forward state was replaced.
        self.generation = 0
        if backward_schedule != "auto":
            self.set_schedule(backward_schedule)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.qoc_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, device: bool):
        if device:
            import torch
            _check(_lib.qoc_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def set_stream(self, hip_stream_handle: int):
        _check(_lib.qoc_set_stream(self.h, ctypes.c_void_p(hip_stream_handle)))

    def set_controls(self, alpha):
        p, kind, keep = _ptr_and_kind(alpha, "f8")
        self._stream(kind == QOC_DEVICE)
        self.generation += 1
        _check(_lib.qoc_set_controls(self.h, p, self.d, kind))
        self._alpha_keep = keep

    def set_window_states(self, W):
        n = 2 * (self.M - 1) * self.N * self.E
        self.generation += 1
        if self.M == 1:
            _check(_lib.qoc_set_window_states(self.h, None, 0, QOC_HOST))
            return
        if tuple(W.shape) != (self.M - 1, self.E, self.N):
            raise ValueError(f"W must have shape {(self.M - 1, self.E, self.N)}")
        p, kind, keep = _ptr_and_kind(W, "c16")
        self._stream(kind == QOC_DEVICE)
        _check(_lib.qoc_set_window_states(self.h, p, n, kind))
        self._W_keep = keep

    def _outputs(self, device: bool, grad: bool):
        shapes = {"P": (1,), "terms": (4 + self.M,), "grad_alpha": (self.d,), "grad_W": (self.M - 1, self.E, self.N)}
        if device:
            import torch
            out = {k: torch.empty(v, dtype=torch.complex128 if k == "grad_W" else torch.float64, device="cuda")
                   for k, v in shapes.items() if grad or k in ("P", "terms")}
            ptr = {k: t.data_ptr() for k, t in out.items()}
        else:
            out = {k: np.empty(v, dtype=np.complex128 if k == "grad_W" else np.float64)
                   for k, v in shapes.items() if grad or k in ("P", "terms")}
            ptr = {k: a.ctypes.data for k, a in out.items()}
        if grad and self.M == 1:
            ptr["grad_W"] = None
        return out, ptr

    def objective(self, device: bool = False):
        """Returns (P, terms)."""
        self._stream(device)
        out, ptr = self._outputs(device, grad=False)
        self.generation += 1
        _check(_lib.qoc_objective(self.h, ptr["P"], ptr["terms"], QOC_DEVICE if device else QOC_HOST))
        return (out["P"] if device else float(out["P"][0])), out["terms"]

    def gradient(self, device: bool = False):
        """Returns (P, terms, grad_alpha, grad_W)."""
        self._stream(device)
        out, ptr = self._outputs(device, grad=True)
        self.generation += 1
        _check(_lib.qoc_gradient(self.h, ptr["P"], ptr["terms"], ptr["grad_alpha"], ptr["grad_W"],
                                 QOC_DEVICE if device else QOC_HOST))
        P = out["P"] if device else float(out["P"][0])
        return P, out["terms"], out["grad_alpha"], out["grad_W"]

    def gradient_into(self, P, terms, grad_alpha, grad_W):
        """Device-resident variant writing into caller tensors (no allocation, no sync)."""
        self._stream(True)
        self.generation += 1
        _check(_lib.qoc_gradient(self.h, P.data_ptr(), terms.data_ptr() if terms is not None else None,
                                 grad_alpha.data_ptr(), grad_W.data_ptr() if grad_W is not None else None, QOC_DEVICE))

    def backward(self, device: bool = False):
        """Adjoint sweep for the inputs of the last objective() call: (grad_alpha, grad_W)."""
        self._stream(device)
        out, ptr = self._outputs(device, grad=True)
        _check(_lib.qoc_backward(self.h, ptr["grad_alpha"], ptr["grad_W"], QOC_DEVICE if device else QOC_HOST))
        return out["grad_alpha"], out["grad_W"]

    def backward_into(self, grad_alpha, grad_W):
        self._stream(True)
        _check(_lib.qoc_backward(self.h, grad_alpha.data_ptr(), grad_W.data_ptr() if grad_W is not None else None,
                                 QOC_DEVICE))

    def objective_into(self, P, terms):
        self._stream(True)
        self.generation += 1
        _check(_lib.qoc_objective(self.h, P.data_ptr(), terms.data_ptr() if terms is not None else None, QOC_DEVICE))

    def rollout(self, device: bool = False):
        """Returns (W_rollout [M-1, E, N], U(T) [E, N]) under the current controls."""
        self._stream(device)
        if device:
            import torch
            W = torch.empty((max(self.M - 1, 0), self.E, self.N), dtype=torch.complex128, device="cuda")
            U = torch.empty((self.E, self.N), dtype=torch.complex128, device="cuda")
            _check(_lib.qoc_rollout(self.h, W.data_ptr() if self.M > 1 else None, U.data_ptr(), QOC_DEVICE))
        else:
            W = np.empty((max(self.M - 1, 0), self.E, self.N), dtype=np.complex128)
            U = np.empty((self.E, self.N), dtype=np.complex128)
            _check(_lib.qoc_rollout(self.h, W.ctypes.data if self.M > 1 else None, U.ctypes.data, QOC_HOST))
        return W, U

    def synchronize(self):
        _check(_lib.qoc_synchronize(self.h))

    def read_results(self, device: bool = False, grad: bool = True):
        """(P, terms, grad_alpha, grad_W) of the last evaluation (e.g. a batched one)."""
        out, ptr = self._outputs(device, grad=grad)
        _check(_lib.qoc_read_results(self.h, ptr["P"], ptr["terms"], ptr.get("grad_alpha"), ptr.get("grad_W"),
                                     QOC_DEVICE if device else QOC_HOST))
        P = out["P"] if device else float(out["P"][0])
        return P, out["terms"], out.get("grad_alpha"), out.get("grad_W")

    def read_results_into(self, P, terms, grad_alpha, grad_W):
        ptr = lambda t: t.data_ptr() if t is not None else None
        _check(_lib.qoc_read_results(self.h, ptr(P), ptr(terms), ptr(grad_alpha), ptr(grad_W), QOC_DEVICE))

    def enable_timing(self, on: bool = True):
        _check(_lib.qoc_enable_timing(self.h, 1 if on else 0))

    def set_schedule(self, backward: str = "auto"):
        """Backward-sweep schedule: "auto", "one_wave", "two_waves" or "three_waves" (qoc_set_schedule)."""
        if backward not in SCHEDULES:
            raise ValueError(f"unknown backward schedule {backward!r}; expected one of {sorted(SCHEDULES)}")
        _check(_lib.qoc_set_schedule(self.h, SCHEDULES[backward]))

    def schedule(self) -> str:
        """The backward schedule in force, with "auto" resolved."""
        v = ctypes.c_int32()
        _check(_lib.qoc_get_schedule(self.h, ctypes.byref(v)))
        return {QOC_BWD_ONE_WAVE: "one_wave", QOC_BWD_TWO_WAVES: "two_waves",
                QOC_BWD_THREE_WAVES: "three_waves"}[v.value]

    def schedules(self):
        """The backward schedules this system's layout offers."""
        return ["one_wave", "two_waves", "three_waves"] if self.info["columns_per_wave"] == 1 else ["one_wave", "two_waves"]

    def timings(self):
        """Mean kernel ms per phase over the evaluations recorded since enable_timing()."""
        t = Timings()
        _check(_lib.qoc_get_timings(self.h, ctypes.byref(t)))
        out = {name: t.mean_ms[i] for i, name in enumerate(PHASES)}
        out.update(n_calls=t.n_calls, n_grad_calls=t.n_grad_calls, fixed_point_iters=t.fixed_point_iters)
        return out


class Batch:
    """Batched evaluation of several Systems: one launch per phase for all of them (qoc_batch_*)."""

    def __init__(self, max_contexts: int, max_items: int, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.qoc_batch_create(device, max_contexts, max_items, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.qoc_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, systems, want_grad=None, stream: Optional[int] = None):
        """Evaluate all systems (their current inputs) asynchronously on `stream` (default: torch's current)."""
        n = len(systems)
        arr = (ctypes.c_void_p * n)(*[s.h.value for s in systems])
        wg = None
        if want_grad is not None:
            self._wg = (ctypes.c_int32 * n)(*[1 if g else 0 for g in want_grad])
            wg = ctypes.cast(self._wg, ctypes.c_void_p)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        for s in systems:
            s.generation += 1
        _check(_lib.qoc_batch_run(self.h, arr, n, wg, ctypes.c_void_p(stream)))
        self._n = n

    def status(self):
        """Per-system outcome of the last run (qoc_batch_status): QOC_OK or QOC_ENOTCONV each.
        Waits for the run's work to finish."""
        n = getattr(self, "_n", 0)
        st = (ctypes.c_int32 * max(n, 1))()
        _check(_lib.qoc_batch_status(self.h, ctypes.cast(st, ctypes.c_void_p), n))
        return [int(x) for x in st[:n]]


def batch_run_noalloc(systems, want_grad=None, stream: Optional[int] = None):
    """qoc_batch_run_noalloc: the batched evaluation with the library's static tables (no device
    allocation); asynchronous on `stream` (default: torch's current).  Read results with
    read_results; bound violations stay in each System (synchronize() reports them)."""
    n = len(systems)
    arr = (ctypes.c_void_p * n)(*[s.h.value for s in systems])
    wg = None
    if want_grad is not None:
        keep = (ctypes.c_int32 * n)(*[1 if g else 0 for g in want_grad])
        wg = ctypes.cast(keep, ctypes.c_void_p)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    for s in systems:
        s.generation += 1
    _check(_lib.qoc_batch_run_noalloc(arr, n, wg, ctypes.c_void_p(stream)))


def batch_gradient(systems, want_grad=None):
    """qoc_batch_gradient: evaluate all systems in one batched call and wait for it.  Raises
    QocError(QOC_ENOTCONV) when a system exceeded the fixed-point bound (the others' results
    stay valid; read them with read_results)."""
    n = len(systems)
    arr = (ctypes.c_void_p * n)(*[s.h.value for s in systems])
    wg = None
    if want_grad is not None:
        keep = (ctypes.c_int32 * n)(*[1 if g else 0 for g in want_grad])
        wg = ctypes.cast(keep, ctypes.c_void_p)
    for s in systems:
        s.generation += 1
    _check(_lib.qoc_batch_gradient(arr, n, wg))


STOP_REASONS = {0: "running", 1: "estimate", 2: "gradient", 3: "line search"}


class Optimizer:
    """Quadratic-penalty L-BFGS over a System (qoc_opt_*; iteration as specified in include/qoc.h).

    Defaults follow Sec. 5: sigma 0.1 (of the scanned 0.05..0.15), gamma_tik 1e-3/d, gamma_energy 1e-3,
    pulse amplitude bound 25 MHz, stop at a roll-out estimate of 1e-3.  W0=None starts from the
    roll-out of alpha0 (computed on the GPU).  The System belongs to the optimiser until close()."""

    def __init__(self, system: System, alpha0, W0=None, sigma: float = 0.1, gamma_tik: Optional[float] = None,
                 gamma_energy: float = 1e-3, amp_bound: float = 0.025, memory: int = 10,
                 tol_estimate: float = 1e-3, tol_grad: float = 0.0):
        lib = load_library()
        self.system = system
        self.desc = OptDesc(sigma, (1e-3 / system.d) if gamma_tik is None else gamma_tik, gamma_energy, amp_bound,
                            memory, tol_estimate, tol_grad)
        a = np.ascontiguousarray(alpha0, dtype=np.float64)
        Wp = None
        if W0 is not None and system.M > 1:
            Wk = np.ascontiguousarray(W0, dtype=np.complex128)
            if Wk.shape != (system.M - 1, system.E, system.N):
                raise ValueError(f"W0 must have shape {(system.M - 1, system.E, system.N)}")
            self._W0 = Wk
            Wp = Wk.ctypes.data
        h = ctypes.c_void_p()
        _check(lib.qoc_opt_create(system.h, ctypes.byref(self.desc), a.ctypes.data, Wp, QOC_HOST, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.qoc_opt_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n_iters: int) -> dict:
        """Up to n_iters iterations; returns the status of the current iterate."""
        st = OptStatus()
        _check(_lib.qoc_opt_run(self.h, n_iters, ctypes.byref(st)))
        out = {f: getattr(st, f) for f, _ in OptStatus._fields_}
        out["stop_reason"] = STOP_REASONS.get(st.stop, str(st.stop))
        return out

    def state(self):
        """(alpha [d], W [M-1, E, N] unscaled or None) of the current iterate, as numpy arrays."""
        s = self.system
        alpha = np.empty(s.d)
        W = np.empty((s.M - 1, s.E, s.N), dtype=np.complex128) if s.M > 1 else None
        _check(_lib.qoc_opt_get(self.h, alpha.ctypes.data, W.ctypes.data if W is not None else None, QOC_HOST))
        return alpha, W
