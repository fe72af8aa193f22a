"""Python face of the plain FP64 CPU oracle (qoc_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product path never imports it.  It shares no
code with the HIP library.  The arithmetic lives in qoc_oracle.c; this module
only marshals numpy arrays (layouts as in the inputs module: window states
[M-1, E, N] complex, target [E, E] column-major, alpha [d]).

Parity status: every function is pinned by tests/test_oracle_pins.py
(closed forms, invariants, brute-force dense references, central finite
differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qoc_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over windows x columns)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int), ("L", ctypes.c_int),
        ("detuning", ctypes.c_void_p), ("anharm", ctypes.c_void_p), ("cross_kerr", ctypes.c_void_p),
        ("nf", ctypes.c_int), ("carrier", ctypes.c_void_p),
        ("d1", ctypes.c_int), ("T", ctypes.c_double), ("n_steps", ctypes.c_long),
        ("M", ctypes.c_int), ("mu", ctypes.c_double), ("target", ctypes.c_void_p),
        ("dipole", ctypes.c_void_p),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("QOC_ORACLE_LIB_OVERRIDE")   # planted-mistake builds (tests only)
            if not path:
                if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                    build(force=True)
                path = LIB
            lib = ctypes.CDLL(path)
            P = ctypes.POINTER(_Problem)
            vp, i, l, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_double
            sig = {
                "orc_objective": [P, vp, vp, vp, vp],
                "orc_gradient": [P, vp, vp, vp, vp, vp, vp],
                "orc_windows": [P, vp, vp, i, i, vp, vp, vp, vp],
                "orc_rollout": [P, vp, vp, vp],
                "orc_drift": [P, vp],
                "orc_essential_rows": [P, vp],
                "orc_controls": [P, vp, dbl, vp],
                "orc_spline_values": [P, dbl, vp],
                "orc_apply_H": [P, vp, dbl, i, vp, vp],
                "orc_propagate": [P, vp, l, l, i, i, vp],
                "orc_infidelity": [P, vp, vp],
                "orc_energy": [P, vp, vp, vp],
                "orc_window_starts": [P, vp],
            }
            for name, args in sig.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            lib.orc_max_threads.argtypes = []
            lib.orc_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


class Problem:
    """A workload's system as the oracle sees it (keeps the arrays alive)."""

    def __init__(self, w):
        self.w = w
        self.q, self.L, self.N, self.E = w.q, w.L, w.N, w.E
        self.M, self.d = w.n_windows, w.d
        self._arrays = [
            np.ascontiguousarray(w.detuning, dtype=np.float64),
            np.ascontiguousarray(w.anharmonicity, dtype=np.float64),
            np.ascontiguousarray(w.cross_kerr if w.q > 1 else np.zeros(1), dtype=np.float64),
            np.ascontiguousarray(w.carriers.reshape(-1), dtype=np.float64),
            np.ascontiguousarray(w.target, dtype=np.complex128),
            np.ascontiguousarray(w.dipole_or_zero if w.q > 1 else np.zeros(1), dtype=np.float64),
        ]
        a = self._arrays
        self.s = _Problem(w.q, w.L, a[0].ctypes.data, a[1].ctypes.data, a[2].ctypes.data, w.n_carriers,
                          a[3].ctypes.data, w.n_splines, w.T, w.n_steps, w.n_windows, w.mu, a[4].ctypes.data,
                          a[5].ctypes.data if w.dipole is not None else None)

    def ref(self):
        return ctypes.byref(self.s)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _w_or_dummy(pb: Problem, W):
    if W is None or pb.M == 1:
        return np.zeros(2, dtype=np.complex128)
    W = _c(W, np.complex128)
    assert W.shape == (pb.M - 1, pb.E, pb.N), W.shape
    return W


def objective(w, alpha, W):
    """Returns (P, terms) with terms = [J, penalty, |U^M|^2, Re gamma, Im gamma, |C^m|^2 ...]."""
    pb = Problem(w)
    lib = _load()
    alpha = _c(alpha, np.float64)
    Wc = _w_or_dummy(pb, W)
    P = np.zeros(1)
    terms = np.zeros(4 + pb.M)
    _check(lib.orc_objective(pb.ref(), alpha.ctypes.data, Wc.ctypes.data, P.ctypes.data, terms.ctypes.data),
           "objective")
    return float(P[0]), terms


def gradient(w, alpha, W):
    """Returns (P, terms, grad_alpha [d], grad_W [M-1, E, N] complex: re = dP/dReW, im = dP/dImW)."""
    pb = Problem(w)
    lib = _load()
    alpha = _c(alpha, np.float64)
    Wc = _w_or_dummy(pb, W)
    P = np.zeros(1)
    terms = np.zeros(4 + pb.M)
    ga = np.zeros(pb.d)
    gW = np.zeros((max(pb.M - 1, 0), pb.E, pb.N), dtype=np.complex128)
    _check(lib.orc_gradient(pb.ref(), alpha.ctypes.data, Wc.ctypes.data, P.ctypes.data, terms.ctypes.data,
                            ga.ctypes.data, gW.ctypes.data), "gradient")
    return float(P[0]), terms, ga, gW


def windows(w, alpha, W, m0: int, m1: int, adjoint: bool = True):
    """Per-window pieces for windows m0..m1 (1-based, inclusive).

    Returns dict(Ufin [nw, E, N], pen [nw], lam0 [nw, E, N] or None, grad_alpha_part [d] or None).
    """
    pb = Problem(w)
    lib = _load()
    nw = m1 - m0 + 1
    alpha = _c(alpha, np.float64)
    Wc = _w_or_dummy(pb, W)
    Uf = np.zeros((nw, pb.E, pb.N), dtype=np.complex128)
    pen = np.zeros(nw)
    lam = np.zeros((nw, pb.E, pb.N), dtype=np.complex128) if adjoint else None
    ga = np.zeros(pb.d) if adjoint else None
    _check(lib.orc_windows(pb.ref(), alpha.ctypes.data, Wc.ctypes.data, m0, m1, Uf.ctypes.data, pen.ctypes.data,
                           lam.ctypes.data if adjoint else None, ga.ctypes.data if adjoint else None), "windows")
    return {"Ufin": Uf, "pen": pen, "lam0": lam, "grad_alpha_part": ga}


def rollout(w, alpha):
    """Returns (W_true [M-1, E, N], U_T [E, N]) from one propagation over [0, T] starting at W^0 = I."""
    pb = Problem(w)
    lib = _load()
    alpha = _c(alpha, np.float64)
    Wt = np.zeros((max(pb.M - 1, 1), pb.E, pb.N), dtype=np.complex128)
    UT = np.zeros((pb.E, pb.N), dtype=np.complex128)
    _check(lib.orc_rollout(pb.ref(), alpha.ctypes.data, Wt.ctypes.data, UT.ctypes.data), "rollout")
    return Wt[: pb.M - 1], UT


def drift(w) -> np.ndarray:
    pb = Problem(w)
    h = np.zeros(pb.N)
    _check(_load().orc_drift(pb.ref(), h.ctypes.data), "drift")
    return h


def essential_rows(w) -> np.ndarray:
    pb = Problem(w)
    rows = np.zeros(pb.E, dtype=np.int32)
    _check(_load().orc_essential_rows(pb.ref(), rows.ctypes.data), "essential_rows")
    return rows


def controls(w, alpha, t: float) -> np.ndarray:
    """c_j(t) = 2 pi d_j(t) for each qubit (complex [q])."""
    pb = Problem(w)
    out = np.zeros(pb.q, dtype=np.complex128)
    _check(_load().orc_controls(pb.ref(), _c(alpha, np.float64).ctypes.data, float(t), out.ctypes.data), "controls")
    return out


def spline_values(w, t: float) -> np.ndarray:
    pb = Problem(w)
    out = np.zeros(w.n_splines)
    _check(_load().orc_spline_values(pb.ref(), float(t), out.ctypes.data), "spline_values")
    return out


def apply_H(w, alpha, t: float, X) -> np.ndarray:
    """H(t) applied to columns X [ncol, N] (complex)."""
    pb = Problem(w)
    X = _c(np.atleast_2d(X), np.complex128)
    out = np.zeros_like(X)
    _check(_load().orc_apply_H(pb.ref(), _c(alpha, np.float64).ctypes.data, float(t), X.shape[0],
                               X.ctypes.data, out.ctypes.data), "apply_H")
    return out


def propagate(w, alpha, k0: int, k1: int, U, reverse: bool = False) -> np.ndarray:
    """Implicit-midpoint propagation of columns U [ncol, N] over steps k0..k1-1 (or backwards)."""
    pb = Problem(w)
    U = _c(np.atleast_2d(U), np.complex128).copy()
    _check(_load().orc_propagate(pb.ref(), _c(alpha, np.float64).ctypes.data, int(k0), int(k1),
                                 -1 if reverse else 1, U.shape[0], U.ctypes.data), "propagate")
    return U


def infidelity(w, U) -> float:
    """J_V(U) for U given as columns [E, N]."""
    pb = Problem(w)
    U = _c(U, np.complex128)
    assert U.shape == (pb.E, pb.N)
    J = np.zeros(1)
    _check(_load().orc_infidelity(pb.ref(), U.ctypes.data, J.ctypes.data), "infidelity")
    return float(J[0])


def energy(w, alpha, grad: bool = True):
    """Control energy Ee(alpha) = dt sum_k sum_j |d_j(t_{k+1/2})|^2 (GHz^2 ns) and its gradient [d]."""
    pb = Problem(w)
    E = np.zeros(1)
    g = np.zeros(w.d) if grad else None
    _check(_load().orc_energy(pb.ref(), _c(alpha, np.float64).ctypes.data, E.ctypes.data,
                              g.ctypes.data if grad else None), "energy")
    return (float(E[0]), g) if grad else float(E[0])


def window_starts(w) -> np.ndarray:
    pb = Problem(w)
    out = np.zeros(pb.M + 1, dtype=np.int64)
    _check(_load().orc_window_starts(pb.ref(), out.ctypes.data), "window_starts")
    return out


def max_threads() -> int:
    """OpenMP threads the oracle's (window, column) loops run on."""
    return int(_load().orc_max_threads())
