"""Plain CPU version of the optimisation driver: the quadratic-penalty method of Sec. 3 with the
settings of Sec. 5 (L-BFGS, pulse-amplitude box, Tikhonov and control-energy terms, window states
scaled by sigma, the roll-out-estimate stopping rule of eq. rollout-infid-est), on the FP64 oracle.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to check the GPU driver iterate by iterate; the
product path never imports it.  It shares no code with the HIP library.  The iteration follows
the specification of the driver (projected L-BFGS, two-loop recursion, backtracking Armijo on the
projected step), written out plainly with numpy; `minimize` is generic so that it can be pinned on
problems with known minimisers.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

ARMIJO = 1e-4
MAX_HALVINGS = 30
CURVATURE = 1e-12


def rollout_estimate(J: float, window_norms2, E: int) -> float:
    """eq. rollout-infid-est: J + 2/sqrt(n) sqrt(J) sum|C^m| + (sum|C^m|)^2 / n, with n = E."""
    csum = float(np.sum(np.sqrt(np.maximum(np.asarray(window_norms2, dtype=float), 0.0))))
    return J + 2.0 / math.sqrt(E) * math.sqrt(max(J, 0.0)) * csum + csum * csum / E


def active_mask(x, g, nb: int, lo: float, hi: float):
    """Entries i < nb at a bound whose gradient points out of the box."""
    act = np.zeros(x.shape, dtype=bool)
    act[:nb] = ((x[:nb] <= lo) & (g[:nb] > 0)) | ((x[:nb] >= hi) & (g[:nb] < 0))
    return act


def two_loop(gr, pairs):
    """-H gr for the L-BFGS inverse-Hessian approximation of `pairs` [(s, y), ...] (oldest first),
    H0 = (s.y / y.y) I of the newest pair."""
    q = gr.copy()
    a = []
    for s, y in reversed(pairs):
        rho = 1.0 / float(s @ y)
        ai = rho * float(s @ q)
        q = q - ai * y
        a.append(ai)
    s, y = pairs[-1]
    q = (float(s @ y) / float(y @ y)) * q
    for (s, y), ai in zip(pairs, reversed(a)):
        rho = 1.0 / float(s @ y)
        b = rho * float(y @ q)
        q = q + (ai - b) * s
    return -q


def minimize(fun, grad, x0, nb: int, amax: float, memory: int, max_iters: int, stop=None):
    """Projected L-BFGS.  fun(x) -> (F, info); grad(x) -> g (at the last fun point); entries < nb of
    x are boxed to [-amax, amax].  stop(info, grad_inf) -> 0 (go on) or a stop code.  Returns the
    list of iterates as dicts (x, F, info, t, grad_inf, stop)."""
    lo, hi = -amax, amax
    x = np.array(x0, dtype=float)
    x[:nb] = np.clip(x[:nb], lo, hi)
    F, info = fun(x)
    g = grad(x)
    pairs = []
    hist = [dict(x=x.copy(), F=F, info=info, t=0.0, grad_inf=None, stop=0)]
    for _ in range(max_iters + 1):
        act = active_mask(x, g, nb, lo, hi)
        gr = np.where(act, 0.0, g)
        ginf = float(np.max(np.abs(gr))) if gr.size else 0.0
        hist[-1]["grad_inf"] = ginf
        code = stop(info, ginf) if stop else 0
        if code:
            hist[-1]["stop"] = code
            break
        if len(hist) > max_iters:
            break
        used = bool(pairs)
        p = two_loop(gr, pairs) if used else -gr
        p = np.where(act, 0.0, p)
        if not float(g @ p) < 0.0:
            pairs = []
            used = False
            p = -gr
        t = 1.0 if used else 1.0 / max(1.0, math.sqrt(float(gr @ gr)))
        accepted = False
        for _h in range(MAX_HALVINGS):
            xt = x + t * p
            xt[:nb] = np.clip(xt[:nb], lo, hi)
            Ft, info_t = fun(xt)
            if Ft <= F + ARMIJO * float(g @ (xt - x)):
                accepted = True
                break
            t *= 0.5
        if not accepted:
            hist[-1]["stop"] = 3
            break
        gt = grad(xt)
        s, y = xt - x, gt - g
        if float(s @ y) > CURVATURE * math.sqrt(float(s @ s) * float(y @ y)):
            pairs.append((s, y))
            if len(pairs) > memory:
                pairs.pop(0)
        x, g, F, info = xt, gt, Ft, info_t
        hist.append(dict(x=x.copy(), F=F, info=info, t=t, grad_inf=None, stop=0))
    return hist


class PenaltyProblem:
    """F(x) = P(alpha, W) + gamma_tik/2 |alpha|^2 + gamma_energy Ee(alpha) on x = [alpha, sigma W]
    (W interleaved re/im in the [M-1, E, N] layout), with the oracle's P, gradient and energy."""

    def __init__(self, w, sigma=0.1, gamma_tik=None, gamma_energy=1e-3, amp_bound=0.025):
        self.w = w
        self.sigma = sigma
        self.gamma_tik = 1e-3 / w.d if gamma_tik is None else gamma_tik
        self.gamma_energy = gamma_energy
        self.amax = amp_bound / (math.sqrt(2.0) * w.n_carriers)
        self.d = w.d
        self._last = None

    def pack(self, alpha, W):
        parts = [np.asarray(alpha, dtype=float)]
        if self.w.n_windows > 1:
            parts.append((self.sigma * np.ascontiguousarray(W, dtype=np.complex128)).view(np.float64).ravel())
        return np.concatenate(parts)

    def unpack(self, x):
        w = self.w
        alpha = x[:self.d].copy()
        if w.n_windows == 1:
            return alpha, None
        W = np.ascontiguousarray(x[self.d:]).view(np.complex128).reshape(w.n_windows - 1, w.E, w.N) * (1.0 / self.sigma)
        return alpha, W

    def fun(self, x):
        alpha, W = self.unpack(x)
        P, terms, ga, gW = O.gradient(self.w, alpha, W)
        En, gE = O.energy(self.w, alpha)
        tik = 0.5 * self.gamma_tik * float(alpha @ alpha)
        F = P + tik + self.gamma_energy * En
        g = ga + self.gamma_tik * alpha + self.gamma_energy * gE
        if self.w.n_windows > 1:
            g = np.concatenate([g, (np.ascontiguousarray(gW) * (1.0 / self.sigma)).view(np.float64).ravel()])
        self._last = (x.copy(), g)
        est = rollout_estimate(terms[0], terms[5:], self.w.E)
        return F, dict(P=P, J=terms[0], penalty=terms[1], energy=En, tikhonov=tik, estimate=est)

    def grad(self, x):
        assert self._last is not None and np.array_equal(self._last[0], x)
        return self._last[1]

    def run(self, alpha0, W0, max_iters, memory=10, tol_estimate=1e-3, tol_grad=0.0):
        def stop(info, ginf):
            if info["estimate"] < tol_estimate:
                return 1
            if tol_grad > 0 and ginf < tol_grad:
                return 2
            return 0
        return minimize(self.fun, self.grad, self.pack(alpha0, W0), self.d, self.amax, memory, max_iters, stop)
