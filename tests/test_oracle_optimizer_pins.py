"""Pins of the oracle side of the optimisation driver (Sec. 3 penalty method with the Sec. 5 settings).

The control energy is checked against closed forms and central differences; the L-BFGS pieces
against the explicit BFGS inverse-Hessian recursion (Nocedal-Wright, the update the paper cites),
against closed-form minimisers of quadratics, and against scipy's independent L-BFGS-B on a
box-constrained quadratic.  The full objective F (penalty + Tikhonov + energy, scaled W) is
checked by central differences.
"""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import lbfgs as LB
from paper_2407_13950_amd import workloads as WL


def tiny(q=2, L=3, n_steps=60, M=3, d1=6, T=40.0, nf=2, **kw):
    w = WL.make_system("tiny", q, L, T, n_steps, M, d1)
    rng = np.random.default_rng(q * 100 + L)
    return w.replace(carriers=rng.uniform(-0.4, 0.4, size=(q, nf)), **kw)


def coef(w, j, f, part, s):
    return ((j * w.n_carriers + f) * 2 + part) * w.n_splines + s


# ----------------------------------------------------------------------------- control energy

def test_energy_of_a_constant_envelope_is_T_a_squared(oracle_mod):
    """One carrier with a constant envelope a (all splines, partition of unity): |d_j(t)| = a on [0, T]."""
    w = tiny(n_steps=137, T=53.0)
    a = 0.0123
    alpha = np.zeros(w.d)
    for s in range(w.n_splines):
        alpha[coef(w, 1, 0, 1, s)] = a          # imaginary part: |i a e^{iWt}| = a
    E, _ = oracle_mod.energy(w, alpha)
    assert abs(E - w.T * a * a) < 1e-15


def test_energy_of_two_carriers_matches_the_geometric_sum(oracle_mod):
    """|a e^{iW1 t} + b e^{iW2 t}|^2 = a^2 + b^2 + 2ab cos((W1-W2)t); the midpoint sum of the cosine
    over K steps is sin(K th)/(2 sin(th/2)) with th = (W1-W2) dt."""
    w = tiny(n_steps=211, T=47.0)
    a, b = 0.007, -0.004
    alpha = np.zeros(w.d)
    for s in range(w.n_splines):
        alpha[coef(w, 0, 0, 0, s)] = a
        alpha[coef(w, 0, 1, 0, s)] = b
    E, _ = oracle_mod.energy(w, alpha)
    dt = w.T / w.n_steps
    th = (w.carriers[0, 0] - w.carriers[0, 1]) * dt
    K = w.n_steps
    want = w.T * (a * a + b * b) + 2 * a * b * dt * math.sin(K * th) / (2 * math.sin(th / 2))
    assert abs(E - want) < 1e-15


def test_energy_gradient_matches_central_differences(oracle_mod):
    w = tiny(q=3, L=2, n_steps=90, T=35.0, d1=7)
    alpha = np.random.default_rng(3).uniform(-0.02, 0.02, w.d)
    E, g = oracle_mod.energy(w, alpha)
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(8):
        v = rng.standard_normal(w.d)
        v /= np.linalg.norm(v)
        fd = (oracle_mod.energy(w, alpha + h * v, grad=False) - oracle_mod.energy(w, alpha - h * v, grad=False)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-8 * max(1.0, abs(g @ v))


def test_energy_is_quadratic_in_alpha(oracle_mod):
    """Ee(c alpha) = c^2 Ee(alpha) and grad Ee(alpha) . alpha = 2 Ee(alpha) (Euler's theorem)."""
    w = tiny()
    alpha = np.random.default_rng(5).uniform(-0.02, 0.02, w.d)
    E, g = oracle_mod.energy(w, alpha)
    assert abs(oracle_mod.energy(w, 3.0 * alpha, grad=False) - 9.0 * E) < 1e-14
    assert abs(g @ alpha - 2.0 * E) < 1e-14


# ----------------------------------------------------------------------------- L-BFGS pieces

def explicit_inverse_hessian(pairs, n):
    s, y = pairs[-1]
    H = (s @ y) / (y @ y) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / (s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def test_two_loop_recursion_equals_the_explicit_bfgs_matrix():
    rng = np.random.default_rng(0)
    n = 7
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    pairs = []
    for _ in range(4):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s))
    g = rng.standard_normal(n)
    H = explicit_inverse_hessian(pairs, n)
    assert np.allclose(LB.two_loop(g, pairs), -H @ g, rtol=1e-12, atol=1e-13)


def test_bfgs_secant_equation_holds_for_the_newest_pair():
    rng = np.random.default_rng(1)
    n = 5
    pairs = [(rng.standard_normal(n), None) for _ in range(3)]
    A = np.diag(rng.uniform(1, 3, n))
    pairs = [(s, A @ s) for s, _ in pairs]
    s, y = pairs[-1]
    assert np.allclose(-LB.two_loop(y, pairs), s, rtol=1e-12, atol=1e-13)


def quad(A, b):
    return (lambda x: (0.5 * x @ A @ x - b @ x, {})), (lambda x: A @ x - b)


def test_minimize_finds_the_minimiser_of_a_convex_quadratic():
    rng = np.random.default_rng(2)
    n = 12
    A = rng.standard_normal((n, n))
    A = A @ A.T + np.eye(n)
    b = rng.standard_normal(n)
    f, g = quad(A, b)
    # (below |g| ~ 1e-9 the Armijo comparisons of F ~ 1 reach rounding level)
    hist = LB.minimize(f, g, np.zeros(n), 0, 1.0, 5, 300, stop=lambda info, gi: 2 if gi < 1e-8 else 0)
    assert hist[-1]["stop"] == 2 and len(hist) < 80
    assert np.allclose(hist[-1]["x"], np.linalg.solve(A, b), rtol=0, atol=1e-8)
    F = [h["F"] for h in hist]
    assert all(b_ <= a_ for a_, b_ in zip(F, F[1:]))      # Armijo: monotone


def test_minimize_matches_scipy_lbfgsb_on_a_box_constrained_quadratic():
    """Bounds on the first nb entries only; the KKT point from scipy's independent L-BFGS-B."""
    rng = np.random.default_rng(3)
    n, nb, amax = 10, 6, 0.3
    A = rng.standard_normal((n, n))
    A = A @ A.T + 0.5 * np.eye(n)
    b = 3.0 * rng.standard_normal(n)
    f, g = quad(A, b)
    hist = LB.minimize(f, g, rng.uniform(-0.1, 0.1, n), nb, amax, 6, 500,
                       stop=lambda info, gi: 2 if gi < 1e-7 else 0)
    assert hist[-1]["stop"] == 2
    x = hist[-1]["x"]
    ref = scipy.optimize.minimize(lambda z: f(z)[0], np.zeros(n), jac=g, method="L-BFGS-B",
                                  bounds=[(-amax, amax)] * nb + [(None, None)] * (n - nb),
                                  options=dict(ftol=1e-16, gtol=1e-12, maxiter=10000))
    assert np.allclose(x, ref.x, atol=1e-7)
    assert np.any(np.abs(x[:nb]) == amax)                    # the box is active
    assert np.all(np.abs(x[:nb]) <= amax)


def test_active_mask_marks_only_outward_gradients_at_bounds():
    x = np.array([-1.0, -1.0, 1.0, 1.0, 0.2, 5.0])
    g = np.array([1.0, -1.0, -1.0, 1.0, 3.0, 2.0])
    m = LB.active_mask(x, g, 5, -1.0, 1.0)
    assert m.tolist() == [True, False, True, False, False, False]


# ----------------------------------------------------------------------------- penalty problem

def test_penalty_problem_gradient_matches_central_differences(oracle_mod):
    """F = P(alpha, x_W / sigma) + Tikhonov + energy; gradient over (alpha, sigma W) by central differences."""
    w = tiny(q=2, L=3, n_steps=48, M=3)
    pr = LB.PenaltyProblem(w, sigma=0.13, gamma_tik=0.02, gamma_energy=0.5)
    alpha = np.random.default_rng(6).uniform(-0.01, 0.01, w.d)
    Wt, _ = oracle_mod.rollout(w, alpha)
    x = pr.pack(alpha, Wt + WL.gen_noise(w, 6, std=0.02))
    F, info = pr.fun(x)
    g = pr.grad(x).copy()
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(10):
        v = rng.standard_normal(x.size)
        v /= np.linalg.norm(v)
        fd = (pr.fun(x + h * v)[0] - pr.fun(x - h * v)[0]) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * max(1e-3, abs(g @ v))
    # the unscaled states round-trip
    a2, W2 = pr.unpack(x)
    assert np.array_equal(a2, alpha) and np.allclose(pr.pack(a2, W2), x, rtol=1e-15, atol=0)


def test_penalty_problem_box_bounds_the_pulse_amplitude(oracle_mod):
    """|alpha| <= A/(sqrt(2) nf) keeps |d_j(t)| <= A everywhere (Sec. 5: 25 MHz)."""
    w = tiny(n_steps=40)
    pr = LB.PenaltyProblem(w, amp_bound=0.025)
    alpha = np.where(np.random.default_rng(8).random(w.d) < 0.5, -pr.amax, pr.amax)
    worst = 0.0
    for t in np.linspace(0, w.T, 203):
        worst = max(worst, float(np.max(np.abs(oracle_mod.controls(w, alpha, t)))) / (2 * math.pi))
    assert worst <= 0.025 + 1e-15


def test_penalty_run_decreases_F_and_reports_the_rollout_estimate(oracle_mod):
    w = tiny(q=2, L=3, n_steps=60, M=3)
    pr = LB.PenaltyProblem(w)
    alpha = np.random.default_rng(9).uniform(-0.005, 0.005, w.d)     # inside the box
    Wt, _ = oracle_mod.rollout(w, alpha)
    hist = pr.run(alpha, Wt, max_iters=6, tol_estimate=0.0)
    F = [h["F"] for h in hist]
    assert len(hist) == 7 and all(b <= a for a, b in zip(F, F[1:])) and F[-1] < F[0]
    assert abs(hist[0]["info"]["estimate"] - hist[0]["info"]["J"]) < 1e-15   # roll-out states: C^m = 0
