"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them retypes the oracle's
formulas: the references are scipy/numpy library routines (B-spline basis,
dense Kronecker operators, dense linear solves, eigh, expm, FFT), closed forms,
invariants and central finite differences.  A plausible slip in the oracle (a
dropped term, a wrong sign, index or operand order) breaks at least one test
here; tests/test_oracle_mutants.py plants such slips and checks that.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import dense_ref as D
from paper_2407_13950_amd import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(q=2, L=3, n_steps=60, M=3, d1=6, T=40.0, nf=2, **kw):
    """A small system with the synthetic drift (detuning, anharmonicity, cross-Kerr)."""
    w = WL.make_system("tiny", q, L, T, n_steps, M, d1)
    rng = np.random.default_rng(q * 100 + L)
    car = rng.uniform(-0.4, 0.4, size=(q, nf))
    w = w.replace(carriers=car, **kw)
    return w


def rand_alpha(w, seed, amp=0.02):
    return np.random.default_rng(seed).uniform(-amp, amp, w.d)


# ----------------------------------------------------------------------------- controls (Sec. 2)

def test_bspline_matches_scipy_basis(oracle_mod):
    """Quadratic cardinal B-splines (Sec. 2): B_s = scipy basis element on knots c_s + dtau*(-3/2..3/2)."""
    from scipy.interpolate import BSpline
    w = tiny(d1=9, T=70.0)
    dtau = w.T / (w.n_splines - 2)
    for t in np.linspace(0.0, w.T, 97):
        got = oracle_mod.spline_values(w, t)
        for s in range(w.n_splines):
            c = (s - 0.5) * dtau
            b = BSpline.basis_element(c + dtau * np.array([-1.5, -0.5, 0.5, 1.5]), extrapolate=False)(t)
            b = 0.0 if np.isnan(b) else b
            assert abs(got[s] - b) < 1e-14


def test_bspline_partition_of_unity_and_support(oracle_mod):
    """Cardinal quadratic B-splines sum to one on [0, T]; at most three are nonzero at any t."""
    w = tiny(d1=12, T=50.0)
    for t in np.linspace(0.0, w.T, 301):
        v = oracle_mod.spline_values(w, t)
        assert abs(v.sum() - 1.0) < 1e-14
        assert np.count_nonzero(v) <= 3
    dtau = w.T / (w.n_splines - 2)
    v = oracle_mod.spline_values(w, 2.5 * dtau)          # centre of s = 3
    assert abs(v[3] - 0.75) < 1e-15 and abs(v[2] - 0.125) < 1e-15
    v = oracle_mod.spline_values(w, 3.0 * dtau)          # knot between s = 3 and 4
    assert abs(v[3] - 0.5) < 1e-15 and abs(v[4] - 0.5) < 1e-15


@pytest.mark.parametrize("part", [0, 1])
def test_constant_envelope_gives_pure_carrier(oracle_mod, part):
    """eq. dj-ctrl with a constant envelope: d_j(t) = (a1 + i a2) exp(i Omega t) exactly (partition of unity)."""
    w = tiny(q=3, L=2, nf=3, d1=8, T=30.0)
    j, f, a = 1, 2, 0.0123
    alpha = np.zeros(w.d)
    for s in range(w.n_splines):
        alpha[((j * w.n_carriers + f) * 2 + part) * w.n_splines + s] = a
    for t in np.linspace(0.0, w.T, 23):
        c = oracle_mod.controls(w, alpha, t)
        expect = 2 * math.pi * a * (1j if part else 1.0) * np.exp(1j * w.carriers[j, f] * t)
        assert abs(c[j] - expect) < 1e-15
        assert np.all(np.abs(np.delete(c, j)) == 0.0)


def test_controls_match_direct_sum(oracle_mod):
    w = tiny(q=2, L=3, nf=2, d1=7)
    alpha = rand_alpha(w, 3)
    for t in np.linspace(0.0, w.T, 11):
        assert np.allclose(oracle_mod.controls(w, alpha, t), D.controls_ref(w, alpha, t), rtol=0, atol=1e-14)


# ----------------------------------------------------------------------------- Hamiltonian (Sec. 2)

@pytest.mark.parametrize("q,L", [(2, 3), (3, 2), (2, 4), (3, 3)])
def test_drift_matches_kronecker_number_operators(oracle_mod, q, L):
    w = tiny(q=q, L=L)
    Hd = D.drift_matrix(w)
    assert np.allclose(np.diag(Hd).real, oracle_mod.drift(w), rtol=0, atol=1e-14)
    assert np.count_nonzero(Hd - np.diag(np.diag(Hd))) == 0


@pytest.mark.parametrize("q,L", [(2, 3), (3, 2), (2, 4), (3, 3)])
def test_apply_H_matches_dense_kronecker(oracle_mod, q, L):
    """eqs. sys-ham/ctrl-ham: H = H_d + sum_j d_j a_j + conj(d_j) a_j^+, a_j = I x .. x a x .. x I."""
    w = tiny(q=q, L=L)
    alpha = rand_alpha(w, 5)
    t = 0.37 * w.T
    c = oracle_mod.controls(w, alpha, t)
    Hdense = D.drift_matrix(w) + D.control_matrix(w, c)
    assert np.allclose(Hdense, Hdense.conj().T)
    X = np.random.default_rng(1).standard_normal((5, w.N)) + 1j * np.random.default_rng(2).standard_normal((5, w.N))
    got = oracle_mod.apply_H(w, alpha, t, X)
    assert np.allclose(got, (Hdense @ X.T).T, rtol=0, atol=1e-13)
    # Hermitian as an operator: build the matrix column by column
    Hcols = oracle_mod.apply_H(w, alpha, t, np.eye(w.N, dtype=complex))
    assert np.allclose(Hcols.T, Hcols.T.conj().T, atol=1e-14)


def test_essential_rows_and_target_embedding(oracle_mod):
    for q, L in [(2, 3), (3, 4), (4, 4)]:
        w = WL.make_system("x", q, L, 10.0, 10, 1, 4)
        rows = oracle_mod.essential_rows(w)
        assert np.array_equal(rows, D.essential_rows_ref(q, L))


def test_qft_target_is_inverse_dft_and_unitary():
    """Sec. 5: V_jk = kappa^{jk}/sqrt(n), kappa = exp(2 pi i/n) equals sqrt(n) * ifft of the identity."""
    for E in (4, 8, 16):
        V = WL.qft_target(E).T
        assert np.allclose(V, np.fft.ifft(np.eye(E), axis=0) * math.sqrt(E), atol=1e-14)
        assert np.allclose(V.conj().T @ V, np.eye(E), atol=1e-14)


# ----------------------------------------------------------------------------- time stepping (Sec. 5)

def test_single_step_matches_dense_solve(oracle_mod):
    """Implicit midpoint: (I + i dt/2 H(t_k+1/2)) U_{k+1} = (I - i dt/2 H(t_k+1/2)) U_k, via numpy.linalg.solve."""
    w = tiny(q=2, L=3, n_steps=20, T=20.0)
    alpha = rand_alpha(w, 7, amp=0.05)
    U0 = np.random.default_rng(3).standard_normal((w.E, w.N)) + 0j
    k = 13
    dt = w.T / w.n_steps
    t = (k + 0.5) * dt
    H = D.drift_matrix(w) + D.control_matrix(w, D.controls_ref(w, alpha, t))
    expect = D.dense_step(H, dt, U0.T).T
    got = oracle_mod.propagate(w, alpha, k, k + 1, U0)
    assert np.allclose(got, expect, rtol=0, atol=1e-14)


def test_zero_control_is_cayley_power(oracle_mod):
    """Zero control, diagonal drift: each entry evolves by ((1 - i dt h/2)/(1 + i dt h/2))^K exactly."""
    w = tiny(q=2, L=4, n_steps=500, T=100.0)
    alpha = np.zeros(w.d)
    h = np.diag(D.drift_matrix(w)).real
    dt = w.T / w.n_steps
    U0 = np.random.default_rng(4).standard_normal((3, w.N)) + 1j * np.random.default_rng(5).standard_normal((3, w.N))
    got = oracle_mod.propagate(w, alpha, 0, w.n_steps, U0)
    cay = ((1 - 0.5j * dt * h) / (1 + 0.5j * dt * h)) ** w.n_steps
    assert np.allclose(got, U0 * cay[None, :], rtol=0, atol=1e-12)


def test_second_order_convergence_to_expm(oracle_mod):
    """The implicit midpoint rule is second order: halving dt divides the error against expm by 4."""
    w = tiny(q=2, L=3, T=30.0, nf=2)
    w = w.replace(carriers=np.zeros_like(w.carriers))          # constant H for a constant envelope
    alpha = np.zeros(w.d)
    for j in range(w.q):
        for s in range(w.n_splines):
            alpha[((j * w.n_carriers + 0) * 2 + 0) * w.n_splines + s] = 0.03 * (j + 1)
            alpha[((j * w.n_carriers + 1) * 2 + 1) * w.n_splines + s] = -0.02
    c = oracle_mod.controls(w, alpha, 1.0)
    H = D.drift_matrix(w) + D.control_matrix(w, c)
    U0 = np.eye(w.N, dtype=complex)[:, :4].T
    exact = (scipy.linalg.expm(-1j * H * w.T) @ U0.T).T
    errs = []
    for n in (200, 400, 800):
        wn = w.replace(n_steps=n)
        errs.append(np.abs(oracle_mod.propagate(wn, alpha, 0, n, U0) - exact).max())
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


def test_constant_hamiltonian_eigen_closed_form(oracle_mod):
    """Constant H: U_K = X diag(((1 - i dt l/2)/(1 + i dt l/2))^K) X^+ U_0 with H = X diag(l) X^+ (eigh)."""
    w = tiny(q=3, L=2, T=20.0, n_steps=300, nf=1)
    w = w.replace(carriers=np.zeros_like(w.carriers))
    alpha = np.zeros(w.d)
    for j in range(w.q):
        for s in range(w.n_splines):
            alpha[((j * 1 + 0) * 2 + 0) * w.n_splines + s] = 0.05 / (j + 1)
            alpha[((j * 1 + 0) * 2 + 1) * w.n_splines + s] = 0.01 * j
    H = D.drift_matrix(w) + D.control_matrix(w, oracle_mod.controls(w, alpha, 3.0))
    lam, X = np.linalg.eigh(H)
    dt = w.T / w.n_steps
    cay = ((1 - 0.5j * dt * lam) / (1 + 0.5j * dt * lam)) ** w.n_steps
    U0 = np.random.default_rng(6).standard_normal((2, w.N)) + 0j
    expect = (X @ np.diag(cay) @ X.conj().T @ U0.T).T
    assert np.allclose(oracle_mod.propagate(w, alpha, 0, w.n_steps, U0), expect, rtol=0, atol=1e-12)


def test_propagation_preserves_gram_matrix_and_is_reversible(oracle_mod):
    """S^m is unitary (Sec. 3): U^+U = W^+W; the rule is time-reversible (Sec. 5)."""
    w = tiny(q=2, L=3, n_steps=200, T=60.0)
    alpha = rand_alpha(w, 8, amp=0.05)
    W0 = np.random.default_rng(9).standard_normal((4, w.N)) + 1j * np.random.default_rng(10).standard_normal((4, w.N))
    U = oracle_mod.propagate(w, alpha, 20, 170, W0)
    assert np.allclose(U.conj() @ U.T, W0.conj() @ W0.T, rtol=0, atol=1e-12)
    back = oracle_mod.propagate(w, alpha, 20, 170, U, reverse=True)
    assert np.allclose(back, W0, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------- objective (Sec. 3)

def test_generalised_infidelity_properties(oracle_mod):
    """eq. mod-infid: J(V) = J(beta V) = 0; J >= 0 (Cauchy-Schwarz); J = G for an isometry; quadratic form."""
    w = WL.make_system("x", 2, 3, 10.0, 10, 1, 4)
    V = D.embedded_target(w)
    assert abs(oracle_mod.infidelity(w, V.T)) < 1e-15
    assert abs(oracle_mod.infidelity(w, (0.3 - 1.7j) * V.T)) < 1e-14
    rng = np.random.default_rng(11)
    vV = V.T.reshape(-1)
    Q = np.eye(vV.size) - np.outer(vV, vV.conj()) / w.E
    for _ in range(20):
        U = rng.standard_normal((w.E, w.N)) + 1j * rng.standard_normal((w.E, w.N))
        J = oracle_mod.infidelity(w, U)
        assert J >= 0.0
        vU = U.reshape(-1)
        assert abs(J - (np.vdot(vU, Q @ vU)).real / w.E) < 1e-12 * max(1.0, abs(J))
        Qr, _ = np.linalg.qr(U.T)                     # isometry: |U|_F^2 = E
        G = 1.0 - abs(np.vdot(V, Qr)) ** 2 / w.E ** 2
        assert abs(oracle_mod.infidelity(w, Qr.T) - G) < 1e-14


def test_window_split_is_floor(oracle_mod):
    for nT, M in [(4000, 4), (20000, 32), (100000, 128), (4000, 128), (37, 5)]:
        w = tiny(n_steps=nT, M=M)
        st = oracle_mod.window_starts(w)
        assert list(st) == D.window_starts_ref(w)
        lengths = np.diff(st)
        assert lengths.max() - lengths.min() <= 1 and st[-1] == nT


def test_penalty_vanishes_at_rollout_states(oracle_mod):
    """Constraints satisfied (eq. con0): penalty is exactly zero and P equals the roll-out infidelity."""
    w = tiny(q=2, L=3, n_steps=90, M=4, T=50.0)
    alpha = rand_alpha(w, 12, amp=0.03)
    Wt, UT = oracle_mod.rollout(w, alpha)
    P, terms = oracle_mod.objective(w, alpha, Wt)
    assert terms[1] == 0.0 and np.all(terms[5:] == 0.0)
    assert P == oracle_mod.infidelity(w, UT)
    w1 = w.replace(n_windows=1)                                   # M = 1: reduced-space objective
    P1, _ = oracle_mod.objective(w1, alpha, None)
    assert P1 == P


def test_dense_bruteforce_objective(oracle_mod):
    """The whole objective against dense Kronecker operators and dense solves."""
    w = tiny(q=2, L=3, n_steps=45, M=3, T=30.0)
    rng = np.random.default_rng(15)                      # non-symmetric unitary target
    Vr, _ = np.linalg.qr(rng.standard_normal((w.E, w.E)) + 1j * rng.standard_normal((w.E, w.E)))
    w = w.replace(target=np.ascontiguousarray(Vr.T))
    alpha = rand_alpha(w, 13, amp=0.04)
    W = WL.gen_random_states(w, 14)
    P, terms = oracle_mod.objective(w, alpha, W)
    Pd, Us = D.dense_objective(w, alpha, W)
    assert abs(P - Pd) < 1e-12 * abs(Pd)
    V = D.embedded_target(w)
    g = np.vdot(V, Us[-1])
    assert abs(terms[3] - g.real) < 1e-12 and abs(terms[4] - g.imag) < 1e-12


def test_rollout_estimate_bounds_rollout_infidelity(oracle_mod):
    """eq. rollout-infid-est: J(U_ro) <= J(U^M) + 2/sqrt(n) sqrt(J) sum|C^m| + (sum|C^m|)^2/n."""
    w = tiny(q=2, L=3, n_steps=80, M=5, T=40.0)
    for seed in range(6):
        alpha = rand_alpha(w, 20 + seed, amp=0.03)
        Wt, UT = oracle_mod.rollout(w, alpha)
        W = Wt + WL.gen_noise(w, seed, std=0.05 * (seed + 1))
        P, terms = oracle_mod.objective(w, alpha, W)
        J, Csum = terms[0], np.sqrt(terms[5:]).sum()
        est = J + 2 / math.sqrt(w.E) * math.sqrt(max(J, 0.0)) * Csum + Csum ** 2 / w.E
        assert oracle_mod.infidelity(w, UT) <= est + 1e-14


# ----------------------------------------------------------------------------- gradient (Sec. 3.1, App. B)

def _fd_check(oracle_mod, w, alpha, W, seed, count, h=1e-6, only=None):
    P, terms, ga, gW = oracle_mod.gradient(w, alpha, W)
    worst = 0.0
    for v in WL.gen_directions(w, seed, count):
        va, vw = v["alpha"], v["W"]
        if only == "alpha":
            vw = 0 * vw
        if only == "W":
            va = 0 * va
        Pp, _ = oracle_mod.objective(w, alpha + h * va, W + h * vw)
        Pm, _ = oracle_mod.objective(w, alpha - h * va, W - h * vw)
        fd = (Pp - Pm) / (2 * h)
        an = ga @ va + np.sum(gW.real * vw.real + gW.imag * vw.imag)
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    return worst


def test_gradient_matches_central_differences(oracle_mod):
    """discretize-then-optimize (Sec. 5): the adjoint gradient is the exact gradient of the discrete P."""
    w = tiny(q=2, L=3, n_steps=120, M=4, T=60.0, d1=8)
    alpha = rand_alpha(w, 30, amp=0.03)
    Wt, _ = oracle_mod.rollout(w, alpha)
    W = Wt + WL.gen_noise(w, 30, std=1e-2)
    assert _fd_check(oracle_mod, w, alpha, W, 31, 20) < 1e-7


@pytest.mark.parametrize("only", ["alpha", "W"])
def test_gradient_parts_match_central_differences(oracle_mod, only):
    """eq. grad-int for alpha; for W the factor 2 of eq. dT-dW-j (App. B)."""
    w = tiny(q=3, L=2, n_steps=90, M=3, T=45.0, d1=6)
    alpha = rand_alpha(w, 40, amp=0.03)
    W = WL.gen_random_states(w, 41)
    assert _fd_check(oracle_mod, w, alpha, W, 42, 8, only=only) < 1e-7


def test_single_window_gradient(oracle_mod):
    """M = 1 reverts to the reduced-space problem: gradient w.r.t. alpha only."""
    w = tiny(q=2, L=3, n_steps=100, M=1, T=50.0, d1=7)
    alpha = rand_alpha(w, 50, amp=0.03)
    P, terms, ga, gW = oracle_mod.gradient(w, alpha, None)
    assert gW.size == 0
    h = 1e-6
    for v in WL.gen_directions(w, 51, 6):
        Pp, _ = oracle_mod.objective(w, alpha + h * v["alpha"], None)
        Pm, _ = oracle_mod.objective(w, alpha - h * v["alpha"], None)
        an = ga @ v["alpha"]
        assert abs((Pp - Pm) / (2 * h) - an) < 1e-7 * max(abs(an), 1e-3)


def test_windows_pieces_sum_to_full_gradient(oracle_mod):
    """Per-window adjoint contributions add up to the full alpha-gradient (the sum over m in eq. grad-int)."""
    w = tiny(q=2, L=3, n_steps=80, M=4, T=40.0)
    alpha = rand_alpha(w, 60, amp=0.03)
    W = WL.gen_random_states(w, 61)
    P, terms, ga, gW = oracle_mod.gradient(w, alpha, W)
    a = oracle_mod.windows(w, alpha, W, 1, 2)
    b = oracle_mod.windows(w, alpha, W, 3, 4)
    assert np.allclose(a["grad_alpha_part"] + b["grad_alpha_part"], ga, rtol=1e-12, atol=1e-15)
    assert np.allclose(np.concatenate([a["pen"], b["pen"][:1]]), terms[5:], rtol=1e-14, atol=0)
    # W-gradient from per-window pieces: mu (W^m - U^m) - 2 Lambda^{m+1}(t_m)
    Uf = np.concatenate([a["Ufin"], b["Ufin"]])
    lam = np.concatenate([a["lam0"], b["lam0"]])
    gW2 = w.mu * (W - Uf[:3]) - 2 * lam[1:]
    assert np.allclose(gW2, gW, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------- paper tables

def test_golden_system_parameters_feed_the_workloads():
    """System-parameter table (Sec. 5): transition and carrier frequencies of QFT-4/8/16."""
    with open(os.path.join(GOLDEN, "systemparams.json")) as f:
        g = json.load(f)
    for key, mk in (("QFT-4", WL.c1), ("QFT-8", WL.c2), ("QFT-16", WL.c3)):
        row = g["cases"][key]
        w = mk()
        omega = np.array(row["omega_GHz"])
        assert np.allclose(w.detuning, 2 * math.pi * (omega - omega.mean()), atol=1e-15)
        for j, lst in enumerate(row["carriers_MHz"]):
            got = list(np.round(w.carriers[j] / (2 * math.pi) * 1e3, 6))
            assert got[: len(lst)] == lst
        assert w.E == row["n"]
