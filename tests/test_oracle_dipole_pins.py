"""Pins of the oracle's dipole-coupled drift (eq. sys-ham: J_jk (A_k^+ A_j + A_k A_j^+) on the
nearest neighbours of the chain), against what the paper and the mathematics fix.

* The paper's carrier frequencies (Sec. 5, system-parameter table) are the transition
  frequencies of its coupled system: the single-excitation eigenvalues of H_s with the
  table's detunings and J = 5 MHz.  This fixes the size of J, which pairs it couples and that
  the 2-level model has no other off-diagonal static term.
* Dense Kronecker operators (numpy, independent of the oracle's index arithmetic), dense
  implicit-midpoint solves, a closed-form 2x2 Cayley power, conservation of the excitation
  number, unitarity and central finite differences of the gradient.
"""
import json
import math
import os

import numpy as np
import pytest

import dense_ref as D
from paper_2407_13950_amd import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def coupled(q=2, L=3, n_steps=60, M=3, d1=6, T=40.0, nf=2, seed=0):
    """A small system with the synthetic diagonal drift plus a dipole chain with distinct J per pair."""
    w = WL.make_system("tiny-dipole", q, L, T, n_steps, M, d1)
    rng = np.random.default_rng([q, L, seed])
    J = 2 * math.pi * rng.uniform(0.004, 0.02, size=q - 1) * rng.choice([-1.0, 1.0], size=q - 1)
    return w.replace(carriers=rng.uniform(-0.4, 0.4, size=(q, nf)), dipole=J)


def rand_alpha(w, seed, amp=0.02):
    return np.random.default_rng(seed).uniform(-amp, amp, w.d)


def full_H(oracle_mod, w, alpha, t):
    """H(t) as a matrix, column by column through the oracle's apply."""
    return oracle_mod.apply_H(w, alpha, t, np.eye(w.N, dtype=complex)).T


@pytest.mark.parametrize("q,L", [(2, 2), (3, 2), (4, 2), (2, 3), (3, 3), (2, 4)])
def test_apply_H_with_dipole_matches_dense_kronecker(oracle_mod, q, L):
    w = coupled(q=q, L=L)
    alpha = rand_alpha(w, 5)
    t = 0.41 * w.T
    c = oracle_mod.controls(w, alpha, t)
    H = D.static_matrix(w) + D.control_matrix(w, c)
    assert np.count_nonzero(D.dipole_matrix(w)) > 0
    assert np.allclose(full_H(oracle_mod, w, alpha, t), H, rtol=0, atol=1e-14)


@pytest.mark.parametrize("case,q", [("QFT-4", 2), ("QFT-8", 3), ("QFT-16", 4)])
def test_single_excitation_spectrum_gives_the_papers_carriers(oracle_mod, case, q):
    """Sec. 5: the carrier frequencies are the resonances of the coupled chain.  With the table's
    transition frequencies (rotating frame at their mean) and J = 5 MHz, the eigenvalues of H_s
    on the single-excitation states equal the set of printed carriers (to their printed digits)."""
    g = json.load(open(os.path.join(GOLDEN, "systemparams.json")))["cases"][case]
    w = WL.paper_qft(q, 1, n_steps=10)
    Hs = full_H(oracle_mod, w, np.zeros(w.d), 0.0)
    rows = [w.L ** (q - 1 - j) for j in range(q)]          # one excitation, on qubit j
    S = Hs[np.ix_(rows, rows)]
    lam_mhz = np.sort(np.linalg.eigvalsh(S)) / (2 * math.pi) * 1e3
    printed = np.array(sorted({f for lst in g["carriers_MHz"] for f in lst}))
    assert lam_mhz.shape == printed.shape
    assert np.max(np.abs(lam_mhz - printed)) < 0.02, (lam_mhz, printed)
    # no coupling out of the single-excitation block at zero control (excitation number conserved)
    others = [r for r in range(w.N) if r not in rows]
    assert np.count_nonzero(np.abs(Hs[np.ix_(others, rows)]) > 0) == 0


def test_two_level_pair_closed_form(oracle_mod):
    """Two 2-level qubits, zero control: |01>, |10> mix by the 2x2 block [[d1, J], [J, d0]];
    the implicit midpoint rule gives the Cayley power of its eigenvalues exactly.  Closed form:
    lambda = (d0+d1)/2 +- r, r = sqrt(((d0-d1)/2)^2 + J^2), eigenvectors (cos th, sin th) with
    tan(2 th) = 2J/(d1-d0) in the basis (|01>, |10>)."""
    w = WL.make_system("pair", 2, 2, 150.0, 1200, 1, 5, dipole_mhz=7.0, cross_kerr_ghz=0.0)
    w = w.replace(detuning=np.array([0.21, -0.13]))
    d0, d1 = w.detuning
    J = w.dipole[0]
    dt = w.T / w.n_steps
    K = w.n_steps

    def cay(lam):
        return ((1 - 0.5j * dt * lam) / (1 + 0.5j * dt * lam)) ** K

    a = 0.5 * (d1 - d0)
    r = math.hypot(a, J)
    th = 0.5 * math.atan2(J, a)
    ct, st = math.cos(th), math.sin(th)
    lp, lm = 0.5 * (d0 + d1) + r, 0.5 * (d0 + d1) - r
    # basis (|01>, |10>): rows 1 and 2; |01> has qubit 1 excited (energy d1), |10> qubit 0 (d0)
    B = np.array([[ct * ct * cay(lp) + st * st * cay(lm), ct * st * (cay(lp) - cay(lm))],
                  [ct * st * (cay(lp) - cay(lm)), st * st * cay(lp) + ct * ct * cay(lm)]])
    U0 = np.eye(4, dtype=complex)
    U = oracle_mod.propagate(w, np.zeros(w.d), 0, K, U0)        # rows: columns of U (state vectors)
    Um = U.T
    assert abs(Um[0, 0] - 1.0) < 1e-12                          # |00>: energy 0
    assert abs(Um[3, 3] - cay(d0 + d1)) < 1e-12                 # |11>: no exchange partner at L = 2
    assert np.allclose(Um[1:3, 1:3], B, rtol=0, atol=1e-12)
    assert abs(Um[1, 2]) > 0.1                                   # the pair really exchanges population


def test_exchange_conserves_excitation_number_and_norm(oracle_mod):
    """Zero control: H_s commutes with the total number operator, so the weight of every
    excitation sector is conserved; with control the propagation stays unitary."""
    w = coupled(q=3, L=3, n_steps=300, T=80.0, M=1)
    rng = np.random.default_rng(3)
    U0 = rng.standard_normal((4, w.N)) + 1j * rng.standard_normal((4, w.N))
    U = oracle_mod.propagate(w, np.zeros(w.d), 0, w.n_steps, U0)
    digits = np.array([[(r // w.L ** (w.q - 1 - j)) % w.L for j in range(w.q)] for r in range(w.N)])
    nexc = digits.sum(axis=1)
    for n in np.unique(nexc):
        sel = nexc == n
        assert np.allclose(np.sum(np.abs(U[:, sel]) ** 2, axis=1), np.sum(np.abs(U0[:, sel]) ** 2, axis=1),
                           rtol=1e-12, atol=0)
    assert np.abs(U - U0).max() > 0.1                       # the exchange moved amplitude within sectors
    alpha = rand_alpha(w, 4, amp=0.05)
    U = oracle_mod.propagate(w, alpha, 0, w.n_steps, U0)
    assert np.allclose(U.conj() @ U.T, U0.conj() @ U0.T, rtol=0, atol=1e-11)
    back = oracle_mod.propagate(w, alpha, 0, w.n_steps, U, reverse=True)
    assert np.allclose(back, U0, rtol=0, atol=1e-11)


def test_single_step_with_dipole_matches_dense_solve(oracle_mod):
    w = coupled(q=3, L=2, n_steps=20, T=20.0)
    alpha = rand_alpha(w, 7, amp=0.05)
    U0 = np.random.default_rng(3).standard_normal((w.E, w.N)) + 0j
    k = 11
    dt = w.T / w.n_steps
    t = (k + 0.5) * dt
    H = D.static_matrix(w) + D.control_matrix(w, D.controls_ref(w, alpha, t))
    expect = D.dense_step(H, dt, U0.T).T
    assert np.allclose(oracle_mod.propagate(w, alpha, k, k + 1, U0), expect, rtol=0, atol=1e-14)


def test_dense_bruteforce_objective_with_dipole(oracle_mod):
    w = coupled(q=2, L=3, n_steps=45, M=3, T=30.0)
    alpha = rand_alpha(w, 11, amp=0.03)
    W = WL.gen_random_states(w, 12)
    P, terms = oracle_mod.objective(w, alpha, W)
    P_ref, _ = D.dense_objective(w, alpha, W)
    assert abs(P - P_ref) <= 1e-12 * max(1.0, abs(P_ref))


def _fd_check(oracle_mod, w, alpha, W, seed, count):
    P, terms, ga, gW = oracle_mod.gradient(w, alpha, W)
    h = 1e-6
    worst = 0.0
    for d in WL.gen_directions(w, seed, count):
        va, vw = d["alpha"], d["W"]
        fp, _ = oracle_mod.objective(w, alpha + h * va, W + h * vw)
        fm, _ = oracle_mod.objective(w, alpha - h * va, W - h * vw)
        fd = (fp - fm) / (2 * h)
        an = ga @ va + np.sum(gW.real * vw.real + gW.imag * vw.imag)
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    return worst


@pytest.mark.parametrize("q,L", [(2, 3), (3, 2)])
def test_gradient_with_dipole_matches_central_differences(oracle_mod, q, L):
    """The discrete adjoint uses the same H (Hermitian, with the exchange term) in its solves."""
    w = coupled(q=q, L=L, n_steps=90, M=3, T=45.0)
    w = w.replace(dipole=w.dipole * 4.0)                 # strong enough to matter over 45 ns
    alpha = rand_alpha(w, 30, amp=0.03)
    Wt, _ = oracle_mod.rollout(w, alpha)
    W = Wt + WL.gen_noise(w, 30, std=1e-2)
    assert _fd_check(oracle_mod, w, alpha, W, 31, 10) < 1e-7
