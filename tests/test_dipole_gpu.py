"""Parity of the dipole-coupled drift (eq. sys-ham, exchange terms of the chain) on the HIP path
with the FP64 oracle, through the C ABI.

The exchange terms keep the digit-sum parity, so the red-black solve takes them from the refreshed
colour's own values; the count bound includes them.  Cases cover every kernel instance family with
a coupling strong enough to matter (|J|/2pi up to 30 MHz, distinct per pair), the paper's QFT-4/8/16
systems (2 levels, J = 5 MHz) at their full step counts, the roll-out, batching with mixed variants,
forced counts and the optimisation driver.  Tolerances as in test_parity_gpu.py.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2407_13950_amd import qoc, workloads as WL

import test_parity_gpu as PG

pytestmark = pytest.mark.gpu


def rel(a, b):
    return PG.rel(a, b)


def with_dipole(w, seed, lo=0.01, hi=0.03):
    rng = np.random.default_rng([seed, 77])
    J = 2 * math.pi * rng.uniform(lo, hi, size=w.q - 1) * rng.choice([-1.0, 1.0], size=w.q - 1)
    return w.replace(dipole=J, name=w.name + "-J")


def dipole_case(q, L, n_steps, M, seed=1):
    w, _, _ = PG.small_case(q, L, n_steps, M, seed=seed)
    w = with_dipole(w, seed)
    alpha = WL.gen_alpha(w, seed)
    W = None
    if M > 1:
        Wt, _ = O.rollout(w, alpha)
        W = Wt + WL.gen_noise(w, seed)
    return w, alpha, W


CASES = [c for c in PG.CASES if c[0] >= 2]


@pytest.mark.parametrize("q,L,n_steps,M", CASES)
def test_fp64_with_dipole_matches_oracle(q, L, n_steps, M):
    w, alpha, W = dipole_case(q, L, n_steps, M)
    P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
    P, t, ga, gW = PG.run_gpu(w, alpha, W, "fp64")
    print(f"{w.name}: P={P:.15g} oracle={P0:.15g} alpha rel {rel(ga, ga0):.2e}", flush=True)
    assert abs(P - P0) <= 1e-11 * abs(P0)
    assert np.allclose(t, t0, rtol=1e-10, atol=1e-14)
    assert rel(ga, ga0) <= 1e-10
    if M > 1:
        assert rel(gW, gW0) <= 1e-10


@pytest.mark.parametrize("q,L,n_steps,M", CASES)
def test_fp32_with_dipole_matches_oracle(q, L, n_steps, M):
    w, alpha, W = dipole_case(q, L, n_steps, M)
    P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
    P, t, ga, gW = PG.run_gpu(w, alpha, W, "fp32")
    full = rel(np.concatenate([ga, gW.view(np.float64).ravel()]), np.concatenate([ga0, gW0.view(np.float64).ravel()]))
    print(f"{w.name}: P rel {abs(P - P0) / abs(P0):.2e}  grad rel-L2 {full:.2e}  alpha {rel(ga, ga0):.2e}",
          flush=True)
    assert abs(P - P0) <= 1e-5 * abs(P0)
    assert full <= 1e-4
    assert rel(ga, ga0) <= 1e-4


def test_dipole_changes_the_result_and_raises_the_count():
    """The coupling is really applied (P moves well beyond the tolerance) and the count bound grows."""
    w, alpha, W = dipole_case(4, 4, 240, 6)
    w0 = w.replace(dipole=None)
    out = {}
    for name, ww in (("J", w), ("0", w0)):
        s = qoc.System(ww, precision="fp64")
        s.set_controls(alpha)
        s.set_window_states(W)
        s.enable_timing(True)
        P, _ = s.objective()
        out[name] = (P, s.timings()["fixed_point_iters"])
        s.close()
    print(out, flush=True)
    assert abs(out["J"][0] - out["0"][0]) > 1e-6 * abs(out["0"][0])
    assert out["J"][1] >= out["0"][1]


def bound_count(w, alpha, W, prec):
    s = qoc.System(w, precision=prec)
    s.set_controls(alpha)
    s.set_window_states(W)
    s.enable_timing(True)
    s.objective()
    k = s.timings()["fixed_point_iters"]
    s.close()
    return k


@pytest.mark.parametrize("q,L,prec", [(4, 4, "fp32"), (3, 2, "fp32"), (4, 3, "fp64"), (4, 4, "fp64")])
def test_forced_counts_with_dipole_match_oracle(q, L, prec):
    """Counts forced by the caller at and above the bound's count, of both parities (for even L the
    last half sweep, which also takes the lane-digit inner products, is red or black)."""
    w, alpha, W = dipole_case(q, L, 200, 4)
    P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
    g0 = np.concatenate([ga0, gW0.view(np.float64).ravel()])
    tol_P, tol_g = (1e-11, 1e-10) if prec == "fp64" else (1e-5, 1e-4)
    k = bound_count(w, alpha, W, prec)
    for n in (k + 1, k + 2):
        P, t, ga, gW = PG.run_gpu(w, alpha, W, prec, fixed_point_iters=n)
        g = rel(np.concatenate([ga, gW.view(np.float64).ravel()]), g0)
        print(f"{w.name} {prec} count {n}: P rel {abs(P - P0) / abs(P0):.2e}  grad rel-L2 {g:.2e}", flush=True)
        assert abs(P - P0) <= tol_P * abs(P0) and g <= tol_g


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 3e-6)])
def test_rollout_with_dipole_matches_oracle(prec, tol):
    w, alpha, _ = dipole_case(3, 4, 400, 6)
    Wt0, U0 = O.rollout(w, alpha)
    s = qoc.System(w, precision=prec)
    s.set_controls(alpha)
    Wt, U = s.rollout()
    assert rel(Wt, Wt0) <= tol and rel(U, U0) <= tol
    s.close()


@pytest.mark.parametrize("q,M", [(2, 16), (3, 32), (4, 64)])
def test_paper_qft_systems_at_full_size(q, M):
    """The paper's QFT-4/8/16 systems (2 levels, J = 5 MHz, 190/500/900 ns, 2252/19806/106072 steps)
    with the paper's best window counts; start controls U(-10, 10) MHz, W = roll-out + noise."""
    w = WL.paper_qft(q, M)
    alpha = WL.gen_alpha(w, 5)
    Wt, _ = O.rollout(w, alpha)
    W = Wt + WL.gen_noise(w, 5)
    P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
    g0 = np.concatenate([ga0, gW0.view(np.float64).ravel()])
    for prec, tol_P, tol_g in (("fp64", 1e-11, 1e-10), ("fp32", 1e-5, 1e-4)):
        P, t, ga, gW = PG.run_gpu(w, alpha, W, prec)
        g = rel(np.concatenate([ga, gW.view(np.float64).ravel()]), g0)
        print(f"{w.name} M={M} {prec}: P rel {abs(P - P0) / abs(P0):.2e}  grad rel-L2 {g:.2e}", flush=True)
        assert abs(P - P0) <= tol_P * abs(P0) and g <= tol_g


def test_batch_with_mixed_variants_equals_solo():
    """One batched launch over contexts with and without the coupling equals the solo calls bit for bit."""
    ws = [dipole_case(4, 4, 160, 4, seed=2), dipole_case(3, 2, 150, 5, seed=3),
          PG.small_case(4, 4, 160, 4, seed=4), dipole_case(2, 3, 200, 3, seed=5)]
    systems = []
    for w, alpha, W in ws:
        s = qoc.System(w, precision="fp32")
        s.set_controls(torch.tensor(alpha, device="cuda"))
        s.set_window_states(torch.tensor(W, device="cuda"))
        systems.append(s)
    b = qoc.Batch(max_contexts=8, max_items=4096)
    b.run(systems)
    torch.cuda.synchronize()
    for (w, alpha, W), s in zip(ws, systems):
        Pb, tb, gab, gWb = s.read_results()
        P, t, ga, gW = PG.run_gpu(w, alpha, W, "fp32")
        assert Pb == P and np.array_equal(gab, ga) and np.array_equal(gWb, gW)
    for s in systems:
        s.close()
    b.close()


def test_optimizer_on_paper_qft4_follows_the_oracle():
    """The optimisation driver on the QFT-4 system (FP64 propagation) against the CPU version of the
    iteration on the oracle, iterate by iterate."""
    from oracle import lbfgs as LB
    import test_optimizer_gpu as TO
    w = WL.paper_qft(2, 16, n_steps=400)
    alpha0 = 2.0 * WL.gen_alpha(w, 3)
    pr = LB.PenaltyProblem(w)
    Wr, _ = O.rollout(w, np.clip(alpha0, -pr.amax, pr.amax))
    W0 = Wr + WL.gen_noise(w, 3, std=1e-2)
    st = TO.compare_run(w, alpha0, W0, pr, "fp64", iters=6, tol_F=1e-10, tol_x=1e-8)
    assert np.isfinite(st["F"])


def expected_count(w, alpha, prec, red_black):
    """The fixed-point count from its definition, computed independently of the library: the
    contraction bound rho = max_k nu_L sum_j (dt/2)|c_j(t_{k+1/2})| (nu_L = |a + a^+|_2, eigvalsh),
    beta = (dt/2) sum_j |J_j| |a^+ b + a b^+|_2, and the smallest count whose error bound meets the
    solve tolerance (Jacobi: (rho+beta)^(K+1); red-black: the per-colour recursion).  The solve
    is red-black when L is even and the layout keeps a register digit to colour."""
    L, dt = w.L, w.T / w.n_steps
    a = np.diag(np.sqrt(np.arange(1.0, L)), 1)
    nu_L = float(np.linalg.eigvalsh(a + a.T).max())
    nu_X = float(np.abs(np.linalg.eigvalsh(np.kron(a.T, a) + np.kron(a, a.T))).max())
    rho = 0.0
    for k in range(w.n_steps):
        c = O.controls(w, alpha, (k + 0.5) * dt)
        rho = max(rho, float(np.float32(0.5 * dt * float(np.sum(np.abs(c))) * nu_L)))
    rho *= 1.0 + 1e-6
    beta = 0.5 * dt * float(np.sum(np.abs(w.dipole_or_zero))) * nu_X
    tol = 2.0 ** (-54 if prec == "fp64" else -26)
    tau = rho + beta
    if not red_black:
        K, err = 1, tau * tau
        while err > tol and K < 64:
            err *= tau
            K += 1
        return K
    x0 = x1 = tau
    x0 = rho * x1 + beta * x0
    K, err = 1, math.hypot(x0, x1)
    while err > tol and K < 64:
        K += 1
        if K % 2:
            x0 = rho * x1 + beta * x0
        else:
            x1 = rho * x0 + beta * x1
        err = math.hypot(x0, x1)
    return K


@pytest.mark.parametrize("q,L,dip", [(3, 4, False), (3, 4, True), (2, 3, False), (2, 3, True), (3, 2, True)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_count_matches_its_definition(q, L, dip, prec):
    w, alpha, W = dipole_case(q, L, 240, 4) if dip else PG.small_case(q, L, 240, 4)
    alpha = 3.0 * alpha                                   # stronger controls: several counts apart
    k = bound_count(w, alpha, W, prec)
    s = qoc.System(w, precision=prec)
    red_black = w.L % 2 == 0 and s.info["lane_digits"] < w.q
    s.close()
    want = expected_count(w, alpha, prec, red_black)
    print(f"{w.name} {prec}: count {k} (definition {want})", flush=True)
    assert k == want
