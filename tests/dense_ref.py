"""Brute-force dense references for tiny systems (test helper, numpy only).

Operators are built as explicit Kronecker products and each implicit-midpoint
step is a dense `numpy.linalg.solve`; nothing here mirrors the oracle's sparse
index arithmetic or its fixed-point solver.
"""
import math

import numpy as np


def lowering(L):
    return np.diag(np.sqrt(np.arange(1, L, dtype=float)), 1).astype(complex)


def embed(op, j, q, L):
    """I x ... x op (slot j, qubit 0 leftmost/most significant) x ... x I."""
    out = np.array([[1.0 + 0j]])
    for k in range(q):
        out = np.kron(out, op if k == j else np.eye(L))
    return out


def number_ops(q, L):
    a = lowering(L)
    return [embed(a.conj().T @ a, j, q, L) for j in range(q)]


def drift_matrix(w):
    q, L = w.q, w.L
    n = number_ops(q, L)
    Id = np.eye(L ** q)
    H = np.zeros((L ** q, L ** q), dtype=complex)
    for j in range(q):
        H += w.detuning[j] * n[j] + 0.5 * w.anharmonicity[j] * n[j] @ (n[j] - Id)
    for j in range(q - 1):
        H += w.cross_kerr[j] * n[j] @ n[j + 1]
    return H


def dipole_matrix(w):
    """sum_j J_j (a_{j+1}^+ a_j + a_{j+1} a_j^+) over the chain (eq. sys-ham, nearest neighbours)."""
    q, L = w.q, w.L
    a = lowering(L)
    H = np.zeros((L ** q, L ** q), dtype=complex)
    J = w.dipole_or_zero
    for j in range(q - 1):
        Aj, Ak = embed(a, j, q, L), embed(a, j + 1, q, L)
        H += J[j] * (Ak.conj().T @ Aj + Ak @ Aj.conj().T)
    return H


def static_matrix(w):
    """Time-independent part of H: the diagonal drift plus the dipole coupling."""
    return drift_matrix(w) + dipole_matrix(w)


def control_matrix(w, c):
    """sum_j c_j a_j + conj(c_j) a_j^+ with c_j = 2 pi d_j."""
    q, L = w.q, w.L
    a = lowering(L)
    H = np.zeros((L ** q, L ** q), dtype=complex)
    for j in range(q):
        A = embed(a, j, q, L)
        H += c[j] * A + np.conj(c[j]) * A.conj().T
    return H


_BASIS = None


def bspline_ref(x):
    """Quadratic cardinal B-spline from scipy's B-spline basis element on knots -3/2..3/2."""
    global _BASIS
    if _BASIS is None:
        from scipy.interpolate import BSpline
        _BASIS = BSpline.basis_element([-1.5, -0.5, 0.5, 1.5], extrapolate=False)
    v = _BASIS(x)
    return 0.0 if np.isnan(v) else float(v)


def controls_ref(w, alpha, t):
    """c_j(t) by direct summation over all coefficients."""
    q, nf, d1 = w.q, w.n_carriers, w.n_splines
    dtau = w.T / (d1 - 2)
    c = np.zeros(q, dtype=complex)
    for j in range(q):
        for f in range(nf):
            for s in range(d1):
                b = bspline_ref((t - (s - 0.5) * dtau) / dtau)
                a1 = alpha[((j * nf + f) * 2 + 0) * d1 + s]
                a2 = alpha[((j * nf + f) * 2 + 1) * d1 + s]
                c[j] += 2 * math.pi * (a1 + 1j * a2) * b * np.exp(1j * w.carriers[j, f] * t)
    return c


def essential_rows_ref(q, L):
    rows = []
    for e in range(2 ** q):
        bits = [(e >> (q - 1 - j)) & 1 for j in range(q)]
        rows.append(sum(b * L ** (q - 1 - j) for j, b in enumerate(bits)))
    return np.array(rows)


def embedded_target(w):
    V = np.zeros((w.N, w.E), dtype=complex)
    rows = essential_rows_ref(w.q, w.L)
    Vee = w.target.T  # column-major storage -> matrix
    V[rows, :] = Vee
    return V


def window_starts_ref(w):
    return [(m * w.n_steps) // w.n_windows for m in range(w.n_windows + 1)]


def dense_step(H, dt, U):
    n = H.shape[0]
    A = np.eye(n) + 0.5j * dt * H
    B = np.eye(n) - 0.5j * dt * H
    return np.linalg.solve(A, B @ U)


def dense_objective(w, alpha, W):
    """P by dense stepping: W [M-1, E, N] column storage; returns (P, list of U^m as N x E)."""
    dt = w.T / w.n_steps
    Hd = static_matrix(w)
    starts = window_starts_ref(w)
    V = embedded_target(w)
    Us = []
    for m in range(1, w.n_windows + 1):
        if m == 1:
            U = np.zeros((w.N, w.E), dtype=complex)
            U[essential_rows_ref(w.q, w.L), np.arange(w.E)] = 1.0
        else:
            U = W[m - 2].T.copy()
        for k in range(starts[m - 1], starts[m]):
            t = (k + 0.5) * dt
            U = dense_step(Hd + control_matrix(w, controls_ref(w, alpha, t)), dt, U)
        Us.append(U)
    UM = Us[-1]
    gam = np.vdot(V, UM)
    J = np.sum(np.abs(UM) ** 2) / w.E - abs(gam) ** 2 / w.E ** 2
    pen = sum(np.sum(np.abs(Us[m - 1] - W[m - 1].T) ** 2) for m in range(1, w.n_windows))
    return J + 0.5 * w.mu * pen, Us
