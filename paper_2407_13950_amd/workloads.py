"""Seeded synthetic workloads shaped like the paper's 2/3/4-qubit QFT experiments.

This module only produces inputs: system parameters taken from the paper's
system-parameter table (transition frequencies and carrier frequencies of the
QFT-4/8/16 test cases, Sec. 5), the QFT target gate (Sec. 5), and seeded random
numbers (control coefficients, window-state noise, QR-orthonormal window
states, finite-difference directions).  It holds none of the method's
arithmetic: no Hamiltonian, no time stepping, no objective.  Both the HIP
library and the CPU oracle consume what it returns.

Units: frequencies are angular, in rad/ns (GHz * 2*pi); control coefficients
alpha are in GHz (the Hamiltonian multiplies them by 2*pi); times in ns.

Layouts (shared with the C ABI):
  * alpha: float64 [d], index ((j*n_carriers + f)*2 + part)*n_splines + s,
    part 0 = real envelope coefficient alpha^(1), part 1 = imaginary alpha^(2).
  * window states W^1..W^{M-1}: complex128 [M-1, E, N] -- for each window a
    column-major N x E matrix (column c of W^m is W[m-1, c, :]).
  * target: complex128 [E, E] column-major (V[:, k] is target[k, :]).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi

# Transition frequencies omega_j/2pi [GHz] and carrier frequencies Omega_j/2pi [MHz]
# of the paper's QFT test cases (Sec. 5, system-parameter table).  The carrier
# lists are padded to the same count per qubit: each qubit's list is extended
# with the missing frequency of the same test case that has the smallest |Omega|.
PAPER_TRANSITION_GHZ = {
    2: [5.18, 5.12],
    3: [5.18, 5.12, 5.06],
    4: [5.18, 5.12, 5.06, 5.0],
}
PAPER_CARRIERS_MHZ = {
    2: [[-30.41, 30.41], [-30.41, 30.41]],
    3: [[0.0, -60.4], [60.4, 0.0, -60.4], [60.4, 0.0]],
    4: [[-30.0, -90.41], [30.0, -30.0, -90.41], [90.41, 30.0, -30.0], [90.41, -30.0]],
}
ANHARMONICITY_GHZ = -0.2      # per qubit
CROSS_KERR_GHZ = 0.005        # nearest neighbours of the linear chain
# Dipole-dipole coupling J_{j,j+1}/2pi [MHz] of the linear chain and the gate durations [ns]
# and step counts of the QFT-4/8/16 test cases (Sec. 5, system-parameter and test-case tables).
PAPER_DIPOLE_MHZ = 5.0
PAPER_DURATION_NS = {2: 190.0, 3: 500.0, 4: 900.0}
PAPER_STEPS = {2: 2252, 3: 19806, 4: 106072}
PAPER_KNOT_SPACING_NS = 3.0


def padded_carriers_mhz(q: int) -> List[List[float]]:
    """Carrier lists of equal length per qubit (missing ones appended, smallest |Omega| first)."""
    lists = [list(x) for x in PAPER_CARRIERS_MHZ[q]]
    n = max(len(x) for x in lists)
    pool = sorted({f for x in lists for f in x}, key=lambda f: (abs(f), f))
    for x in lists:
        for f in pool:
            if len(x) >= n:
                break
            if f not in x:
                x.append(f)
    return lists


def qft_target(E: int) -> np.ndarray:
    """QFT gate V_jk = kappa^{jk}/sqrt(E), kappa = exp(2*pi*i/E) (Sec. 5); returned column-major."""
    j = np.arange(E)
    V = np.exp(2j * np.pi * np.outer(j, j) / E) / math.sqrt(E)
    return np.ascontiguousarray(V.T)


@dataclasses.dataclass
class Workload:
    name: str
    q: int
    L: int
    T: float
    n_steps: int
    n_windows: int
    n_splines: int
    mu: float
    detuning: np.ndarray          # [q] rad/ns
    anharmonicity: np.ndarray     # [q] rad/ns
    cross_kerr: np.ndarray        # [q-1] rad/ns
    carriers: np.ndarray          # [q, nf] rad/ns
    target: np.ndarray            # [E, E] complex, column-major
    window_states: str = "rollout_noise"   # or "qr"
    noise_std: float = 1e-3
    checkpoint_every: int = 0
    dipole: Optional[np.ndarray] = None    # [q-1] rad/ns: J_{j,j+1} of the chain (None: no coupling)

    @property
    def dipole_or_zero(self) -> np.ndarray:
        return np.zeros(max(self.q - 1, 0)) if self.dipole is None else np.asarray(self.dipole, dtype=float)

    @property
    def has_dipole(self) -> bool:
        return self.dipole is not None and bool(np.any(np.asarray(self.dipole) != 0.0))

    @property
    def N(self) -> int:
        return self.L ** self.q

    @property
    def E(self) -> int:
        return 2 ** self.q

    @property
    def n_carriers(self) -> int:
        return int(self.carriers.shape[1])

    @property
    def d(self) -> int:
        return 2 * self.n_splines * self.q * self.n_carriers

    @property
    def n_w(self) -> int:
        """Number of complex window-state entries (M-1)*N*E."""
        return (self.n_windows - 1) * self.N * self.E

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def make_system(name: str, q: int, L: int, T: float, n_steps: int, n_windows: int,
                n_splines: int, mu: Optional[float] = None, window_states: str = "rollout_noise",
                checkpoint_every: int = 0, dipole_mhz: float = 0.0,
                cross_kerr_ghz: float = CROSS_KERR_GHZ) -> Workload:
    omega = np.array(PAPER_TRANSITION_GHZ[q])
    rot = omega.mean()
    carriers = np.array(padded_carriers_mhz(q)) * 1e-3 * TWO_PI
    E = 2 ** q
    return Workload(
        name=name, q=q, L=L, T=float(T), n_steps=int(n_steps), n_windows=int(n_windows),
        n_splines=int(n_splines), mu=float(2.0 / E if mu is None else mu),
        detuning=TWO_PI * (omega - rot),
        anharmonicity=np.full(q, TWO_PI * ANHARMONICITY_GHZ),
        cross_kerr=np.full(max(q - 1, 0), TWO_PI * cross_kerr_ghz),
        carriers=carriers, target=qft_target(E), window_states=window_states,
        checkpoint_every=checkpoint_every,
        dipole=np.full(max(q - 1, 0), TWO_PI * dipole_mhz * 1e-3) if dipole_mhz else None)


def c1() -> Workload:
    """2 qubits x 3 levels, T=200 ns, 4000 steps, 4 windows, 20 splines/carrier (FP64 plain case)."""
    return make_system("C1-q2L3", 2, 3, 200.0, 4000, 4, 20)


def c2() -> Workload:
    """3 qubits x 4 levels, T=400 ns, 20000 steps, 32 windows, 40 splines/carrier, QR window states."""
    return make_system("C2-q3L4", 3, 4, 400.0, 20000, 32, 40, window_states="qr")


def c3() -> Workload:
    """4 qubits x 4 levels, T=800 ns, 100000 steps, 128 windows, 60 splines/carrier, checkpoint 1000."""
    return make_system("C3-q4L4", 4, 4, 800.0, 100000, 128, 60, checkpoint_every=1000)


CONFIGS = {"c1": c1, "c2": c2, "c3": c3}


def paper_qft(q: int, n_windows: int, n_steps: Optional[int] = None, L: int = 2) -> Workload:
    """The paper's QFT-4/8/16 system (Sec. 5): q qubits of L levels (n = 2^q without guard levels
    at L = 2) in a chain with dipole coupling J = 5 MHz and no cross-Kerr term, the table's
    transition and carrier frequencies, its gate duration and step count, and B-splines with a
    knot spacing of 3 ns (d1 = ceil(T/3) + 2)."""
    T = PAPER_DURATION_NS[q]
    d1 = int(math.ceil(T / PAPER_KNOT_SPACING_NS - 1e-9)) + 2
    return make_system(f"QFT-{2 ** q}", q, L, T, PAPER_STEPS[q] if n_steps is None else n_steps, n_windows, d1,
                       dipole_mhz=PAPER_DIPOLE_MHZ, cross_kerr_ghz=0.0)


def scaled(w: Workload, n_steps: int, n_windows: Optional[int] = None, n_splines: Optional[int] = None,
           T: Optional[float] = None) -> Workload:
    """Same system with fewer steps/windows (small parity cases); T scales with n_steps unless given."""
    T_new = w.T * n_steps / w.n_steps if T is None else T
    return w.replace(n_steps=int(n_steps), T=float(T_new),
                     n_windows=int(n_windows if n_windows is not None else w.n_windows),
                     n_splines=int(n_splines if n_splines is not None else w.n_splines),
                     name=f"{w.name}-small")


# ----------------------------------------------------------------------------- random inputs

def gen_alpha(w: Workload, seed: int, amp: float = 0.01) -> np.ndarray:
    """Control coefficients drawn U(-amp, amp) GHz."""
    rng = np.random.default_rng([seed, 1])
    return rng.uniform(-amp, amp, size=w.d)


def gen_noise(w: Workload, seed: int, std: Optional[float] = None) -> np.ndarray:
    """Complex noise for W^1..W^{M-1}: real and imaginary parts i.i.d. N(0, std^2)."""
    rng = np.random.default_rng([seed, 2])
    s = w.noise_std if std is None else std
    shape = (w.n_windows - 1, w.E, w.N)
    return s * rng.standard_normal(shape) + 1j * s * rng.standard_normal(shape)


def gen_qr_states(w: Workload, seed: int) -> np.ndarray:
    """Window states with orthonormal columns: reduced QR of complex N(0,1) N x E matrices."""
    rng = np.random.default_rng([seed, 3])
    out = np.empty((w.n_windows - 1, w.E, w.N), dtype=np.complex128)
    for m in range(w.n_windows - 1):
        A = rng.standard_normal((w.N, w.E)) + 1j * rng.standard_normal((w.N, w.E))
        Qm, _ = np.linalg.qr(A)
        out[m] = Qm.T
    return out


def gen_random_states(w: Workload, seed: int, scale: float = 1.0) -> np.ndarray:
    """Unstructured complex Gaussian window states (for invariants that hold for any W)."""
    rng = np.random.default_rng([seed, 4])
    shape = (w.n_windows - 1, w.E, w.N)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2 * w.N)


def gen_directions(w: Workload, seed: int, count: int) -> List[Dict[str, np.ndarray]]:
    """Unit-norm random directions over (alpha, Re W, Im W) for central finite differences."""
    rng = np.random.default_rng([seed, 5])
    out = []
    for _ in range(count):
        va = rng.standard_normal(w.d)
        vw = rng.standard_normal((w.n_windows - 1, w.E, w.N)) + 1j * rng.standard_normal(
            (w.n_windows - 1, w.E, w.N))
        nrm = math.sqrt(float(np.sum(va ** 2) + np.sum(np.abs(vw) ** 2)))
        out.append({"alpha": va / nrm, "W": vw / nrm})
    return out


def batch_mix(seed: int, n_c1: int = 32, n_c2: int = 24, n_c3: int = 8,
              windows=(4, 16, 64, 128)) -> List[Dict]:
    """The batched mix: per-eval shape, window count drawn uniformly from `windows`, and seeds."""
    rng = np.random.default_rng([seed, 6])
    shapes = [c1] * n_c1 + [c2] * n_c2 + [c3] * n_c3
    out = []
    for i, mk in enumerate(shapes):
        M = int(rng.choice(windows))
        out.append({"workload": mk().replace(n_windows=M), "seed": int(rng.integers(1 << 31)), "index": i})
    return out
