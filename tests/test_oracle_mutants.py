"""Planted mistakes in the oracle (on the CPU) must each break a pin.

Each mutant is a one-token slip of the kind the pins are meant to catch (a
dropped factor, a wrong sign, index or operand).  The oracle source is copied,
the slip applied to the copy, the copy compiled with gcc, and the pin suite
run against it in a subprocess; the pins must fail for every mutant.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qoc_oracle.c")

MUTANTS = {
    "anharmonicity factor": ("0.5 * p->anharm[j] * l[j] * (l[j] - 1)", "1.0 * p->anharm[j] * l[j] * (l[j] - 1)"),
    "cross-Kerr index": ("l[j] * l[j + 1];", "l[j] * l[j];"),
    "carrier sign": ("cexp(I * p->carrier[j * p->nf + f] * t)", "cexp(-I * p->carrier[j * p->nf + f] * t)"),
    "imaginary coefficient part": ("I * alpha[alpha_index(p, j, f, 1, s)]", "I * alpha[alpha_index(p, j, f, 0, s)]"),
    "spline centre": ("(s - 0.5) * dtau", "(s - 0.0) * dtau"),
    "ladder factor": ("c[j] * sqrt((double)(l + 1)) * x[r + s->stride[j]]", "c[j] * sqrt((double)l) * x[r + s->stride[j]]"),
    "raising conjugate": ("conj(c[j]) * sqrt((double)l) * x[r - s->stride[j]]", "c[j] * sqrt((double)l) * x[r - s->stride[j]]"),
    "step midpoint": ("controls(s->p, alpha, (k + 0.5) * s->dt, c);", "controls(s->p, alpha, k * s->dt, c);"),
    "solve sign": ("(rhs[r] - sgn * I * hdt * work[r])", "(rhs[r] + sgn * I * hdt * work[r])"),
    "penalty weight": ("pen *= 0.5 * p->mu;", "pen *= p->mu;"),
    "infidelity normalisation": ("/ (E * E);\n    double pen", "/ E;\n    double pen"),
    "terminal weight": ("lam[r] = 0.5 * p->mu * (w_entry", "lam[r] = p->mu * (w_entry"),
    "terminal conjugate": ("lam[r] = (o->gamma * s->V", "lam[r] = (conj(o->gamma) * s->V"),
    "W-gradient factor 2 (as printed in eq. dP-dW)": ("- 2.0 * lam0[((size_t)m * E + c) * N + r]", "- lam0[((size_t)m * E + c) * N + r]"),
    "adjoint real part": ("creal(ip1);   /* d/d(Re d_j) */", "cimag(ip1);   /* d/d(Re d_j) */"),
    "projection sign": ("+= b * (-sn * X + cs * Y)", "+= b * (sn * X + cs * Y)"),
    "adjoint solve sign": ("imr_solve(s, cc, -1, lam, y, work)", "imr_solve(s, cc, +1, lam, y, work)"),
    "target transpose": ("p->target[2 * (c * s->E + e)] + I * p->target[2 * (c * s->E + e) + 1]",
                         "p->target[2 * (e * s->E + c)] + I * p->target[2 * (e * s->E + c) + 1]"),
    "essential row order": ("((e >> (p->q - 1 - j)) & 1)", "((e >> j) & 1)"),
    "energy gradient conjugate": ("creal(conj(dj) * b * ph)", "creal(dj * b * ph)"),
    "energy imaginary derivative": ("creal(conj(dj) * I * b * ph)", "creal(conj(dj) * b * ph)"),
    "energy normalisation": ("c[j] / (2.0 * M_PI)", "c[j] / M_PI"),
    "dipole weight": ("J * sqrt((double)(la + 1)) * sqrt((double)lb)", "J * sqrt((double)la) * sqrt((double)lb)"),
    "dipole direction": ("x[r + s->stride[j] - s->stride[j + 1]]", "x[r - s->stride[j] + s->stride[j + 1]]"),
    "dipole neighbour": ("lb = s->digit[r * q + j + 1]", "lb = s->digit[r * q + j]"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_breaks_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, QOC_ORACLE_LIB_OVERRIDE=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_optimizer_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_dipole_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant '{name}' survived the pins:\n{r.stdout[-2000:]}"
