"""Batched evaluation: many systems of different shapes and window counts in one launch per phase.

Each system's result in the batch must equal its solo result bit for bit (same
per-item kernels, same reduction order), and the solo path is the one checked
against the oracle in test_parity_gpu.py / test_fullsize_gpu.py; a reduced mix
is also checked against the oracle directly.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2407_13950_amd import qoc, workloads as WL

pytestmark = pytest.mark.gpu


def make_inputs(w, seed):
    alpha = WL.gen_alpha(w, seed)
    W = WL.gen_qr_states(w, seed) if w.n_windows > 1 else None
    return alpha, W


def load(sysm, alpha, W):
    sysm.set_controls(torch.tensor(alpha, device="cuda"))
    sysm.set_window_states(torch.tensor(W, device="cuda") if W is not None else None)


def solo(w, alpha, W, prec="fp32", grad=True):
    s = qoc.System(w, precision=prec)
    load(s, alpha, W)
    out = s.gradient() if grad else s.objective()
    s.close()
    return out


def small_mix(seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(12):
        base = [WL.c1, WL.c2, WL.c3][i % 3]()
        nT = int(rng.integers(150, 400))
        M = int(rng.choice([1, 2, 4, 7]))
        w = WL.scaled(base, nT, M, n_splines=6)
        out.append((w, *make_inputs(w, 100 + i)))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_solo_bitwise(prec):
    mix = small_mix(1)
    systems = []
    for w, a, W in mix:
        s = qoc.System(w, precision=prec)
        load(s, a, W)
        systems.append(s)
    want = [i % 4 != 3 for i in range(len(mix))]           # every fourth objective-only
    b = qoc.Batch(max_contexts=64, max_items=100000)
    b.run(systems, want_grad=want)
    torch.cuda.synchronize()
    for s, (w, a, W), g in zip(systems, mix, want):
        if g:
            P, t, ga, gW = s.read_results()
            P0, t0, ga0, gW0 = solo(w, a, W, prec)
            assert P == P0 and np.array_equal(t, t0) and np.array_equal(ga, ga0)
            if w.n_windows > 1:
                assert np.array_equal(gW, gW0)
        else:
            P, t, _, _ = s.read_results(grad=False)
            P0, t0 = solo(w, a, W, prec, grad=False)
            assert P == P0 and np.array_equal(t, t0)
            with pytest.raises(qoc.QocError) as e:
                s.read_results()
            assert e.value.code == qoc.QOC_ESTATE
    # a second run of the same batch object (staging reuse) gives the same numbers
    b.run(systems)
    torch.cuda.synchronize()
    w, a, W = mix[0]
    assert systems[0].read_results()[0] == solo(w, a, W, prec)[0]


def test_batch_reduced_mix_matches_oracle():
    mix = small_mix(2)[:6]
    systems = []
    for w, a, W in mix:
        s = qoc.System(w, precision="fp32")
        load(s, a, W)
        systems.append(s)
    qoc.Batch(16, 50000).run(systems)
    torch.cuda.synchronize()
    for s, (w, a, W) in zip(systems, mix):
        P, t, ga, gW = s.read_results()
        P0, t0, ga0, gW0 = O.gradient(w, a, W)
        assert abs(P - P0) <= 1e-5 * abs(P0)
        g = np.concatenate([ga, gW.view(np.float64).ravel()])
        g0 = np.concatenate([ga0, gW0.view(np.float64).ravel()])
        assert np.linalg.norm(g - g0) <= 1e-4 * np.linalg.norm(g0)


MIX_SEED = 7
MIX = WL.batch_mix(MIX_SEED)
MIX_Q4 = [e["index"] for e in MIX if e["workload"].q == 4]

# Per-window penalty tolerance of FP32 propagation against the oracle, derived in
# tests/test_longwindow_gpu.py (random-walk rounding model; 4x its prediction at 25,000 steps).
PEN_RTOL_FP32 = 1e-6


@pytest.fixture(scope="module")
def mix64():
    """The 32/24/8 mix of 2/3/4-qubit systems with window counts in {4,16,64,128}, run as one
    batch (one launch per phase); every member's results are read back to the host."""
    systems, inputs = [], []
    for e in MIX:
        w = e["workload"]
        a, W = make_inputs(w, e["seed"])
        s = qoc.System(w, precision="fp32")
        load(s, a, W)
        systems.append(s)
        inputs.append((w, a, W))
    b = qoc.Batch(max_contexts=64, max_items=400000)
    b.run(systems)
    torch.cuda.synchronize()
    results = []
    for s in systems:
        s.synchronize()                  # raises on a fixed-point bound violation
        results.append(s.read_results())
        s.close()
    b.close()
    return inputs, results


def test_full_mix_64_evaluations_equal_solo(mix64):
    inputs, results = mix64
    for idx in list(range(0, 64, 5)) + [56, 63]:           # a spread of members, all three shapes
        w, a, W = inputs[idx]
        P, t, ga, gW = results[idx]
        P0, t0, ga0, gW0 = solo(w, a, W)
        assert P == P0 and np.array_equal(ga, ga0) and np.array_equal(gW, gW0), (idx, w.name, w.n_windows)


def mix_errors(w, res, ref):
    P, t, ga, gW = res
    P0, t0, ga0, gW0 = ref
    g = np.concatenate([ga, gW.view(np.float64).ravel()])
    g0 = np.concatenate([ga0, gW0.view(np.float64).ravel()])
    e = {"P": abs(P - P0) / abs(P0), "grad": np.linalg.norm(g - g0) / np.linalg.norm(g0),
         "alpha": np.linalg.norm(ga - ga0) / np.linalg.norm(ga0),
         "pen": float(np.max(np.abs(t[5:] - t0[5:]) / np.abs(t0[5:]))) if w.n_windows > 1 else 0.0}
    return e


@pytest.mark.timeout(600)
def test_full_mix_small_members_match_oracle(mix64):
    """Every 2- and 3-qubit member of the 64-eval mix, whole objective, terms and gradient, against the oracle."""
    import time
    inputs, results = mix64
    t0 = time.time()
    worst = {2: {}, 3: {}}
    for (w, a, W), res in zip(inputs, results):
        if w.q == 4:
            continue
        e = mix_errors(w, res, O.gradient(w, a, W))
        assert e["P"] <= 1e-5 and e["grad"] <= 1e-4 and e["alpha"] <= 1e-4, (w.name, w.n_windows, e)
        assert e["pen"] <= PEN_RTOL_FP32, (w.name, w.n_windows, e)
        worst[w.q] = {k: max(worst[w.q].get(k, 0.0), v) for k, v in e.items()}
    print(f"worst errors by qubits: {worst}; oracle {time.time() - t0:.1f} s", flush=True)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("idx", MIX_Q4)
def test_full_mix_4qubit_member_matches_oracle(mix64, idx):
    """Each 4-qubit member of the 64-eval mix (N_T = 100000, M in {4,16,64,128}, windows of up to
    25,000 steps, three-wavefront backward where the rule picks it), whole, against the oracle."""
    import time
    inputs, results = mix64
    w, a, W = inputs[idx]
    t0 = time.time()
    e = mix_errors(w, results[idx], O.gradient(w, a, W))
    print(f"mix member {idx} ({w.name}, M={w.n_windows}): {e}; oracle {time.time() - t0:.1f} s", flush=True)
    assert e["P"] <= 1e-5 and e["grad"] <= 1e-4 and e["alpha"] <= 1e-4, e
    assert e["pen"] <= PEN_RTOL_FP32, e


def test_batch_argument_errors():
    w, a, W = small_mix(3)[0]
    s1 = qoc.System(w, precision="fp32")
    s2 = qoc.System(w, precision="fp64")
    load(s1, a, W)
    load(s2, a, W)
    b = qoc.Batch(2, 10000)
    with pytest.raises(qoc.QocError):
        b.run([s1, s2])                       # mixed precision
    with pytest.raises(qoc.QocError):
        b.run([s1, s1])                       # duplicate
    s3 = qoc.System(w, precision="fp32")
    with pytest.raises(qoc.QocError) as e:
        b.run([s3])                           # no inputs
    assert e.value.code == qoc.QOC_ESTATE
    with pytest.raises(qoc.QocError):
        qoc.Batch(1, 10).run([s1, s1])        # too many contexts


def test_batch_status_fails_only_the_unconverged_context():
    """A context whose controls are far too strong for its time step is flagged by the fixed-point
    bound check; qoc_batch_status reports it alone and the other contexts' results equal their
    solo evaluations bit for bit.  qoc_batch_gradient (the one-call form) reports QOC_ENOTCONV
    for the same set and succeeds without it."""
    mix = small_mix(4)[:4]
    systems = []
    for i, (w, a, W) in enumerate(mix):
        s = qoc.System(w, precision="fp32")
        load(s, a * (400.0 if i == 2 else 1.0), W)
        systems.append(s)
    b = qoc.Batch(8, 100000)
    b.run(systems)
    assert b.status() == [qoc.QOC_OK, qoc.QOC_OK, qoc.QOC_ENOTCONV, qoc.QOC_OK]
    for i, (s, (w, a, W)) in enumerate(zip(systems, mix)):
        if i == 2:
            continue
        P, t, ga, gW = s.read_results()
        P0, t0, ga0, gW0 = solo(w, a, W)
        assert P == P0 and np.array_equal(t, t0) and np.array_equal(ga, ga0)
    # the flag moved into the batch: the context itself no longer reports it
    systems[2].synchronize()
    with pytest.raises(qoc.QocError) as e:
        qoc.batch_gradient(systems)
    assert e.value.code == qoc.QOC_ENOTCONV and "2" in str(e.value)
    good = [s for i, s in enumerate(systems) if i != 2]
    qoc.batch_gradient(good, want_grad=[True, False, True])
    w, a, W = mix[3]
    P, t, ga, gW = good[2].read_results()
    P0, t0, ga0, gW0 = solo(w, a, W)
    assert P == P0 and np.array_equal(ga, ga0)
    P, t, _, _ = good[1].read_results(grad=False)
    w, a, W = mix[1]
    assert P == solo(w, a, W, grad=False)[0]
