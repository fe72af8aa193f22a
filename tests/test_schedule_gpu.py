"""Backward-sweep schedules (qoc_set_schedule) and the measured tuner, on the GPU.

Every schedule computes the discrete adjoint sweep of App. B; they differ only in how the
state reconstruction, the adjoint and the inner products are spread over wavefronts, so each
must match the FP64 oracle to the stated tolerances on its own.  Forcing them also exercises the
one-wavefront sweep of the one-column layout (4 qubits x 4 levels) at small window
counts, where the default rule picks three wavefronts.  A schedule belongs to its
context: batched results equal the single calls under the same schedule bit for bit,
also after the tuner has set them.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2407_13950_amd import autotune, qoc

import test_parity_gpu as PG
import test_dipole_gpu as TD

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-11, 1e-10), "fp32": (1e-5, 1e-4)}


def grad_rel(ga, gW, ga0, gW0):
    return PG.rel(np.concatenate([ga, gW.view(np.float64).ravel()]),
                  np.concatenate([ga0, gW0.view(np.float64).ravel()]))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("dip", [False, True])
@pytest.mark.parametrize("sched", ["one_wave", "two_waves", "three_waves"])
def test_forced_schedules_match_oracle(prec, dip, sched):
    w, alpha, W = TD.dipole_case(4, 4, 240, 6, seed=3) if dip else PG.small_case(4, 4, 240, 6, seed=3)
    P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
    P, t, ga, gW = PG.run_gpu(w, alpha, W, prec, backward_schedule=sched)
    g = grad_rel(ga, gW, ga0, gW0)
    print(f"{w.name} {prec} {sched}: P rel {abs(P - P0) / abs(P0):.2e}  grad rel-L2 {g:.2e}", flush=True)
    tol_P, tol_g = TOL[prec]
    assert abs(P - P0) <= tol_P * abs(P0) and g <= tol_g


SPLIT_SHAPES = [(1, 3, 100, 3), (2, 3, 403, 5), (2, 4, 210, 4), (3, 2, 150, 5), (3, 3, 180, 4), (4, 2, 160, 4),
                (4, 3, 120, 3), (5, 2, 120, 3), (6, 2, 90, 2)]


@pytest.mark.parametrize("q,L,n_steps,M", SPLIT_SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("sched", ["one_wave", "two_waves"])
def test_schedules_on_multi_column_layouts_match_oracle(q, L, n_steps, M, prec, sched):
    """Layouts with several columns per wavefront, with and without the dipole chain: one wavefront
    (state and adjoint in its two halves, inner products on its chain), or two (the solves in one,
    the inner products in a second, one step behind)."""
    cases = [PG.small_case(q, L, n_steps, M, seed=4)]
    if q >= 2:
        cases.append(TD.dipole_case(q, L, n_steps, M, seed=4))
    for w, alpha, W in cases:
        P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
        s = qoc.System(w, precision=prec)
        assert s.info["columns_per_wave"] >= 2 and s.schedules() == ["one_wave", "two_waves"]
        s.close()
        P, t, ga, gW = PG.run_gpu(w, alpha, W, prec, backward_schedule=sched)
        g = grad_rel(ga, gW, ga0, gW0) if M > 1 else PG.rel(ga, ga0)
        print(f"{w.name} {prec} {sched}: P rel {abs(P - P0) / abs(P0):.2e}  grad rel-L2 {g:.2e}", flush=True)
        tol_P, tol_g = TOL[prec]
        assert abs(P - P0) <= tol_P * abs(P0) and g <= tol_g


@pytest.mark.parametrize("q,L,sched", [(4, 4, "one_wave"), (4, 4, "two_waves"), (4, 4, "three_waves"),
                                        (3, 4, "one_wave"), (3, 4, "two_waves"), (3, 4, "three_waves"),
                                        (2, 3, "two_waves"), (2, 2, "two_waves")])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_schedules_with_a_single_window(q, L, sched, prec):
    """M = 1: no window states, the only window's terminal condition is the infidelity's."""
    w, alpha, W = PG.small_case(q, L, 180, 1, seed=6)
    assert W is None
    P0, t0, ga0, _ = O.gradient(w, alpha, W)
    P, t, ga, _ = PG.run_gpu(w, alpha, W, prec, backward_schedule=sched)
    tol_P, tol_g = TOL[prec]
    assert abs(P - P0) <= tol_P * abs(P0) and PG.rel(ga, ga0) <= tol_g


@pytest.mark.parametrize("sched", ["one_wave", "two_waves", "three_waves"])
def test_forced_schedules_with_checkpoints_and_one_step_windows(sched):
    """Checkpoint re-syncs inside windows, and windows of a single step."""
    for w, alpha, W in (PG.small_case(4, 4, 200, 4, ckpt=7), PG.small_case(4, 4, 8, 8)):
        P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
        P, t, ga, gW = PG.run_gpu(w, alpha, W, "fp32", backward_schedule=sched)
        assert abs(P - P0) <= 1e-5 * abs(P0) and grad_rel(ga, gW, ga0, gW0) <= 1e-4


def test_schedule_query_and_errors():
    w, alpha, W = PG.small_case(4, 4, 64, 4)
    s = qoc.System(w, precision="fp32")
    assert s.schedules() == ["one_wave", "two_waves", "three_waves"]
    assert s.schedule() == "three_waves"                 # 4 x 16 items: the rule picks three wavefronts
    s.set_schedule("one_wave")
    assert s.schedule() == "one_wave"
    s.set_schedule("two_waves")
    assert s.schedule() == "two_waves"
    s.set_schedule("auto")
    assert s.schedule() == "three_waves"
    with pytest.raises(ValueError):
        s.set_schedule("four_waves")
    lib = qoc.load_library()
    assert lib.qoc_set_schedule(s.h, 7) == qoc.QOC_EINVAL
    assert lib.qoc_get_schedule(s.h, None) == qoc.QOC_EINVAL
    s.close()
    big = w.replace(n_windows=128, n_steps=1280)             # 128 x 16 items: one wavefront
    s = qoc.System(big, precision="fp32")
    assert s.schedule() == "one_wave"
    s.close()
    for M, want in ((16, "three_waves"), (17, "one_wave")):  # FP64: at most 256 items
        s = qoc.System(w.replace(n_windows=M, n_steps=10 * M), precision="fp64")
        assert s.schedule() == want, (M, s.schedule())
        s.close()
    w3, _, _ = PG.small_case(3, 3, 64, 4)                    # 3 levels: four columns per wavefront
    s = qoc.System(w3, precision="fp32")
    assert s.schedules() == ["one_wave", "two_waves"] and s.schedule() == "two_waves"   # 4 x 4 items
    with pytest.raises(qoc.QocError) as e:
        s.set_schedule("three_waves")
    assert e.value.code == qoc.QOC_EUNSUPPORTED
    assert s.schedule() == "two_waves"
    s.set_schedule("one_wave")
    assert s.schedule() == "one_wave"
    s.close()
    s = qoc.System(w3.replace(n_windows=300, n_steps=600), precision="fp32")     # 300 x 4 items
    assert s.schedule() == "one_wave"
    s.close()


def test_schedule_change_between_calls_of_one_context():
    """The backward-only call after a schedule change uses the new schedule on the kept forward sweep."""
    w, alpha, W = PG.small_case(4, 4, 160, 4)
    s = qoc.System(w, precision="fp32")
    s.set_controls(alpha)
    s.set_window_states(W)
    P1, _, ga1, gW1 = s.gradient()
    s.set_schedule("one_wave")
    s.objective()
    ga2, gW2 = s.backward()
    s.close()
    P0, _, ga0, gW0 = O.gradient(w, alpha, W)
    assert grad_rel(ga1, gW1, ga0, gW0) <= 1e-4 and grad_rel(ga2, gW2, ga0, gW0) <= 1e-4
    ref = PG.run_gpu(w, alpha, W, "fp32", device=False, backward_schedule="one_wave")
    assert np.array_equal(ga2, ref[2]) and np.array_equal(gW2, ref[3])


def _members(seed=0):
    out = []
    for i, (q, L, n, M, sched) in enumerate([(4, 4, 160, 4, "one_wave"), (4, 4, 160, 4, "two_waves"),
                                               (4, 4, 96, 8, "auto"), (3, 4, 150, 5, "auto"),
                                               (2, 3, 200, 3, "auto"), (4, 4, 130, 5, "three_waves"),
                                               (3, 4, 120, 4, "two_waves"), (2, 2, 90, 3, "two_waves"),
                                               (2, 4, 100, 3, "one_wave")]):
        w, alpha, W = PG.small_case(q, L, n, M, seed=seed + i)
        out.append((w, alpha, W, sched))
    return out


def _open(members):
    systems = []
    for w, alpha, W, sched in members:
        s = qoc.System(w, precision="fp32", backward_schedule=sched)
        s.set_controls(torch.tensor(alpha, device="cuda"))
        s.set_window_states(torch.tensor(W, device="cuda"))
        systems.append(s)
    return systems


def _check_equal_to_solo(members, systems):
    for (w, alpha, W, _), s in zip(members, systems):
        Pb, tb, gab, gWb = s.read_results()
        P, t, ga, gW = PG.run_gpu(w, alpha, W, "fp32", backward_schedule=s.schedule())
        assert Pb == P and np.array_equal(tb, t) and np.array_equal(gab, ga) and np.array_equal(gWb, gW)


def test_batch_with_forced_schedules_equals_solo():
    members = _members()
    systems = _open(members)
    assert [s.schedule() for s in systems] == ["one_wave", "two_waves", "three_waves", "three_waves", "two_waves",
                                               "three_waves", "two_waves", "two_waves", "one_wave"]
    b = qoc.Batch(max_contexts=12, max_items=4096)
    b.run(systems)
    torch.cuda.synchronize()
    _check_equal_to_solo(members, systems)
    for s in systems:
        s.close()
    b.close()


def test_tuner_choices_are_valid_and_keep_bit_identity():
    members = _members(seed=10)
    systems = _open(members)
    r = autotune.tune_system(systems[0], reps=2, warmup=1)
    assert r["choice"] in ("one_wave", "two_waves", "three_waves") and systems[0].schedule() == r["choice"]
    assert all(ms > 0 for ms in r["backward_ms"].values()) and len(r["backward_ms"]) == 3
    r3 = autotune.tune_system(systems[4], reps=1, warmup=1)          # a multi-column layout: two schedules
    assert r3["choice"] in ("one_wave", "two_waves") and list(r3["backward_ms"]) == ["one_wave", "two_waves"]
    b = qoc.Batch(max_contexts=12, max_items=4096)
    rb = autotune.tune_batch(b, systems, reps=2)
    keys = {autotune.group_key(s) for s in systems if len(s.schedules()) > 1}
    assert set(rb["choice"]) == keys
    for s in systems:
        g = autotune.group_key(s)
        if g in rb["choice"]:
            assert s.schedule() == rb["choice"][g]
    assert rb["tuned_ms"] <= rb["auto_ms"] and len(rb["trials"]) >= 1 + len(keys)
    b.run(systems)
    torch.cuda.synchronize()
    _check_equal_to_solo(members, systems)
    for s in systems:
        s.close()
    b.close()


@pytest.mark.parametrize("q,L,sched", [(4, 4, "three_waves"), (4, 4, "two_waves"), (3, 4, "three_waves"),
                                        (2, 3, "two_waves"), (3, 3, "two_waves")])
def test_odd_window_lengths_with_two_step_blocks(q, L, sched):
    """Windows of odd length (203 steps over 4 windows: 50, 51, 51, 51) with checkpoints every 7
    steps: the schedules that hand step records between wavefronts work in blocks of two steps,
    so each window's last block is a single step."""
    w, alpha, W = PG.small_case(q, L, 203, 4, seed=9, ckpt=7)
    P0, t0, ga0, gW0 = O.gradient(w, alpha, W)
    for prec in ("fp32", "fp64"):
        P, t, ga, gW = PG.run_gpu(w, alpha, W, prec, backward_schedule=sched)
        tol_P, tol_g = TOL[prec]
        g = grad_rel(ga, gW, ga0, gW0)
        print(f"{w.name} {prec} {sched}: P rel {abs(P - P0) / abs(P0):.2e}  grad rel-L2 {g:.2e}", flush=True)
        assert abs(P - P0) <= tol_P * abs(P0) and g <= tol_g
