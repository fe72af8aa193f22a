"""Host logic of the schedule tuner (autotune.tune_batch), on the CPU with stand-in systems and a
stand-in batch timer: the joint moves, the per-group moves, the min_gain threshold, and that the
chosen schedules are left set on the systems."""
import types

import pytest

from paper_2407_13950_amd import autotune


class FakeSystem:
    """A system of one group with the schedules its layout offers; `rule` is what "auto" resolves to."""

    def __init__(self, q, M, offers, rule):
        self.w = types.SimpleNamespace(q=q, L=4, n_windows=M, n_steps=1000, has_dipole=False)
        self.precision = "fp32"
        self._offers = list(offers)
        self._rule = rule
        self._sched = "auto"

    def schedules(self):
        return list(self._offers)

    def set_schedule(self, name):
        assert name == "auto" or name in self._offers, name
        self._sched = name

    def schedule(self):
        return self._rule if self._sched == "auto" else self._sched


def run_tuner(monkeypatch, systems, cost, min_gain=0.02):
    """cost(assignment by group) -> ms; the batch timer reads the systems' schedules."""
    calls = []

    def fake_time(batch, syss, reps, want_grad):
        a = {autotune.group_key(s): s.schedule() for s in syss if len(s.schedules()) > 1}
        calls.append(a)
        return cost(a)

    monkeypatch.setattr(autotune, "_time_batch", fake_time)
    return autotune.tune_batch(None, systems, reps=1, min_gain=min_gain), calls


def makespan(a, table):
    """A batch takes as long as its slowest group (each group's time depends on its own schedule)."""
    return max(table[g][s] for g, s in a.items())


def test_joint_move_finds_what_single_moves_cannot(monkeypatch):
    long_ = [FakeSystem(4, 4, ["one_wave", "two_waves", "three_waves"], "two_waves") for _ in range(2)]
    mid = [FakeSystem(4, 16, ["one_wave", "two_waves", "three_waves"], "two_waves")]
    short = [FakeSystem(2, 16, ["one_wave", "two_waves"], "two_waves")]
    systems = long_ + mid + short
    g_long, g_mid, g_short = (autotune.group_key(x[0]) for x in (long_, mid, short))
    table = {g_long: {"one_wave": 90, "two_waves": 80, "three_waves": 60},
             g_mid: {"one_wave": 85, "two_waves": 80, "three_waves": 62},
             g_short: {"one_wave": 10, "two_waves": 12}}
    r, calls = run_tuner(monkeypatch, systems, lambda a: makespan(a, table))
    assert r["auto_ms"] == 80
    assert r["choice"][g_long] == "three_waves" and r["choice"][g_mid] == "three_waves"
    assert r["tuned_ms"] == 62
    # the choice is left set on every member of each group
    for s in systems:
        assert s.schedule() == r["choice"][autotune.group_key(s)]
    # a schedule no group of a multi-column layout offers is never set on it
    assert all(a[g_short] in ("one_wave", "two_waves") for a in calls)


def test_single_group_move_and_min_gain(monkeypatch):
    a = [FakeSystem(4, 4, ["one_wave", "two_waves", "three_waves"], "three_waves")]
    b = [FakeSystem(3, 32, ["one_wave", "two_waves"], "two_waves")]
    ga, gb = autotune.group_key(a[0]), autotune.group_key(b[0])

    def cost(asg):                                    # additive: each group's move pays off on its own
        return {"one_wave": 30, "two_waves": 25, "three_waves": 20}[asg[ga]] + {"one_wave": 9.9, "two_waves": 10}[asg[gb]]

    r, _ = run_tuner(monkeypatch, a + b, cost)
    # group b's one-wave move gains 0.1 ms of 30 (< 2%): not kept
    assert r["choice"] == {ga: "three_waves", gb: "two_waves"} and r["tuned_ms"] == r["auto_ms"] == 30
    r, _ = run_tuner(monkeypatch, a + b, cost, min_gain=0.0)
    assert r["choice"] == {ga: "three_waves", gb: "one_wave"} and r["tuned_ms"] == pytest.approx(29.9)


def test_no_tunable_groups(monkeypatch):
    systems = [FakeSystem(3, 4, ["one_wave"], "one_wave")]
    r, calls = run_tuner(monkeypatch, systems, lambda a: 5.0)
    assert r["choice"] == {} and r["tuned_ms"] == r["auto_ms"] == 5.0 and len(r["trials"]) == 1
