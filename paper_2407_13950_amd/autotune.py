"""Measured choice of the backward-sweep schedule (qoc_set_schedule).

The adjoint sweep of App. B can spread its work over wavefronts in more than one
way (one wavefront per (window, column group) carrying the state reconstruction
and the adjoint; or, on layouts with one column per wavefront, two wavefronts per
item, one for each, or three, the third taking the per-step inner products).  Which is faster depends on how many items share the GPU:
two or three wavefronts shorten a window's chain of steps, one wavefront spends
fewer instructions per item-step.  The library's default rule uses the item count
of the launch; the functions here measure instead.

* `tune_system`: times the backward phase of one system under each schedule its
  layout offers (the library's own HIP events, mean over `reps` gradient calls
  after warm-up) and keeps the fastest.
* `tune_batch`: a batched evaluation's makespan depends on all of its members,
  so the candidates are timed on the batch itself.  Tunable systems are grouped
  by (qubits, levels, windows, steps, dipole, precision).  The makespan is a
  maximum over the members' chains, so moving one group alone often changes
  nothing; the tuner first tries every schedule for all groups that offer it at
  once against the default rule, keeps the best, and then switches each group in turn to every
  other schedule while the rest stay as they are (one pass of coordinate descent).
  A move is kept when it shortens the batch by more than `min_gain`.

A schedule is a property of the context, used by its single and batched calls
alike, so a tuned batch still returns each member's single-call result bit for
bit.  Both functions leave the chosen schedules set on the systems.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence

import numpy as np


def group_key(system) -> str:
    w = system.w
    hop = bool(getattr(w, "has_dipole", False))
    return f"q{w.q}L{w.L}-M{w.n_windows}-NT{w.n_steps}" + ("-J" if hop else "") + f"-{system.precision}"


def tune_system(system, reps: int = 5, warmup: int = 2) -> Dict:
    """Time the backward phase under each offered schedule; keep the fastest.

    The system must hold controls and window states.  Returns
    {"choice": name, "backward_ms": {name: mean ms}}."""
    times = {}
    for name in system.schedules():
        system.set_schedule(name)
        for _ in range(warmup):
            system.gradient(device=True)
        system.enable_timing(True)
        for _ in range(reps):
            system.gradient(device=True)
        times[name] = system.timings()["backward"]
        system.enable_timing(False)
    best = min(times, key=times.get)
    system.set_schedule(best)
    return {"choice": best, "backward_ms": times}


def _time_batch(batch, systems, reps: int, want_grad) -> float:
    import torch
    batch.run(systems, want_grad)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        batch.run(systems, want_grad)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    return 1e3 * float(np.median(t))


def tune_batch(batch, systems: Sequence, reps: int = 3, want_grad: Optional[Sequence[int]] = None,
               min_gain: float = 0.02) -> Dict:
    """Coordinate descent over the schedule of each group of tunable systems, timed on the batch.

    Returns {"choice": {group: schedule}, "auto_ms": ms, "tuned_ms": ms, "trials": [...]}."""
    groups: Dict[str, List] = {}
    for s in systems:
        if len(s.schedules()) > 1:
            groups.setdefault(group_key(s), []).append(s)
    for s in systems:
        s.set_schedule("auto")
    current = {g: members[0].schedule() for g, members in groups.items()}    # the rule's choice
    for g, members in groups.items():
        for s in members:
            s.set_schedule(current[g])
    best_ms = _time_batch(batch, systems, reps, want_grad)
    auto_ms = best_ms
    trials = [{"assignment": dict(current), "ms": best_ms}]
    offered = sorted({c for members in groups.values() for c in members[0].schedules()})
    for cand in offered:                    # joint moves: every group that offers the schedule at once
        assign = {g: (cand if cand in members[0].schedules() else current[g]) for g, members in groups.items()}
        if assign == current:
            continue
        for g, members in groups.items():
            for s in members:
                s.set_schedule(assign[g])
        ms = _time_batch(batch, systems, reps, want_grad)
        trials.append({"assignment": dict(assign), "ms": ms})
        if ms < best_ms * (1.0 - min_gain):
            best_ms, current = ms, assign
    for g, members in groups.items():
        for s in members:
            s.set_schedule(current[g])
    for g, members in groups.items():                             # then one group at a time
        start = current[g]
        for cand in members[0].schedules():
            if cand == start:
                continue
            for s in members:
                s.set_schedule(cand)
            ms = _time_batch(batch, systems, reps, want_grad)
            trials.append({"assignment": dict(current, **{g: cand}), "ms": ms})
            if ms < best_ms * (1.0 - min_gain):
                best_ms, current[g] = ms, cand
        for s in members:
            s.set_schedule(current[g])
    return {"choice": current, "auto_ms": auto_ms, "tuned_ms": best_ms, "trials": trials}


def apply(systems: Sequence, choice: Dict[str, str]) -> None:
    """Set the schedules of a tuning result on systems of the same groups (others keep theirs)."""
    for s in systems:
        g = group_key(s)
        if g in choice:
            s.set_schedule(choice[g])
