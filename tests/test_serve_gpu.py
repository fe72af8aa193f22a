"""The continuous-batching server on the GPU: every result equals the same evaluation done alone."""
import numpy as np
import pytest
import torch

from paper_2407_13950_amd import qoc, serve, workloads as WL

pytestmark = pytest.mark.gpu


def small_runs(n_runs, seed=0):
    rng = np.random.default_rng(seed)
    base = [WL.c1, WL.c2, WL.c3]
    runs = {}
    for r in range(n_runs):
        w = WL.scaled(base[r % 3](), int(rng.integers(100, 300)), int(rng.choice([1, 2, 4, 8])), n_splines=6)
        runs[r] = w
    return runs


@pytest.mark.parametrize("schedule", ["one_wave", "auto"])
def test_served_results_equal_solo_results(schedule):
    """Every served result equals the single call with the same backward schedule, bit for bit."""
    runs = small_runs(9)
    _, reqs, counts = serve.make_trace(120, rate=3000.0, seed=1, n_runs=9)
    be = serve.QocBackend(precision="fp32", n_streams=2, max_batch=16, max_items=100000, keep_results=True,
                          schedule=schedule)
    srv = serve.Server(be, hbm_budget=8 << 30, max_batch=16)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r], initial=serve.initial_inputs(w, 100 + r))
    summary = srv.run_trace(reqs)
    torch.cuda.synchronize()
    print(summary, "batches", srv.batches, "mean size", np.mean(srv.batch_sizes), flush=True)
    assert summary["requests"] == 120
    assert max(srv.batch_sizes) > 1                      # requests were actually batched
    solo = {}
    for q in srv.completed:
        assert q.error == 0
        w = runs[q.run_id]
        if q.run_id not in solo:
            solo[q.run_id] = qoc.System(w, precision="fp32", backward_schedule=schedule)
        s = solo[q.run_id]
        alpha, W = q.inputs
        s.set_controls(alpha)
        s.set_window_states(W if W is not None else None)
        if q.want_grad:
            P, t, ga, gW = s.gradient()
            assert P == q.result["P"] and np.array_equal(t, q.result["terms"])
            assert np.array_equal(ga, q.result["grad_alpha"])
            if q.result["grad_W"] is not None:
                assert np.array_equal(gW, q.result["grad_W"])
        else:
            P, t = s.objective()
            assert P == q.result["P"] and np.array_equal(t, q.result["terms"])


def test_unconverged_request_fails_alone():
    """One run's controls are far too strong for its time step: the fixed-point bound check
    flags its evaluations (qoc_batch_status), those requests fail with QOC_ENOTCONV, and every
    other request of the same batches completes with the result of its solo evaluation."""
    runs = small_runs(6, seed=3)
    bad_run = 1
    _, reqs, counts = serve.make_trace(60, rate=3000.0, seed=3, n_runs=6)
    be = serve.QocBackend(precision="fp32", n_streams=2, max_batch=8, max_items=100000, keep_results=True)
    srv = serve.Server(be, hbm_budget=8 << 30, max_batch=8)
    for r, w in runs.items():
        a0, W0 = serve.initial_inputs(w, 300 + r)
        if r == bad_run:
            a0 = a0 * 400.0
        srv.register_run(r, w, counts[r], initial=(a0, W0))
    summary = srv.run_trace(reqs)
    assert summary["requests"] == 60 and summary["failed"] == counts[bad_run] > 0
    assert max(srv.batch_sizes) > 1
    mixed = 0
    by_rid = {q.rid: q for q in srv.completed}
    for q in srv.completed:
        if q.run_id == bad_run:
            assert q.error == qoc.QOC_ENOTCONV and q.result is None
            continue
        assert q.error == 0
        s = qoc.System(runs[q.run_id], precision="fp32")
        alpha, W = q.inputs
        s.set_controls(alpha)
        s.set_window_states(W if W is not None else None)
        P, t = s.objective()
        s.close()
        assert P == q.result["P"] and np.array_equal(t, q.result["terms"])
    print(summary, flush=True)


def test_plain_fp64_path_serves_the_same_trace():
    runs = small_runs(4, seed=2)
    _, reqs, counts = serve.make_trace(24, rate=2000.0, seed=2, n_runs=4)
    srv = serve.Server(serve.PlainBackend("fp64"), hbm_budget=8 << 30, max_batch=1)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r], initial=serve.initial_inputs(w, 200 + r))
    summary = srv.run_trace(reqs)
    assert summary["requests"] == 24 and max(srv.batch_sizes) == 1
    for q in srv.completed:
        assert q.error == 0 and np.isfinite(q.result["P"]) and np.all(np.isfinite(q.result["terms"]))
