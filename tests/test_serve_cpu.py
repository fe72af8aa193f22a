"""Scheduling logic of the continuous-batching server on the CPU with a simulated device."""
import collections

import pytest

from paper_2407_13950_amd import serve, workloads as WL


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5          # every look at the clock advances it (the server busy-polls)
        return self.t


class FakeBackend(serve.Backend):
    """Device stand-in: a batch finishes `service(items)` seconds after launch."""

    def __init__(self, clock, n_streams=2):
        self.clock = clock
        self.n = n_streams
        self.open_handles = set()
        self.mem = 0
        self.peak = 0
        self.active = collections.Counter()     # run -> batches in flight containing it
        self.log = []

    def footprint(self, w):
        return w.N * w.E * w.n_windows * 16

    def streams(self):
        return self.n

    def open(self, w, initial):
        h = (object(), self.footprint(w))
        self.open_handles.add(h)
        self.mem += h[1]
        self.peak = max(self.peak, self.mem)
        return h

    def close(self, h):
        self.open_handles.remove(h)
        self.mem -= h[1]

    def launch(self, st, items, handles):
        for h in handles:
            assert h in self.open_handles
        for r in items:
            self.active[r.run_id] += 1
            assert self.active[r.run_id] == 1, "a run is in two batches at once"
        work = sum(2e-4 if r.want_grad else 1e-4 for r in items)
        self.log.append((st, [r.rid for r in items]))
        return self.clock.t + 1e-3 + work

    def ready(self, token):
        return self.clock.t >= token

    def collect(self, token, items, handles):
        for r in items:
            self.active[r.run_id] -= 1
            r.result = {"ok": True, "grad": r.want_grad}


def small_runs(n_runs):
    ws = [WL.scaled(WL.c1(), 40, 4), WL.scaled(WL.c2(), 40, 8), WL.scaled(WL.c3(), 40, 16)]
    return {r: ws[r % 3] for r in range(n_runs)}


@pytest.mark.parametrize("budget_runs", [3, 100])
def test_all_requests_complete_in_run_order_within_budget(budget_runs):
    clock = FakeClock()
    be = FakeBackend(clock)
    runs = small_runs(12)
    budget = max(be.footprint(w) for w in runs.values()) * budget_runs
    srv = serve.Server(be, hbm_budget=budget, max_batch=5, clock=clock)
    runs_, reqs, counts = serve.make_trace(400, rate=2000.0, seed=3, n_runs=12)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r])
    summary = srv.run_trace(reqs)
    assert summary["requests"] == 400
    assert srv.peak_used <= budget and be.peak <= budget
    assert srv.used == 0 and not be.open_handles                 # every run released its memory
    assert max(srv.batch_sizes) <= 5
    by_run = collections.defaultdict(list)
    for q in srv.completed:
        by_run[q.run_id].append(q)
        assert q.done >= q.start >= q.arrival
        assert q.result["grad"] == q.want_grad
    for r, lst in by_run.items():
        rids = [q.rid for q in lst]
        assert rids == sorted(rids), "requests of one run completed out of order"


def test_admission_blocks_until_memory_frees():
    clock = FakeClock()
    be = FakeBackend(clock)
    w3 = WL.scaled(WL.c3(), 40, 16)
    runs = {r: w3 for r in range(6)}
    big = be.footprint(w3)
    srv = serve.Server(be, hbm_budget=big, max_batch=8, clock=clock)
    _, reqs, counts = serve.make_trace(60, rate=5000.0, seed=4, n_runs=6)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r])
    assert srv.used <= big and len(be.open_handles) == 1       # only one run fits at a time
    srv.run_trace(reqs)
    assert be.peak <= big
    assert len(srv.completed) == 60


def test_batches_overlap_on_streams():
    clock = FakeClock()
    be = FakeBackend(clock, n_streams=3)
    runs = small_runs(30)
    srv = serve.Server(be, hbm_budget=10 ** 12, max_batch=4, clock=clock)
    _, reqs, counts = serve.make_trace(300, rate=50000.0, seed=5, n_runs=30)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r])
    srv.run_trace(reqs)
    assert {st for st, _ in be.log} == {0, 1, 2}


def test_run_larger_than_budget_is_rejected():
    clock = FakeClock()
    be = FakeBackend(clock)
    w = WL.scaled(WL.c3(), 40, 16)
    srv = serve.Server(be, hbm_budget=be.footprint(w) // 2, clock=clock)
    with pytest.raises(ValueError):
        srv.register_run(0, w, 3)


class ClassedBackend(FakeBackend):
    def duration_class(self, w):
        return w.q


def test_batches_hold_one_duration_class():
    clock = FakeClock()
    be = ClassedBackend(clock, n_streams=2)
    runs = small_runs(15)
    srv = serve.Server(be, hbm_budget=10 ** 12, max_batch=8, clock=clock)
    _, reqs, counts = serve.make_trace(300, rate=20000.0, seed=6, n_runs=15)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r])
    srv.run_trace(reqs)
    by_rid = {q.rid: q for q in srv.completed}
    for st, rids in be.log:
        assert len({runs[by_rid[i].run_id].q for i in rids}) == 1
    assert len(srv.completed) == 300


class FailingBackend(FakeBackend):
    """Evaluations of the runs in `bad` fail (as a fixed-point bound violation would)."""

    def __init__(self, clock, bad, n_streams=2):
        super().__init__(clock, n_streams)
        self.bad = set(bad)

    def collect(self, token, items, handles):
        super().collect(token, items, handles)
        for r in items:
            if r.run_id in self.bad:
                r.error = -4
                r.result = None


def test_failed_requests_do_not_block_others():
    clock = FakeClock()
    be = FailingBackend(clock, bad={2, 7})
    runs = small_runs(12)
    srv = serve.Server(be, hbm_budget=10 ** 12, max_batch=6, clock=clock)
    _, reqs, counts = serve.make_trace(300, rate=20000.0, seed=8, n_runs=12)
    for r, w in runs.items():
        srv.register_run(r, w, counts[r])
    summary = srv.run_trace(reqs)
    assert summary["requests"] == 300
    assert summary["failed"] == counts[2] + counts[7]
    for q in srv.completed:
        if q.run_id in (2, 7):
            assert q.error and q.result is None
        else:
            assert q.error == 0 and q.result["ok"]
    assert srv.used == 0 and not be.open_handles


def test_qoc_backend_accounts_for_resident_buffers():
    """The HIP backend's footprint covers the run's resident inputs and its reused output buffers
    (alpha, W, P, terms, dP/dalpha, dP/dW) beside the context."""
    w = WL.c3().replace(n_windows=16)
    n_w = 16 * 15 * w.N * w.E
    assert serve.QocBackend.resident_bytes(w) == 2 * n_w + 16 * w.d + 8 * (5 + 16)
