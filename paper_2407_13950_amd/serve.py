"""Continuous-batching server for objective(+gradient) requests of many optimisation runs.

A request belongs to an optimisation run (one system: qubits, levels, windows,
steps) whose controls and window states stay on the device between requests;
it carries the step sizes of the synthetic optimiser update applied before its
evaluation and whether the gradient is wanted.  The scheduler

  * admits a run when its device footprint fits the HBM budget (runs that do
    not fit wait; a run releases its memory when its last request completes),
  * serialises the requests of one run (its device buffers are reused),
  * launches a batch on any idle stream as soon as there is admitted work --
    requests that arrive while other batches are on the GPU go into the next
    batch, so batches overlap on the device; a batch takes the oldest ready
    request and then only requests of the same duration class (a batch
    completes as a whole, so a short request must not wait for a long window
    chain) -- and
  * retires a batch when its completion event has passed, stamping each
    request's completion time (latency = completion - arrival).

The device work of a batch is one qoc_batch_run (one launch per phase for all
its systems).  `Backend` isolates the device so the scheduling logic can be
exercised on the CPU with a simulated device.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, Deque, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    """One evaluation of a run.  The run's controls and window states live on the
    device; before the evaluation they take one gradient-descent step with the
    run's previous gradient (alpha -= lr_alpha * grad_alpha, W -= lr_W * grad_W),
    the synthetic stand-in for an optimiser's update."""
    rid: int
    run_id: int
    arrival: float                       # seconds on the server clock
    want_grad: bool = True
    lr_alpha: float = 0.0
    lr_W: float = 0.0
    # filled in by the server
    start: float = math.nan
    done: float = math.nan
    result: Any = None
    inputs: Any = None
    error: int = 0                       # nonzero: the evaluation failed (a QOC_E* code)


@dataclasses.dataclass
class Run:
    run_id: int
    workload: Any
    handle: Any = None
    footprint: int = 0
    pending: Deque[Request] = dataclasses.field(default_factory=collections.deque)
    busy: bool = False
    remaining: int = 0                   # requests still to arrive or complete
    admitted: bool = False
    cls: int = 0                         # duration class of one evaluation


class Backend:
    """Device operations the scheduler needs (the HIP implementation is QocBackend)."""

    def footprint(self, workload) -> int: ...
    def duration_class(self, workload) -> int:
        """Requests of one class are batched together (0 = no distinction)."""
        return 0
    def open(self, workload, initial) -> Any: ...
    def close(self, handle) -> None: ...
    def streams(self) -> int: ...
    def launch(self, stream: int, items: List[Request], handles: List[Any]) -> Any: ...
    def ready(self, token) -> bool: ...
    def collect(self, token, items: List[Request], handles: List[Any]) -> None: ...


class Server:
    def __init__(self, backend: Backend, hbm_budget: int, max_batch: int = 64, clock: Callable[[], float] = None):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.clock = clock or time.perf_counter
        self.runs: Dict[int, Run] = {}
        self.waiting_runs: Deque[int] = collections.deque()      # registered, not yet admitted
        self.ready_runs: Deque[int] = collections.deque()        # admitted, idle, with pending work (FIFO)
        self.used = 0
        self.peak_used = 0
        self.inflight: Dict[int, Any] = {}                        # stream -> (token, items, handles)
        self.completed: List[Request] = []
        self.batches = 0
        self.batch_sizes: List[int] = []

    # --------------------------------------------------------------- runs
    def register_run(self, run_id: int, workload, n_requests: int, initial=None):
        """initial: (alpha, W) the run starts from (device tensors or numpy)."""
        r = Run(run_id, workload, remaining=n_requests)
        r.footprint = self.backend.footprint(workload)
        r.cls = self.backend.duration_class(workload)
        r.initial = initial
        self.runs[run_id] = r
        self.waiting_runs.append(run_id)
        self._admit()

    def _admit(self):
        while self.waiting_runs:
            r = self.runs[self.waiting_runs[0]]
            if self.used + r.footprint > self.budget and self.used > 0:
                return
            if r.footprint > self.budget:
                raise ValueError(f"run {r.run_id} needs {r.footprint} bytes, over the whole budget {self.budget}")
            self.waiting_runs.popleft()
            r.handle = self.backend.open(r.workload, r.initial)
            r.initial = None
            r.admitted = True
            self.used += r.footprint
            self.peak_used = max(self.peak_used, self.used)
            if r.pending and not r.busy:
                self.ready_runs.append(r.run_id)

    def _release(self, r: Run):
        self.backend.close(r.handle)
        r.handle = None
        r.admitted = False
        self.used -= r.footprint
        self._admit()

    # --------------------------------------------------------------- requests
    def submit(self, req: Request):
        r = self.runs[req.run_id]
        r.pending.append(req)
        if r.admitted and not r.busy and len(r.pending) == 1:
            self.ready_runs.append(r.run_id)

    def _retire(self):
        for st in list(self.inflight):
            token, items, handles = self.inflight[st]
            if not self.backend.ready(token):
                continue
            del self.inflight[st]
            self.backend.collect(token, items, handles)
            now = self.clock()
            for req in items:
                req.done = now
                self.completed.append(req)
                r = self.runs[req.run_id]
                r.busy = False
                r.remaining -= 1
                if r.remaining == 0:
                    self._release(r)
                elif r.pending:
                    self.ready_runs.append(r.run_id)

    def _launch(self):
        for st in range(self.backend.streams()):
            if st in self.inflight or not self.ready_runs:
                continue
            items, handles, rest, cls = [], [], collections.deque(), None
            while self.ready_runs:
                rid = self.ready_runs.popleft()
                r = self.runs[rid]
                if r.busy or not r.pending or not r.admitted:
                    continue
                if cls is None:
                    cls = r.cls
                if r.cls != cls or len(items) >= self.max_batch:
                    rest.append(rid)
                    continue
                req = r.pending.popleft()
                r.busy = True
                req.start = self.clock()
                items.append(req)
                handles.append(r.handle)
            self.ready_runs = rest
            if items:
                token = self.backend.launch(st, items, handles)
                self.inflight[st] = (token, items, handles)
                self.batches += 1
                self.batch_sizes.append(len(items))

    def poll(self):
        self._retire()
        self._launch()

    def idle(self) -> bool:
        return not self.inflight and not self.ready_runs

    # --------------------------------------------------------------- open-loop trace
    def run_trace(self, requests: List[Request], t0: Optional[float] = None, progress: Callable = None):
        """Submit each request at t0 + arrival (open loop) and serve until all complete."""
        order = sorted(requests, key=lambda q: q.arrival)
        t0 = self.clock() if t0 is None else t0
        for q in order:
            q.arrival = t0 + q.arrival
        i, n = 0, len(order)
        last_report = self.clock()
        while len(self.completed) < n:
            now = self.clock()
            while i < n and order[i].arrival <= now:
                self.submit(order[i])
                i += 1
            self.poll()
            if progress and now - last_report > 5.0:
                progress(len(self.completed), n)
                last_report = now
        return summarize(self.completed, self.clock() - t0)


def summarize(done: List[Request], wall: float) -> Dict[str, float]:
    lat = np.array([q.done - q.arrival for q in done])
    return {"requests": len(done), "failed": sum(1 for q in done if q.error), "wall_s": wall,
            "throughput_rps": len(done) / wall if wall > 0 else math.nan,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


# ------------------------------------------------------------------- the HIP backend

class QocBackend(Backend):
    """Runs batches through the C ABI: one qoc_batch per stream, one qoc context per run.

    A run holds, besides its context, its resident controls and window states and one
    set of output buffers (P, terms, dP/dalpha, dP/dW) that every request of the run
    reuses; all of it is in footprint().  The gradients stay on the device for the
    run's next update; collect() copies each request's P and terms to the host (and,
    with keep_results, its inputs and gradients), so completed requests hold no device
    memory.  A request whose evaluation exceeded the fixed-point bound fails alone
    (req.error = QOC_ENOTCONV, from qoc_batch_status); its gradient is not applied."""

    def __init__(self, precision: str = "fp32", n_streams: int = 4, max_batch: int = 64, max_items: int = 400000,
                 keep_results: bool = False, schedule: str = "auto",
                 schedules: Optional[Dict[str, str]] = None):
        """schedule: backward schedule of every context (qoc_set_schedule; default: the library's
        rule); schedules: overrides per system group (autotune.group_key)."""
        import torch
        from . import autotune, qoc
        self.torch, self.qoc, self.autotune = torch, qoc, autotune
        self.precision = precision
        self.schedule = schedule
        self.schedules = schedules or {}
        self._streams = [torch.cuda.Stream() for _ in range(n_streams)]   # default priority
        self._batches = [qoc.Batch(max_batch, max_items) for _ in range(n_streams)]
        self.keep_results = keep_results
        self._fp_cache: Dict[Any, int] = {}

    def streams(self) -> int:
        return len(self._streams)

    def duration_class(self, w) -> int:
        """log4 of the longest window's serial work (steps x qubits): one evaluation's critical path."""
        longest = -(-w.n_steps // w.n_windows)
        return int(math.log(max(longest * w.q, 1), 4))

    @staticmethod
    def resident_bytes(w) -> int:
        """Device bytes a run holds beside its context: alpha and W, and the output buffers
        P and terms (one buffer), dP/dalpha and dP/dW."""
        n_w = 16 * (w.n_windows - 1) * w.N * w.E
        return 2 * n_w + 2 * 8 * w.d + 8 * (5 + w.n_windows)

    def footprint(self, w) -> int:
        key = (w.q, w.L, w.n_steps, w.n_windows, w.n_splines, w.n_carriers, w.checkpoint_every)
        if key not in self._fp_cache:
            s = self.qoc.System(w, precision=self.precision)
            self._fp_cache[key] = s.info["device_bytes"]
            s.close()
        return self._fp_cache[key] + self.resident_bytes(w)

    def open(self, w, initial):
        torch = self.torch
        alpha0, W0 = initial
        s = self.qoc.System(w, precision=self.precision, backward_schedule=self.schedule)
        self.autotune.apply([s], self.schedules)
        f8, c16 = torch.float64, torch.complex128
        # out: P and terms of the last evaluation, one buffer (5 + M doubles), and its pinned
        # host copy, written on the batch's stream so that collect() needs no device call
        h = {"system": s, "w": w, "alpha": torch.as_tensor(alpha0, dtype=f8, device="cuda").clone(), "W": None,
             "out": torch.empty(5 + s.M, dtype=f8, device="cuda"),
             "host": torch.empty(5 + s.M, dtype=f8, pin_memory=True),
             "g_alpha": torch.empty(s.d, dtype=f8, device="cuda"), "g_W": None, "g_ok": False,
             "ready": torch.cuda.Event()}
        if w.n_windows > 1:
            h["W"] = torch.as_tensor(W0, dtype=c16, device="cuda").clone().contiguous()
            h["g_W"] = torch.empty((s.M - 1, s.E, s.N), dtype=c16, device="cuda")
        # the copies above ran on the current stream; the run's first request waits for them
        # on the device (launch()), so admission never blocks the host
        h["ready"].record()
        return h

    def close(self, h):
        h["system"].close()
        h.clear()

    def _prepare(self, req, h):
        """Optimiser-style update of the resident inputs, then load them into the context."""
        s = h["system"]
        if h["g_ok"] and req.lr_alpha:
            h["alpha"].sub_(req.lr_alpha * h["g_alpha"])
        if h["W"] is not None and h["g_ok"] and req.lr_W:
            h["W"].sub_(req.lr_W * h["g_W"])
        s.set_controls(h["alpha"])
        s.set_window_states(h["W"] if h["W"] is not None else None)
        if self.keep_results:
            req.inputs = (h["alpha"].cpu().numpy(), None if h["W"] is None else h["W"].cpu().numpy())

    def _read(self, req, h):
        """The evaluation's results into the run's output buffers and P, terms on to the pinned
        host buffer, all on the current stream."""
        h["system"].read_results_into(h["out"][:1], h["out"][1:], h["g_alpha"] if req.want_grad else None,
                                      h["g_W"] if req.want_grad else None)
        h["host"].copy_(h["out"], non_blocking=True)

    def launch(self, st, items, handles):
        torch = self.torch
        stream = self._streams[st]
        with torch.cuda.stream(stream):
            for req, h in zip(items, handles):
                if h["ready"] is not None:          # first request of the run: its inputs' copies
                    stream.wait_event(h["ready"])
                    h["ready"] = None
                self._prepare(req, h)
            self._batches[st].run([h["system"] for h in handles], [r.want_grad for r in items], stream.cuda_stream)
            for req, h in zip(items, handles):
                self._read(req, h)
            ev = torch.cuda.Event()
            ev.record(stream)
        return (ev, st)

    def ready(self, token) -> bool:
        return token[0].query()

    def _status(self, token, items, handles):
        return self._batches[token[1]].status()

    def collect(self, token, items, handles):
        token[0].synchronize()
        status = self._status(token, items, handles)
        ok = [(req, h) for req, h, code in zip(items, handles, status) if code == self.qoc.QOC_OK]
        for req, h, code in zip(items, handles, status):
            if code != self.qoc.QOC_OK:
                req.error = code
                req.result = None
                h["g_ok"] = False       # the run's next update must not use this gradient
        for req, h in ok:                   # copied on the batch's stream before its event
            vals = h["host"].numpy()
            req.result = {"P": float(vals[0]), "terms": vals[1:].copy()}
            if req.want_grad:
                h["g_ok"] = True
                if self.keep_results:
                    req.result["grad_alpha"] = h["g_alpha"].cpu().numpy()
                    req.result["grad_W"] = None if h["g_W"] is None else h["g_W"].cpu().numpy()


class PlainBackend(QocBackend):
    """The plain per-request path: one request at a time, single-context calls, FP64 by default."""

    def __init__(self, precision: str = "fp64", keep_results: bool = False):
        super().__init__(precision=precision, n_streams=1, max_batch=1, max_items=1, keep_results=keep_results)

    def launch(self, st, items, handles):
        torch = self.torch
        assert len(items) == 1
        req, h = items[0], handles[0]
        stream = self._streams[0]
        with torch.cuda.stream(stream):
            if h["ready"] is not None:
                stream.wait_event(h["ready"])
                h["ready"] = None
            self._prepare(req, h)
            s = h["system"]
            if req.want_grad:
                s.gradient_into(h["out"][:1], h["out"][1:], h["g_alpha"], h["g_W"])
            else:
                s.objective_into(h["out"][:1], h["out"][1:])
            h["host"].copy_(h["out"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return (ev, st)

    def _status(self, token, items, handles):
        codes = []
        for h in handles:               # the call's stream is idle: qoc_synchronize only reads the flag
            try:
                h["system"].synchronize()
                codes.append(self.qoc.QOC_OK)
            except self.qoc.QocError as e:
                codes.append(e.code)
        return codes


# ------------------------------------------------------------------- synthetic trace

def make_trace(n_requests: int, rate: float, seed: int, n_runs: int = 100, objective_only: float = 0.1,
               windows=(4, 16, 64, 128), mix=(0.5, 0.375, 0.125), lr_alpha: float = 1e-3, lr_W: float = 1e-2):
    """Open-loop Poisson trace at `rate` requests/s.

    Returns (runs {run_id: workload}, requests in arrival order, requests per run).  Run
    shapes follow the 2/3/4-qubit mix, window counts are uniform over `windows`, each
    request picks a run uniformly (a run's requests keep their order) and 10% are
    objective-only."""
    from . import workloads as WL
    rng = np.random.default_rng([seed, 11])
    makers = [WL.c1, WL.c2, WL.c3]
    runs = {}
    for r in range(n_runs):
        mk = makers[int(rng.choice(3, p=list(mix)))]
        runs[r] = mk().replace(n_windows=int(rng.choice(windows)))
    owners = rng.integers(0, n_runs, size=n_requests)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    counts = collections.Counter()
    reqs = []
    for i in range(n_requests):
        r = int(owners[i])
        counts[r] += 1
        reqs.append(Request(rid=i, run_id=r, arrival=float(arrivals[i]),
                            want_grad=bool(rng.random() >= objective_only), lr_alpha=lr_alpha, lr_W=lr_W))
    return runs, reqs, counts


def initial_inputs(w, seed: int):
    """Seeded starting point of a run: alpha ~ U(-0.01, 0.01) GHz, QR-orthonormal window states."""
    from . import workloads as WL
    return WL.gen_alpha(w, seed), (WL.gen_qr_states(w, seed) if w.n_windows > 1 else None)
