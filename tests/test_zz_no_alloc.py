"""The allocation-free batched run (qoc_batch_run_noalloc, tables in the library's static device
array) against qoc_batch_run on the same contexts: equal results bit for bit (same kernels, same
item order), on two calls in a row with the second smaller, and the capacity error."""
import numpy as np
import pytest
import torch

from paper_2407_13950_amd import qoc, workloads as WL

pytestmark = pytest.mark.gpu


def load(systems, inputs):
    for s, (a, W) in zip(systems, inputs):
        s.set_controls(torch.tensor(a, device="cuda"))
        s.set_window_states(torch.tensor(W, device="cuda") if W is not None else None)


def results(systems, want):
    torch.cuda.synchronize()
    out = []
    for s, g in zip(systems, want):
        s.synchronize()
        out.append(s.read_results(grad=g))
    return out


def same(r0, r1):
    for a, b in zip(r0, r1):
        assert a[0] == b[0] and np.array_equal(a[1], b[1])
        for x, y in zip(a[2:], b[2:]):
            assert (x is None and y is None) or np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_batch_run(prec):
    mix = WL.batch_mix(11)
    systems, inputs = [], []
    for e in mix:
        w = e["workload"]
        systems.append(qoc.System(w, precision=prec))
        inputs.append((WL.gen_alpha(w, e["seed"]), WL.gen_qr_states(w, e["seed"]) if w.n_windows > 1 else None))
    load(systems, inputs)
    want = [i % 5 != 4 for i in range(len(systems))]
    b = qoc.Batch(max_contexts=64, max_items=400000)
    b.run(systems, want)
    ref = results(systems, want)
    qoc.batch_run_noalloc(systems, want)
    same(ref, results(systems, want))
    # second call, smaller: a subset of the mix with other gradient choices
    sub = systems[::7]
    want2 = [i % 2 == 0 for i in range(len(sub))]
    b.run(sub, want2)
    ref2 = results(sub, want2)
    qoc.batch_run_noalloc(sub, want2)
    same(ref2, results(sub, want2))
    b.close()
    for s in systems:
        s.close()


def test_noalloc_rejects_tables_over_its_capacity():
    """50 contexts of 4 qubits x 128 windows need about 4.4 MB of tables, over the 4 MiB array; the
    call fails before launching anything (no context has results afterwards)."""
    w = WL.scaled(WL.c3(), 128, 128)            # dt as in the 4-qubit configuration
    a = WL.gen_alpha(w, 1)
    W = torch.tensor(WL.gen_qr_states(w, 1), device="cuda")
    systems = [qoc.System(w, precision="fp32") for _ in range(50)]
    for s in systems:
        s.set_controls(a)
        s.set_window_states(W)
    with pytest.raises(qoc.QocError) as e:
        qoc.batch_run_noalloc(systems)
    assert e.value.code == qoc.QOC_EINVAL and "static capacity" in str(e.value)
    with pytest.raises(qoc.QocError) as e:
        systems[0].read_results()
    assert e.value.code == qoc.QOC_ESTATE
    qoc.batch_run_noalloc(systems[:20])            # well within the capacity
    torch.cuda.synchronize()
    P, _, _, _ = systems[3].read_results()
    solo = qoc.System(w, precision="fp32")
    solo.set_controls(a)
    solo.set_window_states(W)
    assert P == solo.gradient()[0]
    solo.close()
    for s in systems:
        s.close()
