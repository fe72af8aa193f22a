"""The autograd.Function (P(alpha, W) with the hand-written adjoint as backward) on one System
shared by several graphs: each graph receives the gradient of its own point."""
import numpy as np
import pytest
import torch

from paper_2407_13950_amd import qoc, workloads as WL
from paper_2407_13950_amd.autograd import penalty_objective

pytestmark = pytest.mark.gpu


def point(w, seed):
    a = torch.tensor(WL.gen_alpha(w, seed), device="cuda", requires_grad=True)
    W = torch.tensor(WL.gen_qr_states(w, seed), device="cuda", requires_grad=True)
    return a, W


def reference(w, a, W, prec):
    s = qoc.System(w, precision=prec)
    s.set_controls(a.detach().cpu().numpy())
    s.set_window_states(W.detach().cpu().numpy())
    out = s.gradient()
    s.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_graphs_on_one_system(prec):
    """P1 and P2 are built on one System before either backward runs: the System's forward
    state is P2's when P1's backward comes, so that backward re-runs P1's forward first."""
    w = WL.scaled(WL.c2(), 300, 4, n_splines=6)
    s = qoc.System(w, precision=prec)
    a1, W1 = point(w, 1)
    a2, W2 = point(w, 2)
    P1 = penalty_objective(a1, W1, s)
    P2 = penalty_objective(a2, W2, s)
    (P1 + 3.0 * P2).backward()
    for (a, W, scale, P) in ((a1, W1, 1.0, P1), (a2, W2, 3.0, P2)):
        Pr, _, ga, gW = reference(w, a, W, prec)
        assert float(P.item()) == Pr
        assert np.array_equal(a.grad.cpu().numpy(), scale * ga)
        assert np.array_equal(W.grad.cpu().numpy(), scale * gW)
    # a probe of another point between forward and backward (as a finite-difference check would do)
    a3, W3 = point(w, 3)
    P3 = penalty_objective(a3, W3, s)
    s.set_controls(a1.detach())
    s.objective()
    P3.backward()
    _, _, ga, gW = reference(w, a3, W3, prec)
    assert np.array_equal(a3.grad.cpu().numpy(), ga) and np.array_equal(W3.grad.cpu().numpy(), gW)
    s.close()


def test_backward_reports_an_unconverged_solve():
    w = WL.scaled(WL.c1(), 40, 2, n_splines=6)
    s = qoc.System(w, precision="fp64")
    a = torch.tensor(WL.gen_alpha(w, 4) * 400.0, device="cuda", requires_grad=True)
    W = torch.tensor(WL.gen_qr_states(w, 4), device="cuda", requires_grad=True)
    P = penalty_objective(a, W, s)
    with pytest.raises(qoc.QocError) as e:
        P.backward()
    assert e.value.code == qoc.QOC_ENOTCONV
    s.close()
