"""Autograd extension: torch.autograd over branch rates of a random-effects
clock, t_b = r_b tau_b, with the pre-order pass as the backward.

Checked against the oracle gradient times tau (FP64, 1e-10 with the A_b rule
scaled by tau), against central differences of the GPU forward in r
(h = 1e-6; rounding-limited, |diff| <= 1e-3 + 1e-4 |g|), and with
torch.autograd.gradcheck on a tiny tree.
"""
import numpy as np
import pytest

import oracle as O
from synth import make_workload
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu


def _lik(w):
    from paper_1905_12146_amd.autograd import PhyloLikelihood
    return PhyloLikelihood(w)


def test_c5_backward_equals_oracle_times_tau(gpu):
    import torch
    w = make_workload("C5")
    lik = _lik(w)
    tau = torch.tensor(w.tau, device="cuda", dtype=torch.float64)
    log_r = torch.tensor(w.log_r, device="cuda", dtype=torch.float64, requires_grad=True)
    logL = lik(torch.exp(log_r) * tau)
    logL.backward()
    g_logr = log_r.grad.cpu().numpy()          # dlogL/dlog r = r tau dlogL/dt
    r = np.exp(w.log_r)
    lin = O.linear_gradient(*args_of(w))
    assert abs(logL.item() - lin["logL"]) <= 1e-10 * abs(lin["logL"])
    scale = r * w.tau
    rel = np.abs(g_logr - scale * lin["grad"]) / (scale * lin["abs_grad"])
    print("C5 dlogL/dlog r vs oracle x r tau, A-rule max", rel.max(), flush=True)
    assert rel.max() <= 1e-10
    sample = [0, 17, 499, 996]
    nv = O.naive_gradient(*args_of(w), branches=sample)
    rel_n = np.abs(g_logr[sample] - scale[sample] * nv["grad"][sample]) / (scale[sample] * nv["abs_grad"][sample])
    assert rel_n.max() <= 1e-10
    lik.close()


def test_c5_backward_against_central_differences(gpu):
    import torch
    w = make_workload("C5")
    lik = _lik(w)
    tau = torch.tensor(w.tau, device="cuda", dtype=torch.float64)
    r0 = torch.tensor(np.exp(w.log_r), device="cuda", dtype=torch.float64, requires_grad=True)
    logL = lik(r0 * tau)
    logL.backward()
    g = r0.grad.cpu().numpy()
    h = 1e-6
    for b in (3, 250, 700, 997):
        with torch.no_grad():
            rp = r0.detach().clone()
            rm = r0.detach().clone()
            rp[b] += h
            rm[b] -= h
            fd = (lik(rp * tau).item() - lik(rm * tau).item()) / (2 * h)
        print("b", b, "fd", fd, "autograd", g[b], flush=True)
        assert abs(fd - g[b]) <= 1e-3 + 1e-4 * abs(g[b])
    lik.close()


def test_gradcheck_tiny(gpu):
    import torch
    w = small(n_tips=6, n_cats=2, n_patterns=12, seed=5, mean_t=0.2)
    lik = _lik(w)
    tau = torch.tensor(w.t, device="cuda", dtype=torch.float64)
    r = torch.ones(len(w.t), device="cuda", dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: lik(x * tau), (r,), eps=1e-6, atol=1e-5, rtol=1e-4)
    lik.close()


def test_backward_after_a_later_forward(gpu):
    import torch
    w = small(n_tips=20, n_cats=4, n_patterns=50, seed=9)
    lik = _lik(w)
    t1 = torch.tensor(w.t, device="cuda", dtype=torch.float64, requires_grad=True)
    t2 = torch.tensor(w.t * 1.5, device="cuda", dtype=torch.float64, requires_grad=True)
    l1 = lik(t1)
    l2 = lik(t2)
    l1.backward()
    l2.backward()
    ref1 = O.linear_gradient(*args_of(w))
    w2 = small(n_tips=20, n_cats=4, n_patterns=50, seed=9)
    w2.t = w.t * 1.5
    ref2 = O.linear_gradient(*args_of(w2))
    for t, ref in ((t1, ref1), (t2, ref2)):
        rel = np.abs(t.grad.cpu().numpy() - ref["grad"]) / ref["abs_grad"]
        assert rel.max() <= 1e-10
    lik.close()
