"""GPU Hessian diagonal (Section 2.7, Eq. Hessian) against the oracle.

Tolerance as for the gradient: |h - h*| <= tol * sum_s w_s (|d2L_s/L_s| +
(dL_s/L_s)^2) per branch (the cancellation-free magnitude of the site sum).
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu


def gpu_hess(w, precision=B.PG_FP64):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        logL, grad = ctx.logL_and_grad(w.t)
        g2, h = ctx.hessian_diag()
    return logL, grad, g2, h


def check(h, ref, absh, tol):
    rel = np.abs(h - ref) / np.maximum(absh, np.finfo(float).tiny)
    print("hess rel (A rule) max", rel.max(), flush=True)
    assert (rel <= tol).all(), rel.max()


@pytest.mark.parametrize("n_tips,n_cats,n_states", [(6, 1, 4), (17, 3, 4), (40, 4, 4), (12, 2, 20)])
def test_hessian_small_fp64(gpu, n_tips, n_cats, n_states):
    w = small(n_tips=n_tips, n_cats=n_cats, n_states=n_states, n_patterns=37, seed=n_tips + n_cats,
              ambiguous=0.05, mean_t=0.15)
    logL, grad, g2, h = gpu_hess(w)
    nh = O.naive_hessian_diag(*args_of(w))
    check(h, nh["hess"], nh["abs_hess"], 1e-10)
    assert np.array_equal(grad, g2)


def test_hessian_c2_fp64(gpu):
    w = make_workload("C2")
    logL, grad, g2, h = gpu_hess(w)
    lin = O.linear_gradient(*args_of(w))
    check(h, lin["hess"], lin["abs_hess"], 1e-10)
    sample = [0, 5, 999, 1500, len(w.t) - 1]
    nh = O.naive_hessian_diag(*args_of(w), branches=sample)
    check(h[sample], nh["hess"][sample], nh["abs_hess"][sample], 1e-10)


def test_hessian_c2_fp32(gpu):
    w = make_workload("C2")
    logL, grad, g2, h = gpu_hess(w, B.PG_FP32)
    lin = O.linear_gradient(*args_of(w))
    check(h, lin["hess"], lin["abs_hess"], 1e-5)


def test_hessian_needs_partials(gpu):
    w = small(n_tips=5)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        with pytest.raises(B.PhyloGradError) as e:
            ctx.hessian_diag()
        assert e.value.code == B.PG_E_STATE
