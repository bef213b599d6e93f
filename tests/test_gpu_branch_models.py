"""Non-homogeneous models on the GPU (one rate matrix per branch): logL,
gradient and Hessian diagonal against the CPU FP64 oracle with the same
per-branch matrices, FP64 (1e-10) and FP32 (1e-5) with the A_b rule; one
model for every branch reproduces the homogeneous result bitwise;
clearing returns to the homogeneous model; errors."""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from synth.workloads import branch_models
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu


def _run(w, precision, Qs=None, model=None, hess=False):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        if Qs is not None:
            ctx.set_branch_models(Qs, model)
        logL, g = ctx.logL_and_grad(w.t)
        h = ctx.hessian_diag()[1] if hess else None
    return logL, g, h


@pytest.mark.parametrize("name,kw,n_models", [
    ("C1", dict(n_tips=8), 3),
    ("C1", dict(n_tips=37, n_patterns=53, n_cats=3, ambiguous_frac=0.1), 4),
    ("C2", dict(n_tips=200, n_patterns=300), 5),
    ("C1", dict(n_tips=24, n_patterns=40, n_cats=2, n_states=20, ambiguous_frac=0.05), 3),
])
@pytest.mark.parametrize("precision,tol", [(B.PG_FP64, 1e-10), (B.PG_FP32, 1e-5)])
def test_branch_models_vs_oracle(gpu, name, kw, n_models, precision, tol):
    w = make_workload(name, seed=31, **kw)
    Qs, model = branch_models(w, n_models, seed=5)
    logL, g, h = _run(w, precision, Qs, model, hess=True)
    a = list(args_of(w))
    a[2] = Qs[model]
    r = O.linear_gradient(*a)
    rep = O.parity_report(logL, g, r["logL"], r["grad"], r["abs_grad"], tol)
    print(name, kw, n_models, precision, rep, flush=True)
    assert rep["ok"], rep
    assert np.all(np.abs(h - r["hess"]) <= tol * r["abs_hess"])


@pytest.mark.parametrize("name,kw,n_models", [
    ("C1", dict(n_tips=20, n_patterns=40, n_cats=2, n_states=61, ambiguous_frac=0.05), 3),
    ("C1", dict(n_tips=33, n_patterns=50, n_cats=3), 4),
])
def test_split_branch_models_vs_oracle(gpu, name, kw, n_models):
    """Split-BF16 with per-branch rate matrices (transition matrices by
    scaling and squaring of each branch's own matrix, Q and Q^2 operands per
    matrix): logL, gradient and Hessian diagonal against the oracle at 1e-5
    (A_b rule); clearing returns to the homogeneous result."""
    w = make_workload(name, seed=33, **kw)
    Qs, model = branch_models(w, n_models, seed=6)
    base = _run(w, B.PG_SPLIT_BF16)
    with B.Context(0, B.PG_SPLIT_BF16) as ctx:
        ctx.set_workload(w)
        ctx.set_branch_models(Qs, model)
        logL, g = ctx.logL_and_grad(w.t)
        h = ctx.hessian_diag()[1]
        ctx.set_branch_models(None, None)
        l2, g2 = ctx.logL_and_grad(w.t)
    a = list(args_of(w))
    a[2] = Qs[model]
    r = O.linear_gradient(*a)
    rep = O.parity_report(logL, g, r["logL"], r["grad"], r["abs_grad"], 1e-5)
    print("split", name, kw, n_models, rep, flush=True)
    assert rep["ok"], rep
    assert np.all(np.abs(h - r["hess"]) <= 1e-5 * r["abs_hess"])
    assert l2 == base[0] and np.array_equal(g2, base[1])


def test_single_model_equals_homogeneous_and_clear(gpu):
    w = small(n_tips=30, n_patterns=70, n_cats=2, seed=12)
    base = _run(w, B.PG_FP64)
    one = _run(w, B.PG_FP64, w.Q[None], np.zeros(len(w.t), np.int32))
    assert one[0] == base[0] and np.array_equal(one[1], base[1])
    Qs, model = branch_models(w, 3, seed=1)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        ctx.set_branch_models(Qs, model)
        l1, _ = ctx.logL_and_grad(w.t)
        ctx.set_branch_models(None, None)
        l2, g2 = ctx.logL_and_grad(w.t)
    assert l1 != base[0] and l2 == base[0] and np.array_equal(g2, base[1])


def test_branch_model_errors(gpu):
    w = small(n_tips=6, n_patterns=10)
    Qs, model = branch_models(w, 2, seed=2)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        bad = model.copy()
        bad[0] = 7
        with pytest.raises(B.PhyloGradError) as e:
            ctx.set_branch_models(Qs, bad)
        assert e.value.code == B.PG_E_INVALID
        Qbad = Qs.copy()
        Qbad[1, 0, 1] = -1.0
        with pytest.raises(B.PhyloGradError) as e:
            ctx.set_branch_models(Qbad, model)
        assert e.value.code == B.PG_E_MODEL
