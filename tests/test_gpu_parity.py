"""GPU parity: the HIP path against the CPU FP64 oracle, through the C-ABI.

Tolerances: FP64 path 1e-10, FP32 path 1e-5, both relative; for a branch
gradient the scale is A_b = sum_s w_s |per-site term| (see oracle.compare),
which is |g_b| whenever the sites do not cancel.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload, states_to_masks
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


def gpu_eval(w, precision=B.PG_FP64, t=None):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        return ctx.logL_and_grad(w.t if t is None else t)


def check(w, precision, tol, branches=None, ref="naive"):
    logL, grad = gpu_eval(w, precision)
    if ref == "naive":
        r = O.naive_gradient(*args_of(w), branches=branches)
    else:
        r = O.linear_gradient(*args_of(w))
    rep = O.parity_report(logL, grad, r["logL"], r["grad"], r["abs_grad"], tol, branches=branches)
    print(w.name, precision, rep, flush=True)
    assert rep["ok"], rep
    return logL, grad, r


def test_c1_fp64_all_branches(gpu):
    w = make_workload("C1")
    check(w, B.PG_FP64, TOL64)


@pytest.mark.parametrize("n_tips,n_patterns,n_cats,amb", [
    (2, 1, 1, 0.0),        # a single cherry, one pattern
    (3, 17, 2, 0.1),       # ragged tail: 17 patterns -> 2 tiles of 16
    (37, 53, 3, 0.1),      # several tiles and levels
    (64, 100, 4, 0.02),
])
def test_small_shapes_fp64(gpu, n_tips, n_patterns, n_cats, amb):
    w = small(n_tips=n_tips, n_patterns=n_patterns, n_cats=n_cats, ambiguous=amb, seed=n_tips)
    check(w, B.PG_FP64, TOL64)


def test_partial_ambiguity_masks(gpu):
    w = small(n_tips=20, n_patterns=48, n_cats=2, ambiguous=0.0, seed=5)
    rng = np.random.default_rng(0)
    masks = w.tip_masks().copy()
    pick = rng.random(masks.shape) < 0.2
    masks[pick] = rng.choice(np.array([3, 5, 6, 9, 10, 12, 7, 11, 13, 14], dtype=np.uint64),
                             size=pick.sum())
    w.masks = masks
    check(w, B.PG_FP64, TOL64)


def test_twenty_states_fp64(gpu):
    w = small(n_tips=24, n_patterns=40, n_cats=2, n_states=20, seed=3, ambiguous=0.05)
    check(w, B.PG_FP64, TOL64)


def test_zero_length_branches(gpu):
    w = small(n_tips=16, n_patterns=40, n_cats=2, seed=9, ambiguous=0.1)
    w.t = w.t.copy()
    w.t[[0, 3, 17, 20]] = 0.0
    check(w, B.PG_FP64, TOL64)


def test_c2_fp64_full_size(gpu):
    """N=1000, K=4, S=2000: every branch against the O(N) oracle route, and a
    sample of branches against the naive O(N^2) oracle."""
    w = make_workload("C2")
    logL, grad = gpu_eval(w, B.PG_FP64)
    lin = O.linear_gradient(*args_of(w))
    sample = list(np.random.default_rng(1).choice(len(w.t), size=24, replace=False)) + [0, len(w.t) - 1]
    nv = O.naive_gradient(*args_of(w), branches=sample)
    rep_n = O.parity_report(logL, grad, nv["logL"], nv["grad"], nv["abs_grad"], TOL64, branches=sample)
    rep_l = O.parity_report(logL, grad, lin["logL"], lin["grad"], lin["abs_grad"], TOL64)
    print("C2 fp64 naive-sample", rep_n, "linear-all", rep_l, flush=True)
    assert rep_n["ok"] and rep_l["ok"]


def test_c2_fp32_full_size(gpu):
    w = make_workload("C2")
    logL, grad = gpu_eval(w, B.PG_FP32)
    lin = O.linear_gradient(*args_of(w))
    rep = O.parity_report(logL, grad, lin["logL"], lin["grad"], lin["abs_grad"], TOL32)
    print("C2 fp32", rep, flush=True)
    assert rep["ok"], rep


def test_fp32_small(gpu):
    w = small(n_tips=37, n_patterns=53, n_cats=3, ambiguous=0.1, seed=37)
    check(w, B.PG_FP32, TOL32)


def test_split_calls_match_fused_and_are_deterministic(gpu):
    w = small(n_tips=50, n_patterns=70, n_cats=4, seed=2)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        l1, g1 = ctx.logL_and_grad(w.t)
        l2 = ctx.logL(w.t)
        g2 = ctx.grad()
        l3, g3 = ctx.logL_and_grad(w.t)
    assert l1 == l2 == l3
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)


def test_device_pointer_entry_point(gpu):
    import torch
    w = small(n_tips=30, n_patterns=33, n_cats=2, seed=4)
    stream = torch.cuda.Stream()
    with B.Context(0, B.PG_FP64) as ctx, torch.cuda.stream(stream):
        ctx.set_workload(w)
        ctx.set_stream(stream.cuda_stream)
        l_ref, g_ref = ctx.logL_and_grad(w.t)
        d_t = torch.tensor(w.t, device="cuda", dtype=torch.float64)
        d_l = torch.zeros(1, device="cuda", dtype=torch.float64)
        d_g = torch.zeros(len(w.t), device="cuda", dtype=torch.float64)
        ctx.logL_and_grad_device(d_t.data_ptr(), d_l.data_ptr(), d_g.data_ptr())
        torch.cuda.synchronize()
        assert ctx.status() == B.PG_OK
        assert d_l.item() == l_ref
        assert np.array_equal(d_g.cpu().numpy(), g_ref)


def test_errors(gpu):
    w = small(n_tips=6, n_patterns=10, seed=1)
    with B.Context(0, B.PG_FP64) as ctx:
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL(w.t)
        assert e.value.code == B.PG_E_STATE
        ctx.set_workload(w)
        bad = w.t.copy()
        bad[2] = -1.0
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL_and_grad(bad)
        assert e.value.code == B.PG_E_INVALID
        with pytest.raises(B.PhyloGradError) as e:
            ctx.grad()
        assert e.value.code == B.PG_E_STATE
        parent = w.parent.copy()
        parent[0] = parent[1] = parent[2] = parent[3]
        with pytest.raises(B.PhyloGradError) as e:
            ctx.set_tree(parent)
        assert e.value.code == B.PG_E_TREE
        Q = w.Q.copy()
        Q[0, 0] += 0.1
        with pytest.raises(B.PhyloGradError) as e:
            ctx.set_model(Q, w.pi, w.rates, w.cat_weights)
        assert e.value.code == B.PG_E_MODEL


def test_zero_likelihood(gpu):
    """Two tips in different states joined by zero-length branches: L = 0."""
    parent = np.array([2, 2, -1], dtype=np.int32)
    masks = states_to_masks(np.array([[0, 1], [1, 1]], dtype=np.int16), 4)
    rng = np.random.default_rng(0)
    from synth import random_rate_matrix
    Q = random_rate_matrix(4, rng)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_tree(parent)
        ctx.set_patterns(masks, np.array([1.0, 2.0]), 4)
        ctx.set_model(Q, np.full(4, 0.25), [1.0], [1.0])
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL_and_grad(np.zeros(2))
        assert e.value.code == B.PG_E_ZERO_LIK
        # zero weight on the impossible pattern: finite again
        ctx.set_patterns(masks, np.array([0.0, 2.0]), 4)
        logL, g = ctx.logL_and_grad(np.zeros(2))
        assert math.isfinite(logL)


# Extreme tree shapes: a balanced tree (every tip in a cherry, i.e. an
# internal node whose children are both tips), a caterpillar (one cherry,
# one node per level) and a cherry directly under the root.
_SHAPES = {
    "balanced8": [8, 8, 9, 9, 11, 11, 12, 12, 10, 10, 14, 13, 13, 14, -1],
    "caterpillar6": [6, 6, 7, 8, 9, 10, 7, 8, 9, 10, -1],
    "root_cherry3": [3, 3, 4, 4, -1],
}


@pytest.mark.parametrize("shape", sorted(_SHAPES))
@pytest.mark.parametrize("precision,tol", [(B.PG_FP64, TOL64), (B.PG_FP32, TOL32)])
def test_tree_shapes(gpu, shape, precision, tol):
    parent = np.array(_SHAPES[shape], dtype=np.int32)
    n = (len(parent) + 1) // 2
    w = small(n_tips=n, n_patterns=37, n_cats=2, ambiguous=0.1, seed=n + 1)
    w.parent = parent
    check(w, precision, tol)


def test_tree_shapes_hessian(gpu):
    parent = np.array(_SHAPES["balanced8"], dtype=np.int32)
    w = small(n_tips=8, n_patterns=37, n_cats=2, ambiguous=0.1, seed=3)
    w.parent = parent
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        ctx.logL(w.t)
        grad, hess = ctx.hessian_diag()
    r = O.linear_gradient(*args_of(w))
    assert np.all(np.abs(grad - r["grad"]) <= TOL64 * r["abs_grad"])
    assert np.all(np.abs(hess - r["hess"]) <= TOL64 * r["abs_hess"])
